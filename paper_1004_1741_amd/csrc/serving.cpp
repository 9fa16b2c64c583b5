// serving.cpp -- job service entry points (implementation pending).
#include "../../include/stencil.h"
#include "internal.h"
extern "C" {
int smooth_init(const smooth_config *, smooth_ctx **) { stk::set_error("service not built"); return ST_EBUSY; }
int smooth_submit(smooth_ctx *, const smooth_job *, uint64_t *) { return ST_EBUSY; }
int smooth_poll(smooth_ctx *, uint64_t, int32_t *, smooth_stats *) { return ST_EBUSY; }
int smooth_wait_all(smooth_ctx *, int64_t) { return ST_EBUSY; }
int smooth_service_info(smooth_ctx *, smooth_service_stats *) { return ST_EBUSY; }
int smooth_shutdown(smooth_ctx *) { return ST_EBUSY; }
}
