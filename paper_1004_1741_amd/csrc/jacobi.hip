// jacobi.hip -- dispatch of the fused Jacobi pass over the level count TB.
// The kernels and launchers are in jacobi_impl.h; each TB is compiled in
// jacobi_t<TB>.hip.
#include "internal.h"

namespace stk {

extern template struct JacobiLevels<1>;
extern template struct JacobiLevels<2>;
extern template struct JacobiLevels<3>;
extern template struct JacobiLevels<4>;
extern template struct JacobiLevels<5>;
extern template struct JacobiLevels<6>;
extern template struct JacobiLevels<7>;
extern template struct JacobiLevels<8>;

JacTileCfg jacobi_tile_cfg(bool fp32, int tb, bool has_f) {
    switch (tb) {
        case 1: return JacobiLevels<1>::cfg(fp32, has_f);
        case 2: return JacobiLevels<2>::cfg(fp32, has_f);
        case 3: return JacobiLevels<3>::cfg(fp32, has_f);
        case 4: return JacobiLevels<4>::cfg(fp32, has_f);
        case 5: return JacobiLevels<5>::cfg(fp32, has_f);
        case 6: return JacobiLevels<6>::cfg(fp32, has_f);
        case 7: return JacobiLevels<7>::cfg(fp32, has_f);
        default: return JacobiLevels<8>::cfg(fp32, has_f);
    }
}

void jacobi_tile_count(bool fp32, int tb, bool has_f, const Geom &g, int *tiles, int *interior) {
    switch (tb) {
        case 1: return JacobiLevels<1>::tiles(fp32, has_f, g, tiles, interior);
        case 2: return JacobiLevels<2>::tiles(fp32, has_f, g, tiles, interior);
        case 3: return JacobiLevels<3>::tiles(fp32, has_f, g, tiles, interior);
        case 4: return JacobiLevels<4>::tiles(fp32, has_f, g, tiles, interior);
        case 5: return JacobiLevels<5>::tiles(fp32, has_f, g, tiles, interior);
        case 6: return JacobiLevels<6>::tiles(fp32, has_f, g, tiles, interior);
        case 7: return JacobiLevels<7>::tiles(fp32, has_f, g, tiles, interior);
        default: return JacobiLevels<8>::tiles(fp32, has_f, g, tiles, interior);
    }
}

hipError_t launch_jacobi_pass(bool fp32, int tb, const Geom &g, const void *src, void *dst,
                              const void *f, double a, double b, double gw, int zc,
                              hipStream_t s) {
    switch (tb) {
        case 1: return JacobiLevels<1>::pass(fp32, g, src, dst, f, a, b, gw, zc, s);
        case 2: return JacobiLevels<2>::pass(fp32, g, src, dst, f, a, b, gw, zc, s);
        case 3: return JacobiLevels<3>::pass(fp32, g, src, dst, f, a, b, gw, zc, s);
        case 4: return JacobiLevels<4>::pass(fp32, g, src, dst, f, a, b, gw, zc, s);
        case 5: return JacobiLevels<5>::pass(fp32, g, src, dst, f, a, b, gw, zc, s);
        case 6: return JacobiLevels<6>::pass(fp32, g, src, dst, f, a, b, gw, zc, s);
        case 7: return JacobiLevels<7>::pass(fp32, g, src, dst, f, a, b, gw, zc, s);
        case 8: return JacobiLevels<8>::pass(fp32, g, src, dst, f, a, b, gw, zc, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_rbgs_pass(bool fp32, int sweeps, const Geom &g, const void *src, void *dst,
                            const void *f, double a, double b, double gw, hipStream_t s) {
    switch (sweeps) {
        case 1: return JacobiLevels<2>::rb_pass(fp32, g, src, dst, f, a, b, gw, s);
        case 2: return JacobiLevels<4>::rb_pass(fp32, g, src, dst, f, a, b, gw, s);
        case 3: return JacobiLevels<6>::rb_pass(fp32, g, src, dst, f, a, b, gw, s);
        case 4: return JacobiLevels<8>::rb_pass(fp32, g, src, dst, f, a, b, gw, s);
        default: return hipErrorInvalidValue;
    }
}

size_t jacobi_batch_table_bytes(int njobs) { return JacobiLevels<1>::table_bytes(njobs); }

hipError_t launch_jacobi_batch(bool fp32, int tb, bool has_a, bool has_f,
                               const std::vector<JacBatchItem> &items, void *table_dev,
                               std::vector<unsigned char> &host_buf, hipStream_t s) {
    if (items.empty()) return hipSuccess;
    switch (tb) {
        case 1: return JacobiLevels<1>::batch(fp32, has_a, has_f, items, table_dev, host_buf, s);
        case 2: return JacobiLevels<2>::batch(fp32, has_a, has_f, items, table_dev, host_buf, s);
        case 3: return JacobiLevels<3>::batch(fp32, has_a, has_f, items, table_dev, host_buf, s);
        case 4: return JacobiLevels<4>::batch(fp32, has_a, has_f, items, table_dev, host_buf, s);
        case 5: return JacobiLevels<5>::batch(fp32, has_a, has_f, items, table_dev, host_buf, s);
        case 6: return JacobiLevels<6>::batch(fp32, has_a, has_f, items, table_dev, host_buf, s);
        case 7: return JacobiLevels<7>::batch(fp32, has_a, has_f, items, table_dev, host_buf, s);
        case 8: return JacobiLevels<8>::batch(fp32, has_a, has_f, items, table_dev, host_buf, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace stk
