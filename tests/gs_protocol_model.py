"""Host model of the Gauss-Seidel wavefront protocol (test infrastructure).

A step-by-step Python emulation of what each wave of the GPU kernel does --
ticket order 2*tau + J + K, per-(sweep, bundle) progress counters, waits
before each chunk load, the 32-position LDS ring with 8-position chunks, the
lane skew i = T - jj - kk -- with a random interleaving of a few "waves".  It
checks the protocol itself (termination for any interleaving and the
fresh/old data each site reads), independently of the HIP code.  Values are
computed with the Sec. 3 update in the same operand order, so the result must
equal the oracle's sequential sweep bit for bit.

Chunks are aligned per line: chunk c of a line covers positions
[8c - s, 8c + 8 - s), where s (0..7) is the line's element offset of i = 0
from an 8-element boundary of the array (base_off shifts the whole array, as
a different allocation alignment would).  Producer and consumer compute s
from the same address, so "chunk c" names the same positions on both sides.
"""
import random

import numpy as np


C, RING = 8, 32

def items_table(nj, nk, S):
    out = []
    kmax = 2*(S-1) + (nj-1) + (nk-1)
    for key in range(kmax+1):
        for tau in range(S):
            rest = key - 2*tau
            if rest < 0: break
            for J in range(nj):
                K = rest - J
                if K < 0: break
                if K >= nk: continue
                out.append((tau, J, K))
    return out

def staged_slot(li):
    if li < 8: return li + 1
    if li < 88: return 10 + (li - 8)
    return 90 + (li - 88) + 1

def simulate(u0, S, h=1, workers=3, seed=0, a=0.0, b=1/6, p_early=0.3, publish_lag=3,
             base_off=0, store_shift_error=0):
    """Run the schedule with `workers` interleaved waves.  Every global load
    and store takes effect at a random moment between its issue and the next
    point where the kernel waits for all of its memory operations (a chunk
    load may also be needed earlier, at its commit to LDS).  publish_lag is
    the kernel's 3 (boundary b publishes chunk b-3, whose stores were issued
    one boundary earlier); 2 would publish a chunk before its stores."""
    u = u0.copy()
    pz, py, px = u.shape
    nz, ny, nx = pz-2*h, py-2*h, px-2*h
    nj, nk = (ny+7)//8, (nz+7)//8
    # chunk counts valid for every line shift s in 0..7: stores reach i = nx-1,
    # loads the x+ ghost i = nx, blocks the last site of the most skewed lane
    ncs = (nx + 6)//C + 1; ncl = (nx + 7)//C + 1; nb = (nx + 14 + C - 1)//C

    def shift(kg, jg):  # element offset of (kg, jg, i=0) past an 8-element boundary
        return (base_off + (kg*py + jg)*px + h) % C
    items = items_table(nj, nk, S)
    # topological check
    pos = {it: n for n, it in enumerate(items)}
    for (tau, J, K), n in pos.items():
        deps = [(tau, J-1, K), (tau, J, K-1), (tau-1, J+1, K), (tau-1, J, K+1), (tau-1, J, K)]
        for d in deps:
            if d in pos: assert pos[d] < n, ("not topological", d, (tau, J, K))
    P = np.zeros((S, nj*nk), dtype=np.int64)
    ticket = [0]
    rng = random.Random(seed)

    def worker():
        while True:
            t = ticket[0]; ticket[0] += 1
            if t >= len(items): return
            tau, J, K = items[t]
            j0, k0 = h + 8*J, h + 8*K
            me = K*nj + J
            ring = np.zeros((100, RING))
            xm = np.zeros(64)
            lanes = [(l >> 3, l & 7) for l in range(64)]  # (jj, kk)
            for l, (jj, kk) in enumerate(lanes):
                j, k = j0+jj, k0+kk
                if j < h+ny and k < h+nz: xm[l] = u[k, j, h-1]
            pending = []   # memory operations issued and not yet performed
            def tick():    # some of them take effect now
                for op in list(pending):
                    if rng.random() < p_early:
                        pending.remove(op); op()
            def wait_all():  # the kernel waits for every memory operation
                while pending:
                    pending.pop(0)()
            def wait_chunk(c):
                if c >= ncs: return  # only positions >= nx: never written
                conds = []
                if tau > 0:
                    conds.append((tau-1, me))
                    if J+1 < nj: conds.append((tau-1, me+1))
                    if K+1 < nk: conds.append((tau-1, me+nj))
                if J > 0: conds.append((tau, me-1))
                if K > 0: conds.append((tau, me-nj))
                for (q0, q1) in conds:
                    while P[q0, q1] < c + 1:
                        yield "wait"
            pf = {}
            def issue_load(c):  # global -> registers, read at some later moment
                vals = {}
                def read():
                    for e in range(768):
                        li = e >> 3
                        slot = staged_slot(li); jl, kl = slot % 10, slot // 10
                        jg, kg = j0-1+jl, k0-1+kl
                        i = c*C + (e & 7) - shift(kg, jg)
                        ok = 0 <= i <= nx and jg <= h+ny and kg <= h+nz
                        vals[e] = (slot, i & (RING-1), u[kg, jg, h+i] if ok else 0.0)
                pf["c"] = (vals, read)
                pending.append(read)
            def commit_load(c):  # registers -> LDS ring (the load has completed)
                vals, read = pf["c"]
                if read in pending:
                    pending.remove(read); read()
                for slot, r, v in vals.values():
                    ring[slot, r] = v
            def issue_store(c):  # LDS read now; global write at some later moment
                vals = []
                for e in range(512):
                    li = e >> 3; jq, kq = li & 7, li >> 3
                    jg, kg = j0+jq, k0+kq
                    i = c*C + (e & 7) - (shift(kg, jg) + store_shift_error) % C
                    if 0 <= i < nx and jg < h+ny and kg < h+nz:
                        vals.append((kg, jg, h+i, ring[(kq+1)*10 + jq+1, i & (RING-1)]))
                def write():
                    for kg, jg, ig, v in vals:
                        u[kg, jg, ig] = v
                pending.append(write)
            def publish(c):
                P[tau, me] = c + 1
            yield from wait_chunk(0); issue_load(0); commit_load(0)
            if ncl > 1:
                yield from wait_chunk(1); issue_load(1); commit_load(1)
            if ncl > 2:
                yield from wait_chunk(2); issue_load(2)
            for bb in range(nb):
                for st in range(C):
                    T = bb*C + st
                    writes = []
                    for l, (jj, kk) in enumerate(lanes):
                        j, k = j0+jj, k0+kk
                        i = T - jj - kk
                        if j < h+ny and k < h+nz and 0 <= i < nx:
                            own = (kk+1)*10 + jj+1; p = i & 31
                            s = xm[l] + ring[own, (i+1) & 31]
                            s = s + ring[own-1, p]; s = s + ring[own+1, p]
                            s = s + ring[own-10, p]; s = s + ring[own+10, p]
                            v = (a*ring[own, p]) + (b*s) if a != 0 else b*s
                            writes.append((own, p, v, l))
                    for own, p, v, l in writes:
                        ring[own, p] = v; xm[l] = v
                    tick()
                    yield "step"
                wait_all()
                if 0 <= bb-publish_lag < ncs: publish(bb-publish_lag)
                yield "boundary"
                if 0 <= bb-2 < ncs: issue_store(bb-2)
                tick()
                if bb+2 < ncl: commit_load(bb+2)
                if bb+3 < ncl:
                    yield from wait_chunk(bb+3); issue_load(bb+3)
            wait_all()
            if 0 <= nb-3 < ncs: publish(nb-3)
            for cs in range(max(0, nb-2), ncs):
                issue_store(cs); wait_all(); publish(cs)
    ws = [worker() for _ in range(workers)]
    stall = 0
    while ws:
        w = rng.choice(ws)
        try:
            r = next(w)
            stall = stall + 1 if r == "wait" else 0
            if stall > 200000: raise RuntimeError("deadlock")
        except StopIteration:
            ws.remove(w)
    return u
