// lbm_tb3.hpp -- three time steps per launch (temporal blocking) for the pull layout, FP32.
#pragma once

#include "lbm_tb2.hpp"

namespace lbm {

// Three time steps per launch, bitwise equal to three launches of step_kernel.  Each wavefront
// owns a strip of kTb3Cols columns and sweeps a segment of rows; lane l holds column
// x0 - 2 + l.  Per row it computes step n+1 from memory (as the two-step kernel does, kept in
// registers, three rows), step n+2 from those rows across lanes (written to a three-row ring in
// LDS, one per wavefront: lanes 1..62 are right), and step n+3 from the ring (lanes 2..61,
// stored).  A wall node's step n+2 comes from its inward neighbour's lane, which writes it into
// the ring; on a south or north wall that row must already have its slot, so the segment that
// holds a walled end sweeps away from it: segment 0 forwards, the last segment backwards (a
// wall row ahead of a sweep is never needed, and its writes are dropped).  Per three steps each
// node crosses memory about once each way, plus the halo rows of the intermediate steps.
constexpr int kTb3Cols = 60;
constexpr int kTb3Waves = 4;
constexpr int kTb3Ring = 3 * kPlanes * 64;   // ring elements per wavefront

template <typename S, typename R, bool PN, bool REV>
__device__ __forceinline__ void tb3_sweep(const S* __restrict__ src, S* __restrict__ dst,
                                          const S* __restrict__ med, const Geo& G,
                                          const Phys<R>& P, int strip, bool active, int ylo,
                                          int yhi, S* __restrict__ ring) {
    constexpr unsigned B = sizeof(S);
    constexpr int D = REV ? -1 : 1;
    const unsigned PB = unsigned(G.plane) * B;
    const unsigned RB = unsigned(G.pitch) * B;
    const TbState<S, 1> rs(src, PB), rd(dst, PB);
    const __amdgpu_buffer_rsrc_t rm = buf_rsrc(med, PN ? 2 * PB : 0);
    const int lane = threadIdx.x & 63;
    const int x0 = strip * kTb3Cols;
    const int ux = x0 - 2 + lane;   // the lane's column, unwrapped
    int x = ux;
    if (x < 0 || x >= G.nx) {
        x = x < 0 ? x + G.nx : x - G.nx;
        if (x < 0 || x >= G.nx) x = 0;
    }
    TbCols cols;
    {
        const bool onW = G.wallW && x == 0, onE = G.wallE && x == G.nx - 1;
        const int xf = x + (onW ? 1 : 0) - (onE ? 1 : 0);
        cols.x = unsigned(x) * B;
        cols.f = unsigned(xf) * B;
        cols.fw = unsigned(xf == 0 ? G.nx - 1 : xf - 1) * B;
        cols.fe = unsigned(xf == G.nx - 1 ? 0 : xf + 1) * B;
    }
    const bool in_grid = ux >= 0 && ux < G.nx;
    const bool wall_x = (G.wallW && x == 0) || (G.wallE && x == G.nx - 1);
    // Step n+2 goes to the ring from lanes 1..62; on a periodic x axis also from the lanes
    // beyond the grid, whose wrapped columns are the halo that step n+3 at columns 0 and nx - 1
    // reads (beyond a wall nothing reads them).
    const bool mid_lane = active && lane >= 1 && lane <= kTb3Cols + 2 && (in_grid || !G.wallW);
    const bool out_lane = active && lane >= 2 && lane <= kTb3Cols + 1 && in_grid;
    const int lm = lane > 0 ? lane - 1 : 0, lp = lane < 63 ? lane + 1 : 63;
    const int yb = REV ? yhi - 1 : ylo;
    const int ye = REV ? ylo - 1 : yhi;
    // ring slot of the row with sweep index i (row yb + i * D), i >= -2
    auto slot = [&](int i) { return ring + ((i + 3) % 3) * (kPlanes * 64); };

    // Step n+2 at the row of sweep index qi from step n+1 at rows qi - 1, qi, qi + 1 (dn, cur,
    // up in grid orientation) and the medium there; into the ring.
    auto mid = [&](int qi, const S* dn, const S* cur, const S* up, const Med<R>& md) {
        const int qg = tb_row(G, yb + qi * D);
        const S f1 = __shfl_up(cur[1], 1, 64), g1 = __shfl_up(cur[10], 1, 64);
        const S f5 = __shfl_up(dn[5], 1, 64), f8 = __shfl_up(up[8], 1, 64);
        const S f3 = __shfl_down(cur[3], 1, 64), g3 = __shfl_down(cur[12], 1, 64);
        const S f6 = __shfl_down(dn[6], 1, 64), f7 = __shfl_down(up[7], 1, 64);
        const bool wall = wall_x || (G.wallS && qg == 0) || (G.wallN && qg == G.ny - 1);
        const bool own = mid_lane && !wall;
        R f[9] = {R(cur[0]), R(f1), R(dn[2]), R(f3), R(up[4]), R(f5), R(f6), R(f7), R(f8)};
        R g[5] = {R(cur[9]), R(g1), R(dn[11]), R(g3), R(up[13])};
        const Mac<R> m = fluid_macros<R>(f, g, md, P);
        if (own)
            step_wall_neighbours<R, PN, S>(
                med, G, P, x, qg, f, g, m, md, [&](int xb, int yb2, const R* fb, const R* gb) {
                    const int di = (yb2 - qg) * D;   // -1 behind, 0 this row, 1 ahead
                    if (di > 0) return;              // ahead of the sweep: not needed here
                    S* sl = slot(qi + di);
                    const int lb = lane + (xb - x);
#pragma unroll
                    for (int i = 0; i < 9; ++i) sl[i * 64 + lb] = S(fb[i]);
#pragma unroll
                    for (int i = 0; i < 5; ++i) sl[(9 + i) * 64 + lb] = S(gb[i]);
                });
        collide<R>(f, g, m, md, P);
        if (own) {
            S* sl = slot(qi);
#pragma unroll
            for (int i = 0; i < 9; ++i) sl[i * 64 + lane] = S(f[i]);
#pragma unroll
            for (int i = 0; i < 5; ++i) sl[(9 + i) * 64 + lane] = S(g[i]);
        }
    };

    // step n+1 at rows yb - 2D .. yb + D, and step n+2 at rows yb - D and yb
    S r0[14], r1[14], r2[14];
    Med<R> md0, md1;   // medium at rows y and y + D of the loop below
    TbRaw<S> raw;
    {
        Med<R> mda, mdb;
        S ra[14];
        int r = tb_row(G, yb - 2 * D);
        tb_load<S, PN, 1>(rs, rm, G, PB, RB, cols, r, raw);
        tb_finish<S, R, PN>(raw, G, P, x, r, ra, mda);
        r = tb_row(G, yb - D);
        tb_load<S, PN, 1>(rs, rm, G, PB, RB, cols, r, raw);
        tb_finish<S, R, PN>(raw, G, P, x, r, r0, mdb);
        r = tb_row(G, yb);
        tb_load<S, PN, 1>(rs, rm, G, PB, RB, cols, r, raw);
        tb_finish<S, R, PN>(raw, G, P, x, r, r1, md0);
        mid(-1, REV ? r1 : ra, r0, REV ? ra : r1, mdb);
        r = tb_row(G, yb + D);
        tb_load<S, PN, 1>(rs, rm, G, PB, RB, cols, r, raw);
        tb_finish<S, R, PN>(raw, G, P, x, r, r2, md1);
        mid(0, REV ? r2 : r0, r1, REV ? r0 : r2, md0);
        tb_load<S, PN, 1>(rs, rm, G, PB, RB, cols, tb_row(G, yb + 2 * D), raw);
    }
    // from here r1 holds step n+1 at row y, r2 at row y + D
    const TbCols none = {kBufOutOfRange, kBufOutOfRange, kBufOutOfRange, kBufOutOfRange};
    int y = yb;
    do {
        const int yi = (y - yb) * D;
        S a[14];
        Med<R> md2;
        tb_finish<S, R, PN>(raw, G, P, x, tb_row(G, y + 2 * D), a, md2);
        tb_load<S, PN, 1>(rs, rm, G, PB, RB, y + D == ye ? none : cols, tb_row(G, y + 3 * D),
                          raw);
        mid(yi + 1, REV ? a : r1, r2, REV ? r1 : a, md1);
        __syncthreads();
        // step n+3 at (x, y) from the ring: f_i from (x - ex_i, y - ey_i)
        const S* cr = slot(yi);
        const S* dn = slot(yi - D);   // row y - 1
        const S* up = slot(yi + D);   // row y + 1
        R f[9] = {R(cr[0 * 64 + lane]), R(cr[1 * 64 + lm]), R(dn[2 * 64 + lane]),
                  R(cr[3 * 64 + lp]),   R(up[4 * 64 + lane]), R(dn[5 * 64 + lm]),
                  R(dn[6 * 64 + lp]),   R(up[7 * 64 + lp]),   R(up[8 * 64 + lm])};
        R g[5] = {R(cr[9 * 64 + lane]), R(cr[10 * 64 + lm]), R(dn[11 * 64 + lane]),
                  R(cr[12 * 64 + lp]), R(up[13 * 64 + lane])};
        const bool wall = wall_x || (G.wallS && y == 0) || (G.wallN && y == G.ny - 1);
        const bool own = out_lane && !wall;
        const Mac<R> m = fluid_macros<R>(f, g, md0, P);
        if (own)
            step_wall_neighbours<R, PN, S>(
                med, G, P, x, y, f, g, m, md0, [&](int xb, int yb2, const R* fb, const R* gb) {
                    const unsigned ob =
                        (unsigned(yb2) * unsigned(G.pitch) + unsigned(xb)) * B;
#pragma unroll
                    for (int i = 0; i < 9; ++i) rd.store(S(fb[i]), i, ob, 0);
#pragma unroll
                    for (int i = 0; i < 5; ++i) rd.store(S(gb[i]), 9 + i, ob, 0);
                });
        collide<R>(f, g, m, md0, P);
        const unsigned vo = own ? cols.x : kBufOutOfRange;
        const unsigned sy = wave_uniform(unsigned(y) * RB);
#pragma unroll
        for (int i = 0; i < 9; ++i) rd.store(S(f[i]), i, vo, sy);
#pragma unroll
        for (int i = 0; i < 5; ++i) rd.store(S(g[i]), 9 + i, vo, sy);
#pragma unroll
        for (int i = 0; i < 14; ++i) {
            r1[i] = r2[i];
            r2[i] = a[i];
        }
        md0 = md1;
        md1 = md2;
        y += D;
    } while (y != ye);
}

}  // namespace lbm
