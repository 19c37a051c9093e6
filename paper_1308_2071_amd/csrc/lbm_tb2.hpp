// lbm_tb2.hpp -- two time steps per launch (temporal blocking) for the pull layout: the per
// strip-and-segment work shared by the single-cavity and the batched two-step kernels.
#pragma once

#include "lbm_device.hpp"
#include "lbm_internal.hpp"

namespace lbm {

// Two time steps per launch (temporal blocking), pull layout, bitwise equal to two launches of
// step_kernel.  Each wavefront owns a strip of kTbCols columns and sweeps a segment of rows.
// Lane l computes the intermediate step n+1 at column x0 - 1 + l (the strip plus one column
// on each side) for each row, straight from the step-n buffer, and keeps three consecutive
// rows of it in registers, rounded to the storage type as a store would round them.  Step n+2
// at row y then gathers its populations from those registers: from its own lane and, across
// lanes, from its left and right neighbours.  A wall node is stepped by its inward
// neighbour's lane, which holds the populations its reconstruction needs.  Per two steps each
// node's populations cross HBM about once each way (plus the halo of the intermediate step),
// against twice for two single steps.

// Raw inputs of the intermediate step at one node, loaded one row ahead of their use so that
// the loads are in flight while the previous row computes: the populations pulled at the node
// (its inward neighbour for a wall node) and the medium there and at the node itself.
template <typename S>
struct TbRaw {
    S f[9], g[5];
    S phi_f, K_f;   // medium where the populations are pulled
    S phi, K;       // medium at the node
};

template <typename S, bool PN>
__device__ __forceinline__ void tb_load(const S* __restrict__ src, const S* __restrict__ med,
                                        const Geo& G, int x, bool ok, int r, TbRaw<S>& raw) {
    // every field is assigned on every path (a field set on one branch only would keep the
    // struct in scratch memory)
    S phi_f = S(1), K_f = S(1), phi = S(1), K = S(1);
    if (ok) {
        const bool onW = G.wallW && x == 0, onE = G.wallE && x == G.nx - 1;
        const bool onS = G.wallS && r == 0, onN = G.wallN && r == G.ny - 1;
        const int xf = x + (onW ? 1 : 0) - (onE ? 1 : 0);
        const int yf = r + (onS ? 1 : 0) - (onN ? 1 : 0);
        pull<S, S>(src, G, xf, yf, raw.f, raw.g);
        if constexpr (PN) {
            constexpr unsigned B = sizeof(S);
            const unsigned of = (unsigned(yf) * unsigned(G.pitch) + unsigned(xf)) * B;
            const unsigned o = (unsigned(r) * unsigned(G.pitch) + unsigned(x)) * B;
            phi_f = at(med, of);
            K_f = at(plane(med, 1, G.plane), of);
            phi = at(med, o);
            K = at(plane(med, 1, G.plane), o);
        }
    } else {
#pragma unroll
        for (int i = 0; i < 9; ++i) raw.f[i] = S(0);
#pragma unroll
        for (int i = 0; i < 5; ++i) raw.g[i] = S(0);
    }
    raw.phi_f = phi_f;
    raw.K_f = K_f;
    raw.phi = phi;
    raw.K = K;
}

// The intermediate step at (x, r) from its raw inputs: node_state's arithmetic, then collide,
// rounded to the storage type.
template <typename S, typename R, bool PN>
__device__ __forceinline__ void tb_finish(const TbRaw<S>& raw, const Geo& G, const Phys<R>& P,
                                          int x, bool ok, int r, S out[14]) {
    if (!ok) {
#pragma unroll
        for (int i = 0; i < 14; ++i) out[i] = S(0);
        return;
    }
    R f[9], g[5];
#pragma unroll
    for (int i = 0; i < 9; ++i) f[i] = R(raw.f[i]);
#pragma unroll
    for (int i = 0; i < 5; ++i) g[i] = R(raw.g[i]);
    const bool onW = G.wallW && x == 0, onE = G.wallE && x == G.nx - 1;
    const bool onS = G.wallS && r == 0, onN = G.wallN && r == G.ny - 1;
    Med<R> md;
    Mac<R> m;
    if constexpr (PN)
        md = medium_from<R>(R(raw.phi), R(raw.K), P);
    else
        md = Med<R>{P.phi, P.inv_phi, P.c_lin, P.c_nl};
    if (!(onW || onE || onS || onN)) {
        m = fluid_macros<R>(f, g, md, P);
    } else {
        Med<R> mdf = md;
        if constexpr (PN) mdf = medium_from<R>(R(raw.phi_f), R(raw.K_f), P);
        const Mac<R> mf = fluid_macros<R>(f, g, mdf, P);
        m = wall_state<R>(onW, onE, onS, onN, f, g, mf, mdf, md, P);
    }
    collide<R>(f, g, m, md, P);
#pragma unroll
    for (int i = 0; i < 9; ++i) out[i] = S(f[i]);
#pragma unroll
    for (int i = 0; i < 5; ++i) out[9 + i] = S(g[i]);
}

// Row r of the intermediate step as seen from this lane: wrapped on a periodic axis, absent
// beyond a walled side.
__device__ __forceinline__ bool tb_rowc(const Geo& G, bool col_ok, int& r) {
    if (r >= 0 && r < G.ny) return col_ok;
    if (G.wallS) return false;
    r = r < 0 ? r + G.ny : r - G.ny;
    return col_ok;
}

// One wavefront's share of a two-step launch: strip `strip` of row segment `seg` (rows per
// segment `rows`).  Every wavefront of the work-group calls this with the same
// segment and runs the same rows (an inactive one, past the last strip, loads and stores
// nothing), since each row ends with a work-group barrier.
template <typename S, typename R, bool PN>
__device__ __forceinline__ void tb2_segment(const S* __restrict__ src, S* __restrict__ dst,
                                            const S* __restrict__ med, const Geo& G,
                                            const Phys<R>& P, int strip, bool active, int seg,
                                            int rows) {
    const int lane = threadIdx.x & 63;
    const int x0 = strip * kTbCols;
    // this lane's column; outside a walled side it computes nothing
    int x = x0 - 1 + lane;
    bool col_ok = active;
    if (x < 0 || x >= G.nx) {
        col_ok = active && !G.wallW;
        x = x < 0 ? x + G.nx : x - G.nx;
        if (x < 0 || x >= G.nx) x = 0;  // only reached by an idle wavefront
    }
    // lanes 1..kTbCols write step n+2 at their column
    const bool out_lane = active && lane >= 1 && lane <= kTbCols && x0 - 1 + lane < G.nx;
    const int y0 = seg * rows;
    const int y1 = min(y0 + rows, G.ny);
    S a[14], b[14], c[14];  // step n+1 at rows y-1, y, y+1 of this lane's column
    S phib = S(1), Kb = S(1), phic = S(1), Kc = S(1);  // medium at (x, y) and (x, y + 1)
    TbRaw<S> raw;
    {
        int r = y0 - 1;
        bool ok = tb_rowc(G, col_ok, r);
        tb_load<S, PN>(src, med, G, x, ok, r, raw);
        tb_finish<S, R, PN>(raw, G, P, x, ok, r, a);
        r = y0;
        ok = tb_rowc(G, col_ok, r);
        tb_load<S, PN>(src, med, G, x, ok, r, raw);
        tb_finish<S, R, PN>(raw, G, P, x, ok, r, b);
        phib = raw.phi;
        Kb = raw.K;
        r = y0 + 1;
        ok = tb_rowc(G, col_ok, r);
        tb_load<S, PN>(src, med, G, x, ok, r, raw);
    }
    for (int y = y0; y < y1; ++y) {
        {
            int r = y + 1;
            const bool ok = tb_rowc(G, col_ok, r);
            tb_finish<S, R, PN>(raw, G, P, x, ok, r, c);
            phic = raw.phi;
            Kc = raw.K;
            r = y + 2;  // issue the next row's loads now; they complete during this row's work
            const bool ok2 = tb_rowc(G, col_ok, r);
            tb_load<S, PN>(src, med, G, x, ok2, r, raw);
        }
        // gather step n+1 populations arriving at (x, y): f_i from (x - ex_i, y - ey_i)
        const S f1 = __shfl_up(b[1], 1, 64), g1 = __shfl_up(b[10], 1, 64);
        const S f5 = __shfl_up(a[5], 1, 64), f8 = __shfl_up(c[8], 1, 64);
        const S f3 = __shfl_down(b[3], 1, 64), g3 = __shfl_down(b[12], 1, 64);
        const S f6 = __shfl_down(a[6], 1, 64), f7 = __shfl_down(c[7], 1, 64);
        const bool wall = (G.wallW && x == 0) || (G.wallE && x == G.nx - 1) ||
                          (G.wallS && y == 0) || (G.wallN && y == G.ny - 1);
        if (out_lane && !wall) {
            R f[9] = {R(b[0]), R(f1), R(a[2]), R(f3), R(c[4]), R(f5), R(f6), R(f7), R(f8)};
            R g[5] = {R(b[9]), R(g1), R(a[11]), R(g3), R(c[13])};
            Med<R> md;
            if constexpr (PN)
                md = medium_from<R>(R(phib), R(Kb), P);
            else
                md = Med<R>{P.phi, P.inv_phi, P.c_lin, P.c_nl};
            const Mac<R> m = fluid_macros<R>(f, g, md, P);
            step_wall_neighbours<R, PN, S>(
                med, G, P, x, y, f, g, m, md, [&](int xb, int yb, const R* fb, const R* gb) {
                    const unsigned ob = unsigned(yb) * unsigned(G.pitch) + unsigned(xb);
#pragma unroll
                    for (int i = 0; i < 9; ++i) plane(dst, i, G.plane)[ob] = S(fb[i]);
#pragma unroll
                    for (int i = 0; i < 5; ++i) plane(dst, 9 + i, G.plane)[ob] = S(gb[i]);
                });
            collide<R>(f, g, m, md, P);
            const unsigned o =
                (unsigned(y) * unsigned(G.pitch) + unsigned(x)) * unsigned(sizeof(S));
            // plain stores: a strip's edge lines are shared with its neighbour, and merge in
            // L2 before they go to HBM (non-temporal stores cost 10 % here)
#pragma unroll
            for (int i = 0; i < 9; ++i) at(plane(dst, i, G.plane), o) = S(f[i]);
#pragma unroll
            for (int i = 0; i < 5; ++i) at(plane(dst, 9 + i, G.plane), o) = S(g[i]);
        }
#pragma unroll
        for (int i = 0; i < 14; ++i) {
            a[i] = b[i];
            b[i] = c[i];
        }
        phib = phic;
        Kb = Kc;
        __syncthreads();
    }
}

// Work-groups are dealt round-robin over the 8 XCDs; this maps a launch's work-group index to a
// logical one so that each XCD gets a contiguous range of logical work-groups (a bijection), and
// neighbouring strips and segments share its L2.
__device__ __forceinline__ int tb_logical_group() {
    const int n = gridDim.x, per = n / 8, extra = n % 8;
    const int wg = blockIdx.x, xcd = wg % 8, slot = wg / 8;
    return xcd * per + min(xcd, extra) + slot;
}

}  // namespace lbm
