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
//
// The state is addressed through raw buffer descriptors: a lane's column offsets are fixed for
// the whole segment, and a row's plane and row offsets are wave-uniform scalars, so no vector
// instruction computes an address on the fast path and a few scalar registers replace the 64-bit
// base of every plane.  A descriptor covers fewer than 2^31 bytes, so that an offset of 2^31 is
// out of range on its own: one covers the 14 planes of a state below 2^31 bytes, two (planes
// 0-6 and 7-13) a larger one whose halves are below it (tb2_descs).

// Fourth descriptor word of a raw buffer on the gfx9 family: 32-bit data format (a zero format
// makes raw loads return zero), no stride, no swizzle.
constexpr int kBufWord3 = 0x00020000;

// A per-lane offset at which a buffer access is out of range whatever the scalar offset: the
// hardware drops such a store and returns zero for such a load.  It needs ranges below 2^31
// bytes and scalar offsets below 2^31, so that the sum cannot wrap.
constexpr unsigned kBufOutOfRange = 0x80000000u;

__device__ __forceinline__ __amdgpu_buffer_rsrc_t buf_rsrc(const void* p, unsigned bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), 0, int(bytes), kBufWord3);
}

// Element at byte offset voff (per lane) + soff (wave-uniform) of a buffer.
template <typename S>
__device__ __forceinline__ S buf_load(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff) {
    if constexpr (sizeof(S) == 4)
        return __builtin_bit_cast(
            S, __builtin_amdgcn_raw_buffer_load_b32(r, int(voff), int(soff), 0));
    else
        return __builtin_bit_cast(
            S, __builtin_amdgcn_raw_buffer_load_b64(r, int(voff), int(soff), 0));
}

template <typename S>
__device__ __forceinline__ void buf_store(S v, __amdgpu_buffer_rsrc_t r, unsigned voff,
                                          unsigned soff) {
    typedef unsigned u32x2 __attribute__((ext_vector_type(2)));
    if constexpr (sizeof(S) == 4)
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, int(voff),
                                              int(soff), 0);
    else
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, int(voff),
                                              int(soff), 0);
}

// The 14 planes of a state through NDESC descriptors (1 or 2; see tb2_descs).  Plane indices
// are constants after unrolling, so the choice of descriptor costs nothing at run time.
template <typename S, int NDESC>
struct TbState {
    static_assert(NDESC == 1 || NDESC == 2, "one or two descriptors");
    __amdgpu_buffer_rsrc_t lo, hi;
    unsigned PB;   // bytes per plane
    __device__ __forceinline__ TbState(const void* base, unsigned pb) : PB(pb) {
        if constexpr (NDESC == 1) {
            lo = hi = buf_rsrc(base, kPlanes * pb);
        } else {
            lo = buf_rsrc(base, kPlanes / 2 * pb);
            hi = buf_rsrc(static_cast<const char*>(base) + size_t(kPlanes / 2) * pb,
                          kPlanes / 2 * pb);
        }
    }
    // plane p at byte offset voff (per lane) + soff (wave-uniform, within the plane)
    __device__ __forceinline__ S load(int p, unsigned voff, unsigned soff) const {
        if (NDESC == 1 || p < kPlanes / 2) return buf_load<S>(lo, voff, soff + unsigned(p) * PB);
        return buf_load<S>(hi, voff, soff + unsigned(p - kPlanes / 2) * PB);
    }
    __device__ __forceinline__ void store(S v, int p, unsigned voff, unsigned soff) const {
        if (NDESC == 1 || p < kPlanes / 2)
            buf_store<S>(v, lo, voff, soff + unsigned(p) * PB);
        else
            buf_store<S>(v, hi, voff, soff + unsigned(p - kPlanes / 2) * PB);
    }
};

// A value every lane of the wavefront holds, kept in a scalar register.
__device__ __forceinline__ unsigned wave_uniform(unsigned v) {
    return unsigned(__builtin_amdgcn_readfirstlane(int(v)));
}

// Raw inputs of the intermediate step at one node, loaded one row ahead of their use so that
// the loads are in flight while the previous row computes: the populations pulled at the node
// (its inward neighbour for a wall node) and the medium there and at the node itself.
template <typename S>
struct TbRaw {
    S f[9], g[5];
    S phi_f, K_f;   // medium where the populations are pulled
    S phi, K;       // medium at the node
};

// Byte offsets of one lane's columns, fixed over a segment: the node's, and those of the node
// it pulls from (its inward neighbour on a west or east wall) and of that node's west and east
// neighbours (wrapping, which only a periodic axis uses).
struct TbCols {
    unsigned x, f, fw, fe;
};

// Loads the raw inputs of the intermediate step at (x, r) for the lane's column.  r is a row
// of the grid; a row beyond a walled side is never consumed, and its caller passes any valid
// row instead.  Every load is unconditional, so every field is defined on every path.
template <typename S, bool PN, int NDESC>
__device__ __forceinline__ void tb_load(const TbState<S, NDESC>& rs, __amdgpu_buffer_rsrc_t rm,
                                        const Geo& G, unsigned PB, unsigned RB,
                                        const TbCols& c, int r, TbRaw<S>& raw) {
    const bool onS = G.wallS && r == 0, onN = G.wallN && r == G.ny - 1;
    const int yf = r + (onS ? 1 : 0) - (onN ? 1 : 0);
    const int ym = yf == 0 ? G.ny - 1 : yf - 1, yp = yf == G.ny - 1 ? 0 : yf + 1;
    const unsigned s0 = wave_uniform(unsigned(yf) * RB);
    const unsigned sm = wave_uniform(unsigned(ym) * RB);
    const unsigned sp = wave_uniform(unsigned(yp) * RB);
    // the medium first: the loop copies it between registers, and an early load is the one
    // most likely to have arrived by then
    if constexpr (PN) {
        const unsigned sr = wave_uniform(unsigned(r) * RB);
        raw.phi_f = buf_load<S>(rm, c.f, s0);
        raw.K_f = buf_load<S>(rm, c.f, s0 + PB);
        raw.phi = buf_load<S>(rm, c.x, sr);
        raw.K = buf_load<S>(rm, c.x, sr + PB);
    } else {
        raw.phi_f = raw.K_f = raw.phi = raw.K = S(1);
    }
    // f_i arrives from (xf - ex_i, yf - ey_i)
    raw.f[0] = rs.load(0, c.f, s0);
    raw.f[1] = rs.load(1, c.fw, s0);
    raw.f[2] = rs.load(2, c.f, sm);
    raw.f[3] = rs.load(3, c.fe, s0);
    raw.f[4] = rs.load(4, c.f, sp);
    raw.f[5] = rs.load(5, c.fw, sm);
    raw.f[6] = rs.load(6, c.fe, sm);
    raw.f[7] = rs.load(7, c.fe, sp);
    raw.f[8] = rs.load(8, c.fw, sp);
    raw.g[0] = rs.load(9, c.f, s0);
    raw.g[1] = rs.load(10, c.fw, s0);
    raw.g[2] = rs.load(11, c.f, sm);
    raw.g[3] = rs.load(12, c.fe, s0);
    raw.g[4] = rs.load(13, c.f, sp);
}

// The intermediate step at (x, r) from its raw inputs: node_state's arithmetic, then collide,
// rounded to the storage type; md receives the medium coefficients at (x, r).
template <typename S, typename R, bool PN>
__device__ __forceinline__ void tb_finish(const TbRaw<S>& raw, const Geo& G, const Phys<R>& P,
                                          int x, int r, S out[14], Med<R>& md) {
    R f[9], g[5];
#pragma unroll
    for (int i = 0; i < 9; ++i) f[i] = R(raw.f[i]);
#pragma unroll
    for (int i = 0; i < 5; ++i) g[i] = R(raw.g[i]);
    const bool onW = G.wallW && x == 0, onE = G.wallE && x == G.nx - 1;
    const bool onS = G.wallS && r == 0, onN = G.wallN && r == G.ny - 1;
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

// Row r of the intermediate step: wrapped on a periodic axis; beyond a walled side the row is
// absent (nothing consumes it) and row 0 stands in for it.
__device__ __forceinline__ int tb_row(const Geo& G, int r) {
    if (r >= 0 && r < G.ny) return r;
    if (G.wallS) return 0;
    return r < 0 ? r + G.ny : r - G.ny;
}

// One wavefront's share of a two-step launch: strip `strip` of row segment `seg` (rows per
// segment `rows`), swept towards increasing y (REV false) or decreasing y (REV true).  Every
// wavefront of the work-group calls this with the same segment and runs the same rows (an
// inactive one, past the last strip, stores nothing), since each row ends with a work-group
// barrier.
template <typename S, typename R, bool PN, bool REV, int NDESC>
__device__ __forceinline__ void tb2_sweep(const S* __restrict__ src, S* __restrict__ dst,
                                          const S* __restrict__ med, const Geo& G,
                                          const Phys<R>& P, int strip, bool active, int seg,
                                          int rows) {
    constexpr unsigned B = sizeof(S);
    constexpr int D = REV ? -1 : 1;              // direction of the sweep along y
    const unsigned PB = unsigned(G.plane) * B;   // bytes per plane
    const unsigned RB = unsigned(G.pitch) * B;   // bytes per row
    const TbState<S, NDESC> rs(src, PB), rd(dst, PB);
    const __amdgpu_buffer_rsrc_t rm = buf_rsrc(med, PN ? 2 * PB : 0);
    const int lane = threadIdx.x & 63;
    const int x0 = strip * kTbCols;
    // this lane's column, wrapped on a periodic axis; outside a walled side (or in an idle
    // wavefront) it is a stand-in whose results nothing consumes
    int x = x0 - 1 + lane;
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
    // lanes 1..kTbCols write step n+2 at their column
    const bool out_lane = active && lane >= 1 && lane <= kTbCols && x0 - 1 + lane < G.nx;
    const int ylo = seg * rows;
    const int yhi = min(ylo + rows, G.ny);
    // the sweep runs y = yb, yb + D, ..., ye - D
    const int yb = REV ? yhi - 1 : ylo;
    const int ye = REV ? ylo - 1 : yhi;
    // step n+1 at rows y - D (behind the sweep), y and y + D (ahead) of this lane's column
    S bh[14], cur[14], ah[14];
    Med<R> mdb, mdn;        // medium at (x, y) and (x, y + D)
    TbRaw<S> raw;
    {
        Med<R> unused;
        int r = tb_row(G, yb - D);
        tb_load<S, PN, NDESC>(rs, rm, G, PB, RB, cols, r, raw);
        tb_finish<S, R, PN>(raw, G, P, x, r, bh, unused);
        r = tb_row(G, yb);
        tb_load<S, PN, NDESC>(rs, rm, G, PB, RB, cols, r, raw);
        tb_finish<S, R, PN>(raw, G, P, x, r, cur, mdb);
        tb_load<S, PN, NDESC>(rs, rm, G, PB, RB, cols, tb_row(G, yb + D), raw);
        // 14 stores that the hardware drops, so that on entering the row loop, as on every
        // later row, the loads in flight are followed by 14 stores: the compiler's wait for
        // those loads at the top of the loop then leaves the previous row's stores in flight
        __builtin_amdgcn_sched_barrier(0);  // keep them after the loads
#pragma unroll
        for (int i = 0; i < 14; ++i) rd.store(S(0), i, kBufOutOfRange, 0);
    }
    // the last row's loads would fetch a row that nothing uses: out of range, they return zero
    // without a memory access
    const TbCols none = {kBufOutOfRange, kBufOutOfRange, kBufOutOfRange, kBufOutOfRange};
    // yb != ye on every segment; the work-group's waves run the same rows
    int y = yb;
    do {
        tb_finish<S, R, PN>(raw, G, P, x, tb_row(G, y + D), ah, mdn);
        // issue the next row's loads now; they complete during this row's work
        tb_load<S, PN, NDESC>(rs, rm, G, PB, RB, y + D == ye ? none : cols, tb_row(G, y + 2 * D),
                              raw);
        // step n+1 at rows y - 1 and y + 1, whichever way the sweep runs
        const S* dn = REV ? ah : bh;   // row y - 1
        const S* up = REV ? bh : ah;   // row y + 1
        // gather step n+1 populations arriving at (x, y): f_i from (x - ex_i, y - ey_i)
        const S f1 = __shfl_up(cur[1], 1, 64), g1 = __shfl_up(cur[10], 1, 64);
        const S f5 = __shfl_up(dn[5], 1, 64), f8 = __shfl_up(up[8], 1, 64);
        const S f3 = __shfl_down(cur[3], 1, 64), g3 = __shfl_down(cur[12], 1, 64);
        const S f6 = __shfl_down(dn[6], 1, 64), f7 = __shfl_down(up[7], 1, 64);
        const bool wall = (G.wallW && x == 0) || (G.wallE && x == G.nx - 1) ||
                          (G.wallS && y == 0) || (G.wallN && y == G.ny - 1);
        // Step n+2 runs on every lane; lanes that own no output (the strip's two halo lanes,
        // columns past the grid, wall nodes, which their inward neighbours step) store
        // through an offset outside the descriptor's range, which the hardware drops.  No
        // branch guards the stores, so the compiler knows they are issued after this row's
        // loads on every path and waits only for the loads at the next row (a guarded store
        // block made it wait for the stores as well, once per row).
        const bool own = out_lane && !wall;
        R f[9] = {R(cur[0]), R(f1), R(dn[2]), R(f3), R(up[4]), R(f5), R(f6), R(f7), R(f8)};
        R g[5] = {R(cur[9]), R(g1), R(dn[11]), R(g3), R(up[13])};
        const Med<R> md = mdb;
        const Mac<R> m = fluid_macros<R>(f, g, md, P);
        if (own)
            step_wall_neighbours<R, PN, S>(
                med, G, P, x, y, f, g, m, md, [&](int xb, int yb2, const R* fb, const R* gb) {
                    const unsigned ob =
                        (unsigned(yb2) * unsigned(G.pitch) + unsigned(xb)) * B;
#pragma unroll
                    for (int i = 0; i < 9; ++i) rd.store(S(fb[i]), i, ob, 0);
#pragma unroll
                    for (int i = 0; i < 5; ++i) rd.store(S(gb[i]), 9 + i, ob, 0);
                });
        collide<R>(f, g, m, md, P);
        // plain stores: a strip's edge lines are shared with its neighbour, and merge in L2
        // before they go to HBM (non-temporal stores cost 10 % here)
        const unsigned vo = own ? cols.x : kBufOutOfRange;
        const unsigned sy = wave_uniform(unsigned(y) * RB);
#pragma unroll
        for (int i = 0; i < 9; ++i) rd.store(S(f[i]), i, vo, sy);
#pragma unroll
        for (int i = 0; i < 5; ++i) rd.store(S(g[i]), 9 + i, vo, sy);
#pragma unroll
        for (int i = 0; i < 14; ++i) {
            bh[i] = cur[i];
            cur[i] = ah[i];
        }
        mdb = mdn;
        __syncthreads();
        y += D;
    } while (y != ye);
}

// One wavefront's share of a two-step launch: strip `strip` of row segment `seg`.  Adjacent
// segments sweep in opposite directions (even segments towards increasing y, odd ones towards
// decreasing y), so that two neighbouring segments read the rows on their common boundary at
// the same time, at both ends of the sweep: running side by side on one XCD, the second reads
// them from L2 instead of memory.  (Swept the same way, the second reached those rows ~rows
// iterations later, after some 2 MB per iteration per XCD had gone through its 4 MB L2.)
template <typename S, typename R, bool PN, int NDESC = 1>
__device__ __forceinline__ void tb2_segment(const S* __restrict__ src, S* __restrict__ dst,
                                            const S* __restrict__ med, const Geo& G,
                                            const Phys<R>& P, int strip, bool active, int seg,
                                            int rows) {
    if (seg & 1)
        tb2_sweep<S, R, PN, true, NDESC>(src, dst, med, G, P, strip, active, seg, rows);
    else
        tb2_sweep<S, R, PN, false, NDESC>(src, dst, med, G, P, strip, active, seg, rows);
}

// Work-groups are dealt round-robin over the 8 XCDs.  This maps a launch's work-group index to a
// logical one (a bijection) so that each XCD takes chunks of `chunk` consecutive logical
// work-groups, the 8 XCDs' chunks side by side: with `chunk` the number of work-groups an XCD
// holds at once, the work-groups resident together form one contiguous band of the grid, each
// XCD's part of it contiguous, so neighbouring strips and segments share that XCD's L2 and all
// XCDs stream nearby rows.  Measured on the 4096^2 FP32 workload: chunks of 128 (one XCD's
// resident set) 66.9k MLUPS, 32: 65.8k, one contiguous range per XCD: 65.5k, plain
// round-robin: 64.3k.  The last incomplete round of chunks falls back to contiguous ranges.
__device__ __forceinline__ int tb_logical_group(int chunk) {
    const int n = gridDim.x, wg = blockIdx.x, xcd = wg % 8, slot = wg / 8;
    const int base = n - n % (8 * chunk);
    const int logical = ((slot / chunk) * 8 + xcd) * chunk + slot % chunk;
    if (logical < base) return logical;
    const int rest = n - base, per = rest / 8, extra = rest % 8;
    return base + xcd * per + min(xcd, extra) + (slot - base / 8);
}

}  // namespace lbm
