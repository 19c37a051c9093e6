// lbm_tile.hip -- several time steps per launch on small grids: each work-group advances one
// square tile of the lattice several steps in LDS (16 x 16 tiles four steps, or on the smallest
// grids 8 x 8 tiles eight steps).
#include "lbm_device.hpp"
#include "lbm_internal.hpp"

namespace lbm {

// On a small grid a step is a few microseconds of fixed cost (the launch, one round of loads
// from L2, the drain of the stores) around a short computation, and one step per launch pays
// that cost every step.  Here a work-group loads its tile of TS x TS nodes plus a halo of K
// nodes on each open side (and one more where the tile is one node thick at a walled end, so
// that its wall nodes' inward neighbours are covered), runs K steps on the region in LDS (two
// buffers, in turn), and writes the tile back: bitwise the result of K launches of step_kernel
// (same per-node arithmetic, and the LDS holds the storage type as a store would round it).
//
// A region node can take step s when every value it reads is valid after step s - 1.  With d
// the node's distance to the region's open sides (a side is closed where it is a wall of the
// grid; on a periodic axis both sides are open) that holds for d >= s, and for a wall node,
// which reads around its inward neighbour, for d(inward neighbour) >= s.  The tile's nodes then
// take every step.  Nodes that cannot are skipped; their stale values are read by no node that
// takes the step.

// LDS row stride and plane stride of a region (its largest side; the same for both forms).
constexpr int kTileRegion = kTileSide + 2 * kTileSteps + 1;
constexpr int kTilePlane = kTileRegion * kTileRegion;

// Pull streaming (Eqs. (18), (35)) from a region in LDS: f_i from (lx - ex_i, ly - ey_i).
template <typename R, typename S>
__device__ __forceinline__ void tile_pull(const S* __restrict__ A, int lx, int ly, R f[9],
                                          R g[5]) {
    constexpr int W = kTileRegion, L = kTilePlane;
    const int c = ly * W + lx;
    f[0] = R(A[0 * L + c]);
    f[1] = R(A[1 * L + c - 1]);
    f[2] = R(A[2 * L + c - W]);
    f[3] = R(A[3 * L + c + 1]);
    f[4] = R(A[4 * L + c + W]);
    f[5] = R(A[5 * L + c - W - 1]);
    f[6] = R(A[6 * L + c - W + 1]);
    f[7] = R(A[7 * L + c + W + 1]);
    f[8] = R(A[8 * L + c + W - 1]);
    g[0] = R(A[9 * L + c]);
    g[1] = R(A[10 * L + c - 1]);
    g[2] = R(A[11 * L + c - W]);
    g[3] = R(A[12 * L + c + 1]);
    g[4] = R(A[13 * L + c + W]);
}

template <typename R, bool PN, typename S>
__device__ __forceinline__ Med<R> tile_medium(const S* __restrict__ M, int lx, int ly,
                                              const Phys<R>& P) {
    if constexpr (PN) {
        const int c = ly * kTileRegion + lx;
        return medium_from<R>(R(M[c]), R(M[kTilePlane + c]), P);
    } else {
        return Med<R>{P.phi, P.inv_phi, P.c_lin, P.c_nl};
    }
}

// Global coordinate of region coordinate r on an axis of n nodes starting at r0 (wrapped on a
// periodic axis).
__device__ __forceinline__ int tile_wrap(int r, int n, bool periodic) {
    if (!periodic) return r;
    r %= n;
    return r < 0 ? r + n : r;
}

template <typename S, typename R, bool PN, int TS, int K>
__global__ __launch_bounds__(kTileThreads) void tile_step_kernel(const S* __restrict__ src,
                                                                 S* __restrict__ dst,
                                                                 const S* __restrict__ med,
                                                                 Geo G, Phys<R> P,
                                                                 int tiles_x) {
    extern __shared__ __align__(16) unsigned char tile_lds[];
    S* const buf0 = reinterpret_cast<S*>(tile_lds);
    S* const buf1 = buf0 + kPlanes * kTilePlane;
    S* const mlds = buf1 + kPlanes * kTilePlane;   // phi, K (per-node medium only)
    constexpr int W = kTileRegion;
    static_assert(TS + 2 * K + 1 <= kTileRegion, "region larger than the LDS planes");

    const int tx = blockIdx.x % tiles_x, ty = blockIdx.x / tiles_x;
    const int x0 = tx * TS, y0 = ty * TS;
    const int x1 = min(x0 + TS, G.nx), y1 = min(y0 + TS, G.ny);
    // a tile one node thick at the east (north) wall has its wall nodes' inward neighbours one
    // node west (south) of it: one more halo node on that side
    const int hW = K + ((x1 - x0 == 1 && G.wallE) ? 1 : 0);
    const int hS = K + ((y1 - y0 == 1 && G.wallN) ? 1 : 0);
    int rx0 = x0 - hW, rx1 = x1 + K, ry0 = y0 - hS, ry1 = y1 + K;
    bool openW = true, openE = true, openS = true, openN = true;
    if (G.wallW && rx0 <= 0) { rx0 = 0; openW = false; }
    if (G.wallE && rx1 >= G.nx) { rx1 = G.nx; openE = false; }
    if (G.wallS && ry0 <= 0) { ry0 = 0; openS = false; }
    if (G.wallN && ry1 >= G.ny) { ry1 = G.ny; openN = false; }
    const int RW = rx1 - rx0, RH = ry1 - ry0;   // at most kTileRegion each

    // one work-item per region node (the region has at most kTileThreads nodes); its place,
    // wall sides and the last step it can take are fixed for the launch
    const int i = threadIdx.x;
    const bool mine = i < RW * RH;
    const int ly = mine ? i / RW : 0, lx = mine ? i - ly * RW : 0;
    const int gx = tile_wrap(rx0 + lx, G.nx, !G.wallW), gy = tile_wrap(ry0 + ly, G.ny, !G.wallS);
    const bool onW = G.wallW && gx == 0, onE = G.wallE && gx == G.nx - 1;
    const bool onS = G.wallS && gy == 0, onN = G.wallN && gy == G.ny - 1;
    const bool wall = onW || onE || onS || onN;
    // the node whose pulled populations this node uses: itself, or its inward neighbour
    const int lxf = lx + (onW ? 1 : 0) - (onE ? 1 : 0);
    const int lyf = ly + (onS ? 1 : 0) - (onN ? 1 : 0);
    int last = mine ? K : 0;
    if (openW) last = min(last, lxf);
    if (openE) last = min(last, RW - 1 - lxf);
    if (openS) last = min(last, lyf);
    if (openN) last = min(last, RH - 1 - lyf);
    const int c = ly * W + lx;

    // load the region: the post-collision state and the medium
    if (mine) {
        const size_t o = size_t(gy) * size_t(G.pitch) + size_t(gx);
#pragma unroll
        for (int p = 0; p < kPlanes; ++p) buf0[p * kTilePlane + c] = src[size_t(p) * G.plane + o];
        if constexpr (PN) {
            mlds[c] = med[o];
            mlds[kTilePlane + c] = med[size_t(G.plane) + o];
        }
    }
    __syncthreads();

    const S* cur = buf0;
    S* nxt = buf1;
    for (int s = 1; s <= K; ++s) {
        if (s <= last) {
            // node_state's arithmetic on the region, then collide, as step_kernel does
            R f[9], g[5];
            Mac<R> m;
            Med<R> md;
            tile_pull<R, S>(cur, lxf, lyf, f, g);
            if (!wall) {
                md = tile_medium<R, PN, S>(mlds, lx, ly, P);
                m = fluid_macros<R>(f, g, md, P);
            } else {
                const Med<R> mdf = tile_medium<R, PN, S>(mlds, lxf, lyf, P);
                const Mac<R> mf = fluid_macros<R>(f, g, mdf, P);
                md = tile_medium<R, PN, S>(mlds, lx, ly, P);
                m = wall_state<R>(onW, onE, onS, onN, f, g, mf, mdf, md, P);
            }
            collide<R>(f, g, m, md, P);
#pragma unroll
            for (int p = 0; p < 9; ++p) nxt[p * kTilePlane + c] = S(f[p]);
#pragma unroll
            for (int p = 0; p < 5; ++p) nxt[(9 + p) * kTilePlane + c] = S(g[p]);
        }
        __syncthreads();
        const S* t = cur;
        cur = nxt;
        nxt = const_cast<S*>(t);
    }

    // write the tile back
    const int ox = rx0 + lx, oy = ry0 + ly;   // unwrapped: the tile lies inside the grid
    if (mine && ox >= x0 && ox < x1 && oy >= y0 && oy < y1) {
        const size_t o = size_t(oy) * size_t(G.pitch) + size_t(ox);
#pragma unroll
        for (int p = 0; p < kPlanes; ++p) dst[size_t(p) * G.plane + o] = cur[p * kTilePlane + c];
    }
}

template <typename S, bool PN>
constexpr size_t tile_lds_bytes() {
    return (2 * kPlanes + (PN ? 2 : 0)) * size_t(kTilePlane) * sizeof(S);
}

// The tile form that beats one step per launch (and the two-step kernel, which the default
// tries first), if any.  Measured on porous cavities (per-node medium / uniform medium), MLUPS
// of 16 x 16 tiles advanced four steps over the best other form:
//   FP32                        64^2 1.09 / 1.19, 128^2 1.36 / 1.49, 256^2 1.47 / 1.54,
//                               512^2 1.12 / 1.00, 1024^2 0.97 / 0.90
//   FP64                        64^2 0.91 / 1.14, 128^2 1.18 / 1.44, 256^2 1.31 / 1.50,
//                               512^2 0.99 / 1.17, 1024^2 0.84 / 0.87
//   FP32 storage, FP64 arith.   64^2 0.93 / 1.17, 128^2 1.12 / 1.35, 256^2 1.28 / 1.41,
//                               512^2 0.64 / 0.73
// On larger grids the halo's redundant work (2.25x the tile's nodes for the first step) costs
// more than the launches it saves.  On the smallest grids 8 x 8 tiles advanced eight steps pay
// the launch cost half as often and keep four times as many work-groups busy, at up to 9x
// redundant work in the first step.  MLUPS of the 8 x 8 form over the 16 x 16 one (uniform /
// per-node medium):
//   FP32                        48^2 1.12 / 1.08, 64^2 1.36 / 1.34, 96^2 1.35 / 1.31,
//                               128^2 1.17 / 1.17, 160^2 0.95 / 0.92
//   FP64                        48^2 1.09 / 1.05, 64^2 1.22 / 1.25, 96^2 1.21 / 1.24,
//                               128^2 1.15 / 1.15, 160^2 0.79 / 0.75
//   FP32 storage, FP64 arith.   48^2 1.04 / 1.00, 64^2 1.19 / 1.20, 96^2 1.19 / 1.20,
//                               128^2 1.10 / 1.11, 160^2 0.72 / 0.71
// With FP64 arithmetic and a per-node medium below 64^2 neither form beats one step per launch.
constexpr long long kTinyTileMaxNodes = 128LL * 128;

template <typename S, typename R>
int tile_steps(const Geo& G, bool per_node_medium) {
    const long long n = (long long)G.nx * G.ny;
    if (n <= kTinyTileMaxNodes)
        return sizeof(R) == 4 || !per_node_medium || n >= 64LL * 64 ? kTinyTileSteps : 0;
    bool pays;
    if (sizeof(R) == 4)
        pays = n <= 512LL * 512;
    else if (!per_node_medium)
        pays = n <= (sizeof(S) == 8 ? 512LL * 512 : 256LL * 256);
    else
        pays = n >= 128LL * 128 && n <= 256LL * 256;
    return pays ? kTileSteps : 0;
}

template <typename S, typename R, int TS, int K>
hipError_t launch_tiles(const void* src, void* dst, const void* med, const Geo& G,
                        const Phys<R>& P, hipStream_t s) {
    const int tiles_x = (G.nx + TS - 1) / TS;
    const int nwg = tiles_x * ((G.ny + TS - 1) / TS);
    if (med) {
        constexpr size_t lds = tile_lds_bytes<S, true>();
        static_assert(lds <= 160 * 1024, "tile region exceeds the LDS of a CU");
        static_assert(kTilePlane <= kTileThreads, "one work-item per region node");
        tile_step_kernel<S, R, true, TS, K><<<nwg, kTileThreads, lds, s>>>(
            (const S*)src, (S*)dst, (const S*)med, G, P, tiles_x);
    } else {
        constexpr size_t lds = tile_lds_bytes<S, false>();
        tile_step_kernel<S, R, false, TS, K><<<nwg, kTileThreads, lds, s>>>(
            (const S*)src, (S*)dst, nullptr, G, P, tiles_x);
    }
    return hipGetLastError();
}

template <typename S, typename R>
hipError_t launch_tile_step(const void* src, void* dst, const void* med, const Geo& G,
                            const Phys<R>& P, int k, hipStream_t s) {
    if (k == kTinyTileSteps)
        return launch_tiles<S, R, kTinyTileSide, kTinyTileSteps>(src, dst, med, G, P, s);
    if (k == kTileSteps) return launch_tiles<S, R, kTileSide, kTileSteps>(src, dst, med, G, P, s);
    return hipErrorInvalidValue;
}

#define LBM_TILE_INST(S, R)                                                                    \
    template int tile_steps<S, R>(const Geo&, bool);                                           \
    template hipError_t launch_tile_step<S, R>(const void*, void*, const void*, const Geo&,    \
                                               const Phys<R>&, int, hipStream_t);
LBM_TILE_INST(float, float)
LBM_TILE_INST(double, double)
LBM_TILE_INST(float, double)
#undef LBM_TILE_INST

}  // namespace lbm
