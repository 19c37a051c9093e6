// lbm_batch.hip -- one launch steps many independent cavities of uneven size and parameters.
//
// The cavities' states sit back to back in two population buffers.  The tiles of all cavities
// form one queue (cavity by cavity, tile row by tile row).  A tile -> cavity table and
// per-cavity geometry / parameter tables (read through the scalar cache: every work-item of a
// tile belongs to the same cavity) give each tile its setting.
// The per-node arithmetic is the plain step's (uniform medium per cavity), so every cavity's
// result is bitwise that of its own plain run.
#include "lbm_device.hpp"
#include "lbm_internal.hpp"
#include "lbm_tb2.hpp"

namespace lbm {

// Tile = 64 * NPT consecutive nodes along x (one wavefront per 64) times TH rows (one
// wavefront per row), so narrow cavities still fill every wavefront.  CHUNKED: each
// work-group walks one contiguous run of the tile queue (consecutive tiles mostly share a
// cavity, so its parameters stay in the scalar cache); otherwise one tile per work-group.
// S: storage type, R: arithmetic type.
template <typename S, typename R, int TH, int NPT, bool CHUNKED>
__global__ __launch_bounds__(64 * TH) void batch_step_kernel(const S* __restrict__ src,
                                                             S* __restrict__ dst,
                                                             const BatchCavity* __restrict__ cav,
                                                             const Phys<R>* __restrict__ phys,
                                                             const int* __restrict__ tile_cav,
                                                             int ntiles) {
    int t0, t1;
    if constexpr (CHUNKED) {
        t0 = int((long long)ntiles * blockIdx.x / gridDim.x);
        t1 = int((long long)ntiles * (blockIdx.x + 1) / gridDim.x);
    } else {
        t0 = blockIdx.x;
        t1 = t0 + 1;
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int t = t0; t < t1; ++t) {
        const int c = tile_cav[t];
        const BatchCavity C = cav[c];
        const Phys<R> P = phys[c];
        const int lt = t - C.tile0;
        const int ty = lt / C.tiles_x;
        const int y = ty * TH + wave;
        if (y >= C.G.ny) continue;
        const int x0 = (lt - ty * C.tiles_x) * (64 * NPT) + lane;
        const S* s = src + C.off;
        S* d = dst + C.off;
#pragma unroll
        for (int k = 0; k < NPT; ++k) {
            const int x = x0 + k * 64;
            if (x < C.G.nx) {
                R f[9], g[5];
                Mac<R> m;
                Med<R> md;
                node_state<R, false, S>(s, nullptr, C.G, P, x, y, f, g, m, md);
                collide<R>(f, g, m, md, P);
                const unsigned o =
                    (unsigned(y) * unsigned(C.G.pitch) + unsigned(x)) * unsigned(sizeof(S));
#pragma unroll
                for (int i = 0; i < 9; ++i)
                    __builtin_nontemporal_store(S(f[i]), &at(plane(d, i, C.G.plane), o));
#pragma unroll
                for (int i = 0; i < 5; ++i)
                    __builtin_nontemporal_store(S(g[i]), &at(plane(d, 9 + i, C.G.plane), o));
            }
        }
    }
}

template <typename S, typename R, int TH, int NPT>
static hipError_t launch_v(const void* src, void* dst, const BatchTable<R>& T, int nwg,
                           hipStream_t s) {
    if (nwg >= T.ntiles)
        batch_step_kernel<S, R, TH, NPT, false><<<T.ntiles, 64 * TH, 0, s>>>(
            (const S*)src, (S*)dst, T.cav, T.phys, T.tile_cav, T.ntiles);
    else
        batch_step_kernel<S, R, TH, NPT, true><<<nwg, 64 * TH, 0, s>>>(
            (const S*)src, (S*)dst, T.cav, T.phys, T.tile_cav, T.ntiles);
    return hipGetLastError();
}

// Supported tile shapes: rows per work-group (work-group = 64 * rows work-items) and 64-node
// segments per work-item along x; nwg >= ntiles launches one tile per work-group, fewer runs
// the chunked persistent form.
template <typename S, typename R>
hipError_t launch_batch_step(const void* src, void* dst, const BatchTable<R>& T, int nodes_x,
                             int rows, int nwg, hipStream_t s) {
    switch (rows * 8 + nodes_x) {
        case 1 * 8 + 1: return launch_v<S, R, 1, 1>(src, dst, T, nwg, s);
        case 1 * 8 + 2: return launch_v<S, R, 1, 2>(src, dst, T, nwg, s);
        case 1 * 8 + 4: return launch_v<S, R, 1, 4>(src, dst, T, nwg, s);
        case 2 * 8 + 1: return launch_v<S, R, 2, 1>(src, dst, T, nwg, s);
        case 2 * 8 + 2: return launch_v<S, R, 2, 2>(src, dst, T, nwg, s);
        case 2 * 8 + 4: return launch_v<S, R, 2, 4>(src, dst, T, nwg, s);
        case 4 * 8 + 1: return launch_v<S, R, 4, 1>(src, dst, T, nwg, s);
        case 4 * 8 + 2: return launch_v<S, R, 4, 2>(src, dst, T, nwg, s);
        case 4 * 8 + 4: return launch_v<S, R, 4, 4>(src, dst, T, nwg, s);
        case 8 * 8 + 1: return launch_v<S, R, 8, 1>(src, dst, T, nwg, s);
        default: return hipErrorInvalidValue;
    }
}

// Two steps per launch for every cavity (the single-cavity two-step kernel's work, uniform
// medium per cavity), TW strips (wavefronts) per work-group: narrow cavities leave fewer
// wavefronts idle with fewer strips per group.  The logical work-groups of all cavities form
// one list: wg_cav[w] is the cavity of logical work-group w, and for that cavity C.tile0 is its
// first logical work-group and C.tiles_x its number of strip groups.
template <typename S, typename R, int TW>
__global__ __launch_bounds__(64 * TW, (tb_min_waves<S, R>())) void batch_tb2_kernel(
    const S* __restrict__ src, S* __restrict__ dst, const BatchCavity* __restrict__ cav,
    const Phys<R>* __restrict__ phys, const int* __restrict__ wg_cav, int rows, int chunk) {
    const int wg = tb_logical_group(chunk);
    const int c = wg_cav[wg];
    const BatchCavity C = cav[c];
    const Phys<R> P = phys[c];
    const int lw = wg - C.tile0;
    const int nstrips = (C.G.nx + kTbCols - 1) / kTbCols;
    const int strip = (lw % C.tiles_x) * TW + (threadIdx.x >> 6), seg = lw / C.tiles_x;
    tb2_segment<S, R, false>(src + C.off, dst + C.off, (const S*)nullptr, C.G, P, strip,
                             strip < nstrips, seg, rows);
}

// Work-groups of batch_tb2_kernel<S, R, TW> one XCD holds at once (the XCD chunk of
// tb_logical_group); queried once, at the first call.
template <typename S, typename R, int TW>
static int batch_tb_chunk() {
    static const int chunk = [] {
        int dev = 0, cus = 0, per_cu = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) !=
                hipSuccess ||
            hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, batch_tb2_kernel<S, R, TW>,
                                                         64 * TW, 0) != hipSuccess)
            return 1;
        return max(1, cus * per_cu / 8);
    }();
    return chunk;
}

template <typename S, typename R>
void prepare_batch_tb2() {
    (void)batch_tb_chunk<S, R, 1>();
    (void)batch_tb_chunk<S, R, 2>();
    (void)batch_tb_chunk<S, R, 4>();
}

template <typename S, typename R>
hipError_t launch_batch_tb2(const void* src, void* dst, const BatchTable<R>& T, int rows,
                            int waves, hipStream_t s) {
    switch (waves) {
        case 1:
            batch_tb2_kernel<S, R, 1><<<T.ntiles, 64, 0, s>>>(
                (const S*)src, (S*)dst, T.cav, T.phys, T.tile_cav, rows,
                batch_tb_chunk<S, R, 1>());
            break;
        case 2:
            batch_tb2_kernel<S, R, 2><<<T.ntiles, 128, 0, s>>>(
                (const S*)src, (S*)dst, T.cav, T.phys, T.tile_cav, rows,
                batch_tb_chunk<S, R, 2>());
            break;
        case 4:
            batch_tb2_kernel<S, R, 4><<<T.ntiles, 256, 0, s>>>(
                (const S*)src, (S*)dst, T.cav, T.phys, T.tile_cav, rows,
                batch_tb_chunk<S, R, 4>());
            break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template hipError_t launch_batch_step<float, float>(const void*, void*, const BatchTable<float>&,
                                                    int, int, int, hipStream_t);
template hipError_t launch_batch_step<double, double>(const void*, void*,
                                                      const BatchTable<double>&, int, int, int,
                                                      hipStream_t);
template hipError_t launch_batch_step<float, double>(const void*, void*,
                                                     const BatchTable<double>&, int, int, int,
                                                     hipStream_t);
template void prepare_batch_tb2<float, float>();
template void prepare_batch_tb2<double, double>();
template void prepare_batch_tb2<float, double>();
template hipError_t launch_batch_tb2<float, float>(const void*, void*, const BatchTable<float>&,
                                                   int, int, hipStream_t);
template hipError_t launch_batch_tb2<double, double>(const void*, void*,
                                                     const BatchTable<double>&, int, int,
                                                     hipStream_t);
template hipError_t launch_batch_tb2<float, double>(const void*, void*,
                                                    const BatchTable<double>&, int, int,
                                                    hipStream_t);

}  // namespace lbm
