// lbm_kernels.hip -- single-cavity kernels: the time step (one step per launch, two steps per
// launch, and the in-place AA-layout forms), the observables pass, the wall Nusselt reduction,
// the stream function and state initialisation.
#include "lbm_device.hpp"
#include "lbm_internal.hpp"
#include "lbm_tb2.hpp"
#include "lbm_tb3.hpp"

namespace lbm {

// One time step for every node: pull (Eqs. (18), (35)) -> wall reconstruction -> macroscopic
// recovery (Eqs. (36), (22), (21), (23), (4)) -> collision (Eqs. (17), (34)) -> store.
// One work-item per node; a work-group covers kTileX consecutive nodes of one row.  S is the
// storage type, R the arithmetic type.
template <typename S, typename R, bool PN>
__global__ __launch_bounds__(kTileX) void step_kernel(const S* __restrict__ src,
                                                      S* __restrict__ dst,
                                                      const S* __restrict__ med, Geo G,
                                                      Phys<R> P, int tiles_x) {
    // Work-groups in launch order walk the lattice row by row.  (Dealing each XCD one
    // contiguous band of rows instead was measured 7% slower: it concentrates each XCD's
    // stream on one address range.)
    const int t = blockIdx.x;
    const int y = t / tiles_x;
    const int x = (t - y * tiles_x) * kTileX + threadIdx.x;
    if (x >= G.nx) return;
    R f[9], g[5];
    Mac<R> m;
    Med<R> md;
    node_state<R, PN, S>(src, med, G, P, x, y, f, g, m, md);
    collide<R>(f, g, m, md, P);
    const unsigned o = (unsigned(y) * unsigned(G.pitch) + unsigned(x)) * unsigned(sizeof(S));
#pragma unroll
    for (int i = 0; i < 9; ++i)
        __builtin_nontemporal_store(S(f[i]), &at(plane(dst, i, G.plane), o));
#pragma unroll
    for (int i = 0; i < 5; ++i)
        __builtin_nontemporal_store(S(g[i]), &at(plane(dst, 9 + i, G.plane), o));
}

// One AA-pattern time step in place (layout L = kAAOpp or kAAOwn read, the other written).
// The per-node arithmetic is step_kernel's.  A wall node is stepped by the thread of its inward
// neighbour, which already holds the populations the reconstruction needs: a wall thread reading
// them itself could see the neighbour's new values.  The thread of node x writes only slots that
// it alone read (its own and those of the wall nodes it steps), so the step is race-free.
template <typename S, typename R, bool PN, int L>
__global__ __launch_bounds__(kTileX) void aa_step_kernel(S* __restrict__ buf,
                                                         const S* __restrict__ med, Geo G,
                                                         Phys<R> P, int tiles_x) {
    const int t = blockIdx.x;
    const int y = t / tiles_x;
    const int x = (t - y * tiles_x) * kTileX + threadIdx.x;
    if (x >= G.nx) return;
    if ((G.wallW && x == 0) || (G.wallE && x == G.nx - 1) || (G.wallS && y == 0) ||
        (G.wallN && y == G.ny - 1))
        return;
    R f[9], g[5];
    pull<R, S, L>(buf, G, x, y, f, g);
    const Med<R> md = load_medium<R, PN, S>(med, y * G.pitch + x, G.plane, P);
    const Mac<R> m = fluid_macros<R>(f, g, md, P);
    step_wall_neighbours<R, PN, S>(med, G, P, x, y, f, g, m, md,
                                   [&](int xb, int yb, const R* fb, const R* gb) {
                                       aa_store<S, R, L>(buf, G, xb, yb, fb, gb);
                                   });
    collide<R>(f, g, m, md, P);
    aa_store<S, R, L>(buf, G, x, y, f, g);
}

template <typename S, typename R, bool PN, int NDESC>
__global__ __launch_bounds__(64 * kTbWaves, (tb_min_waves<S, R>())) void tb2_step_kernel(const S* __restrict__ src,
                                                                 S* __restrict__ dst,
                                                                 const S* __restrict__ med,
                                                                 Geo G, Phys<R> P, int nstrips,
                                                                 int rows, int chunk) {
    // A work-group holds kTbWaves adjacent strips of one row segment, kept in step by a
    // barrier per row, so that the cache lines the neighbouring strips share are used while
    // resident.
    const int wg = tb_logical_group(chunk);
    const int ngrp = (nstrips + kTbWaves - 1) / kTbWaves;
    const int strip = (wg % ngrp) * kTbWaves + (threadIdx.x >> 6), seg = wg / ngrp;
    tb2_segment<S, R, PN, NDESC>(src, dst, med, G, P, strip, strip < nstrips, seg, rows);
}

// Three steps per launch (FP32): a work-group holds kTb3Waves adjacent strips of one row
// segment, each with its own ring of step n+2 rows in LDS, kept in step by a barrier per row.
// Segments alternate their sweep direction, except that the segment at a south wall sweeps
// forwards and the one at a north wall backwards.  The nseg segments split the rows evenly: the
// first `extra` have rows + 1 rows, the others rows, so that no work-group runs long.
template <typename S, typename R, bool PN>
__global__ __launch_bounds__(64 * kTb3Waves, 3) void tb3_step_kernel(const S* __restrict__ src,
                                                                   S* __restrict__ dst,
                                                                   const S* __restrict__ med,
                                                                   Geo G, Phys<R> P, int nstrips,
                                                                   int rows, int extra, int nseg,
                                                                   int chunk) {
    __shared__ S ring[kTb3Waves * kTb3Ring];
    const int wg = tb_logical_group(chunk);
    const int ngrp = (nstrips + kTb3Waves - 1) / kTb3Waves;
    const int w = int(threadIdx.x) >> 6;
    const int strip = (wg % ngrp) * kTb3Waves + w, seg = wg / ngrp;
    const int ylo = seg * rows + min(seg, extra);
    const int yhi = ylo + rows + (seg < extra ? 1 : 0);
    const bool rev = (G.wallN && seg == nseg - 1) || (!(G.wallS && seg == 0) && (seg & 1));
    S* const my = ring + w * kTb3Ring;
    // The relaxation constants from LDS: held in scalar registers across the row loop they
    // overflow the scalar register file, and reloading spilled ones costs a vector instruction
    // each (v_readlane), some 80 per row; from LDS they live in vector registers (1.6 % faster).
    __shared__ Phys<R> sP;
    if (threadIdx.x == 0) sP = P;
    __syncthreads();
    if (rev)
        tb3_sweep<S, R, PN, true>(src, dst, med, G, sP, strip, strip < nstrips, ylo, yhi, my);
    else
        tb3_sweep<S, R, PN, false>(src, dst, med, G, sP, strip, strip < nstrips, ylo, yhi, my);
}

// Maximum and minimum that propagate a NaN (fmax and fmin would drop it), so that a
// non-finite value always reaches the result of a reduction.
__device__ __forceinline__ double obs_max(double a, double b) {
    return (a >= b || a != a) ? a : b;
}
__device__ __forceinline__ double obs_min(double a, double b) {
    return (a <= b || a != a) ? a : b;
}

// Wave-level reductions over the 64 lanes of a wavefront.
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    return v;
}
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = obs_max(v, __shfl_down(v, off, 64));
    return v;
}
__device__ __forceinline__ double wave_min(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = obs_min(v, __shfl_down(v, off, 64));
    return v;
}

// Macroscopic fields at the current time level, plus kObsParts partial results per
// work-group b at part[kObsParts * b + k]: k = 0 max |u|, 1 the sum of stored f' (mass
// deviation), 2 a flag (1 when u, p, T or |v| of Eq. (22) is not finite), 3 min T, 4 max T,
// 5 max |phi p - rho0 cs^2|.  Grid-stride over nodes.
template <typename S, typename R, bool PN, int L>
__global__ __launch_bounds__(256) void observe_kernel(const S* __restrict__ src,
                                                      const S* __restrict__ med, Geo G,
                                                      Phys<R> P, S* __restrict__ ux_out,
                                                      S* __restrict__ uy_out,
                                                      S* __restrict__ p_out,
                                                      S* __restrict__ T_out,
                                                      double* __restrict__ part) {
    const int n = G.nx * G.ny;
    double v[kObsParts] = {0.0, 0.0, 0.0, INFINITY, -INFINITY, 0.0};
    for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < n; k += gridDim.x * blockDim.x) {
        const int y = k / G.nx, x = k - y * G.nx;
        R f[9], g[5];
        Mac<R> m;
        Med<R> md;
        node_state<R, PN, S, L>(src, med, G, P, x, y, f, g, m, md);
        // the pressure of Eq. (23) less its rest value rho0 cs^2 / phi: FP32 could not hold
        // the dynamic part, often below 1e-3 of p, on top of that background
        const R p = m.P * md.inv_phi;
        const R T = P.T0 + m.theta;
        if (ux_out) ux_out[k] = S(m.ux);
        if (uy_out) uy_out[k] = S(m.uy);
        if (p_out) p_out[k] = S(p);
        if (T_out) T_out[k] = S(T);
        const double sp = sqrt(double(m.ux) * double(m.ux) + double(m.uy) * double(m.uy));
        const double Td = double(T), Pd = fabs(double(m.P));
        v[0] = obs_max(v[0], sp);
        if (!isfinite(sp) || !isfinite(double(p)) || !isfinite(Td) || !isfinite(double(m.vv)))
            v[2] = 1.0;
        v[3] = obs_min(v[3], Td);
        v[4] = obs_max(v[4], Td);
        v[5] = obs_max(v[5], Pd);
        const int o = y * G.pitch + x;
        double s = 0.0;
#pragma unroll
        for (int i = 0; i < 9; ++i) s += double(src[i * G.plane + o]);
        v[1] += s;
    }
    __shared__ double red[kObsParts][4];
    v[0] = wave_max(v[0]);
    v[1] = wave_sum(v[1]);
    v[2] = wave_max(v[2]);
    v[3] = wave_min(v[3]);
    v[4] = wave_max(v[4]);
    v[5] = wave_max(v[5]);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) {
#pragma unroll
        for (int k = 0; k < kObsParts; ++k) red[k][w] = v[k];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double r[kObsParts];
#pragma unroll
        for (int k = 0; k < kObsParts; ++k) r[k] = red[k][0];
        for (int i = 1; i < (int)(blockDim.x >> 6); ++i) {
            r[0] = obs_max(r[0], red[0][i]);
            r[1] += red[1][i];
            r[2] = obs_max(r[2], red[2][i]);
            r[3] = obs_min(r[3], red[3][i]);
            r[4] = obs_max(r[4], red[4][i]);
            r[5] = obs_max(r[5], red[5][i]);
        }
#pragma unroll
        for (int k = 0; k < kObsParts; ++k) part[kObsParts * blockIdx.x + k] = r[k];
    }
}

// Temperature deviation theta = T - T0 at (x, y) after streaming and wall reconstruction.
template <typename S, typename R, int L>
__device__ __forceinline__ double node_theta(const S* __restrict__ src, const Geo& G,
                                             const Phys<R>& P, int x, int y) {
    const bool onW = G.wallW && x == 0;
    const bool onE = G.wallE && x == G.nx - 1;
    const bool onS = G.wallS && y == 0;
    const bool onN = G.wallN && y == G.ny - 1;
    const int xf = x + (onW ? 1 : 0) - (onE ? 1 : 0);
    const int yf = y + (onS ? 1 : 0) - (onN ? 1 : 0);
    R f[9], g[5];
    pull<R, S, L>(src, G, xf, yf, f, g);
    const R th = ((g[0] + g[1]) + (g[2] + g[3]) + g[4]) + P.hQs;
    if (!(onW || onE || onS || onN)) return double(th);
    return double(wall_theta<R>(onW, onE, onS, onN, th, P));
}

// Eq. (38): Nu(y) = -L dT/dx / dT at the west (hot) and east (cold) walls with the
// fourth-order one-sided five-point derivative, averaged by the trapezoid rule over the
// ny wall nodes; part = the partial results of observe_kernel (nparts work-groups).
// One work-group; writes out[0] nu_hot, out[1] nu_cold, then out[2 + k] the reduction of
// partial result k: max |u|, sum f', non-finite flag, min T, max T, max |phi p - rho0 cs^2|.
template <typename S, typename R, int L>
__global__ __launch_bounds__(256) void nusselt_kernel(const S* __restrict__ src, Geo G,
                                                      Phys<R> P, double L_over_dT,
                                                      const double* __restrict__ part,
                                                      int nparts, double* __restrict__ out) {
    double h = 0.0, c = 0.0;
    if (G.nx >= 5) {
        for (int y = threadIdx.x; y < G.ny; y += blockDim.x) {
            double Th[5], Tc[5];
#pragma unroll
            for (int k = 0; k < 5; ++k) {
                Th[k] = node_theta<S, R, L>(src, G, P, k, y);
                Tc[k] = node_theta<S, R, L>(src, G, P, G.nx - 1 - k, y);
            }
            const double dh = (-25.0 * Th[0] + 48.0 * Th[1] - 36.0 * Th[2] + 16.0 * Th[3] -
                               3.0 * Th[4]) / 12.0;
            const double dc = (25.0 * Tc[0] - 48.0 * Tc[1] + 36.0 * Tc[2] - 16.0 * Tc[3] +
                               3.0 * Tc[4]) / 12.0;
            const double w = (y == 0 || y == G.ny - 1) ? 0.5 : 1.0;
            h += w * dh;
            c += w * dc;
        }
    }
    __shared__ double red[2][4];
    h = wave_sum(h);
    c = wave_sum(c);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (lane == 0) {
        red[0][wv] = h;
        red[1][wv] = c;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double sh = 0.0, sc = 0.0;
        for (int i = 0; i < (int)(blockDim.x >> 6); ++i) {
            sh += red[0][i];
            sc += red[1][i];
        }
        const double scale = -L_over_dT / double(G.ny - 1);
        out[0] = scale * sh;
        out[1] = scale * sc;
        double r[kObsParts];
#pragma unroll
        for (int k = 0; k < kObsParts; ++k) r[k] = part[k];
        for (int i = 1; i < nparts; ++i) {
            const double* q = part + kObsParts * i;
            r[0] = obs_max(r[0], q[0]);
            r[1] += q[1];
            r[2] = obs_max(r[2], q[2]);
            r[3] = obs_min(r[3], q[3]);
            r[4] = obs_max(r[4], q[4]);
            r[5] = obs_max(r[5], q[5]);
        }
#pragma unroll
        for (int k = 0; k < kObsParts; ++k) out[2 + k] = r[k];
    }
}

// Stream function: one work-item per column x integrates u_x (Eq. (21)) along y with the
// trapezoid rule, psi(x, 0) = 0.
template <typename S, typename R, bool PN, int L>
__global__ void stream_function_kernel(const S* __restrict__ src, const S* __restrict__ med,
                                       Geo G, Phys<R> P, S* __restrict__ psi) {
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= G.nx) return;
    double acc = 0.0, prev = 0.0;
    for (int y = 0; y < G.ny; ++y) {
        R f[9], g[5];
        Mac<R> m;
        Med<R> md;
        node_state<R, PN, S, L>(src, med, G, P, x, y, f, g, m, md);
        const double u = double(m.ux);
        if (y > 0) acc += 0.5 * (prev + u);
        prev = u;
        psi[y * G.nx + x] = S(acc);
    }
}

// Rest state (u = 0, phi p = rho0 cs^2, T = T_init) as deviations: f' = 0, g' = wt (T_init - T0).
template <typename R>
__global__ void rest_kernel(R* __restrict__ dst, Geo G, R g0, R g1) {
    const int n = G.plane;
    for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < n; k += gridDim.x * blockDim.x) {
#pragma unroll
        for (int i = 0; i < 9; ++i) dst[i * n + k] = R(0);
        dst[9 * n + k] = g0;
#pragma unroll
        for (int i = 1; i < 5; ++i) dst[(9 + i) * n + k] = g1;
    }
}

// Pitched copy of a dense [ny][nx] field into a [ny][pitch] plane; a NULL source fills v.
template <typename R>
__global__ void pitch_copy_kernel(R* __restrict__ dst, const R* __restrict__ src, Geo G, R v) {
    const int n = G.nx * G.ny;
    for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < n; k += gridDim.x * blockDim.x) {
        const int y = k / G.nx, x = k - y * G.nx;
        dst[y * G.pitch + x] = src ? src[k] : v;
    }
}

// ---- launchers --------------------------------------------------------------------------------

template <typename S, typename R>
hipError_t launch_step(const void* src, void* dst, const void* med, const Geo& G,
                       const Phys<R>& P, hipStream_t s) {
    const int tiles_x = (G.nx + kTileX - 1) / kTileX;
    const int nwg = tiles_x * G.ny;
    if (med)
        step_kernel<S, R, true><<<nwg, kTileX, 0, s>>>((const S*)src, (S*)dst, (const S*)med, G,
                                                       P, tiles_x);
    else
        step_kernel<S, R, false><<<nwg, kTileX, 0, s>>>((const S*)src, (S*)dst, nullptr, G, P,
                                                        tiles_x);
    return hipGetLastError();
}


// Work-groups of the two-step kernel resident on the device at once (0 if unknown).
template <typename S, typename R, bool PN>
int tb_resident_groups() {
    static const int n = [] {
        int dev = 0, cus = 0, per_cu = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) !=
                hipSuccess ||
            hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, tb2_step_kernel<S, R, PN, 1>,
                                                         64 * kTbWaves, 0) != hipSuccess)
            return 0;
        return cus * per_cu;
    }();
    return n;
}

// Rows per segment of the two-step kernel.  Each segment reads the intermediate step's two
// halo rows and one row past its end on top of its own rows; neighbouring segments, which sweep
// towards each other, find some of those rows in L2.  Longer segments fetch less but live
// longer, and the launch's tail, in which the last work-groups finish on a partly idle device,
// grows with them.  Measured on the 4096^2 workload (FP32, MLUPS; fetched bytes over one read
// of the 16 planes): 5 rows 70.6k, 6 rows (12 rounds of the resident set) 71.6k and 1.36x,
// 11 rows 1.29x, 17 rows 1.24x, 23 rows (3 rounds) 65.2k and 1.21x, 35 rows 1.17x, 69 rows
// (one round) 1.12x.  (Work-groups of 8 strips instead of 4 measured the same in FP32 and 5 %
// slower in FP64, 16 strips 5 % slower; a work-group of two vertically adjacent segments, 8
// wavefronts, fetched and ran the same as two work-groups of one.)
int tb_rows(const Geo& G, int nstrips, int resident) {
    const int ngrp = (nstrips + kTbWaves - 1) / kTbWaves;
    const int nseg = resident > 0 ? max(1, kTbRounds * resident / ngrp) : 1;
    return max(kTbMinRows, (G.ny + nseg - 1) / nseg);
}

template <typename S, typename R>
int tb_resident(bool per_node_medium) {
    return per_node_medium ? tb_resident_groups<S, R, true>()
                           : tb_resident_groups<S, R, false>();
}

// Work-groups of the three-step kernel resident on the device at once (0 if unknown).
template <typename S, typename R, bool PN>
int tb3_resident_groups() {
    static const int n = [] {
        int dev = 0, cus = 0, per_cu = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) !=
                hipSuccess ||
            hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, tb3_step_kernel<S, R, PN>,
                                                         64 * kTb3Waves, 0) != hipSuccess)
            return 0;
        return cus * per_cu;
    }();
    return n;
}

template <typename S, typename R>
int tb3_resident(bool per_node_medium) {
    return per_node_medium ? tb3_resident_groups<S, R, true>()
                           : tb3_resident_groups<S, R, false>();
}

// Rows per segment of the three-step kernel (the least height: the segments split the rows
// evenly, so some take one more), segments and work-groups per launch.  On a walled y axis there
// are at least two segments, so that each walled end is where a segment's sweep starts.  A
// segment recomputes two rows of step n+1 and one of step n+2 beyond each end, so it is at least
// kTb3MinRows high; measured on the 4096^2 FP32 cavity, 16 rows (six rounds of the resident set)
// beat 8 and 32 by 6 %, and on 2048^2, 8 rows beat 4 by 7 %.
constexpr int kTb3Rounds = 6;
constexpr int kTb3MinRows = 8;
void tb3_shape_rows(const Geo& G, int resident, int* rows, int* nseg, int* nwg) {
    const int nstrips = (G.nx + kTb3Cols - 1) / kTb3Cols;
    const int ngrp = (nstrips + kTb3Waves - 1) / kTb3Waves;
    const int want = resident > 0 ? max(1, kTb3Rounds * resident / ngrp) : 1;
    const int r = max(kTb3MinRows, (G.ny + want - 1) / want);
    int n = max(1, G.ny / r);
    if (G.wallS && n < 2) n = 2;
    *rows = G.ny / n;
    *nseg = n;
    *nwg = ngrp * n;
}

// Queries the resident set of the two-step kernel once, outside any graph capture.
template <typename S, typename R>
void prepare_tb2() {
    (void)tb_resident<S, R>(true);
    (void)tb_resident<S, R>(false);
    if constexpr (std::is_same<S, float>::value && std::is_same<R, float>::value) {
        (void)tb3_resident<S, R>(true);
        (void)tb3_resident<S, R>(false);
    }
}

// Whether two steps per launch beat one.  Measured (fused / single MLUPS, per-node medium):
//   FP32           4096^2 1.38, 2048^2 1.26, 1024^2 1.17, 512^2 0.52, 256^2 0.34
//   FP64           4096^2 1.53, 2048^2 1.31, 1024^2 1.19, 512^2 0.58
//   FP32 storage,  4096^2 1.04, 2048^2 0.83, 1024^2 0.64 (225 registers, 2 waves per SIMD)
//   FP64 arithmetic
// On small grids the few long row loops are latency-bound.  With equal types the kernel fuses
// when its work-groups at 16-row segments number at least a quarter of the resident set, with
// FP64 arithmetic on FP32 storage when they number eight times the resident set; and only for
// a state whose halves (7 planes) are below 2 GiB, which two buffer descriptors address.
template <typename S, typename R>
bool tb2_pays(const Geo& G, bool per_node_medium) {
    if (!tb2_fits(G, sizeof(S))) return false;
    const int resident = tb_resident<S, R>(per_node_medium);
    const int nstrips = (G.nx + kTbCols - 1) / kTbCols;
    const long long groups =
        (long long)((nstrips + kTbWaves - 1) / kTbWaves) * ((G.ny + 15) / 16);
    if (resident <= 0) return false;
    return std::is_same<S, R>::value ? 4 * groups >= resident : groups >= 8LL * resident;
}

// Whether three steps per launch beat two (FP32 storage and arithmetic, a state below 2 GiB).
// Measured (three / two steps per launch, FP32; per-node and uniform medium alike):
//   4096^2 1.20 (16-row segments), 2048^2 1.02 (8 rows), 1024^2 0.82
// (at 512^2 the tiles in LDS beat both).  It pays when segments of kTb3MinRows rows make at
// least three rounds of the resident set.
template <typename S, typename R>
bool tb3_pays(const Geo& G, bool per_node_medium) {
    if constexpr (std::is_same<S, float>::value && std::is_same<R, float>::value) {
        if (tb2_descs(G, sizeof(S)) != 1) return false;
        const int resident = tb3_resident<S, R>(per_node_medium);
        if (resident <= 0) return false;
        const long long ngrp = ((G.nx + kTb3Cols - 1) / kTb3Cols + kTb3Waves - 1) / kTb3Waves;
        return ngrp * (G.ny / kTb3MinRows) >= 3LL * resident;
    } else {
        (void)G, (void)per_node_medium;
        return false;
    }
}

template <typename S, typename R>
void tb2_shape(const Geo& G, bool per_node_medium, int* rows, int* nwg) {
    const int nstrips = (G.nx + kTbCols - 1) / kTbCols;
    *rows = tb_rows(G, nstrips, tb_resident<S, R>(per_node_medium));
    *nwg = (nstrips + kTbWaves - 1) / kTbWaves * ((G.ny + *rows - 1) / *rows);
}

template <typename S, typename R>
hipError_t launch_tb2_step(const void* src, void* dst, const void* med, const Geo& G,
                           const Phys<R>& P, hipStream_t s) {
    const int ndesc = tb2_descs(G, sizeof(S));
    if (ndesc == 0) return hipErrorInvalidValue;
    const int nstrips = (G.nx + kTbCols - 1) / kTbCols;
    int rows = 0, nwg = 0;
    tb2_shape<S, R>(G, med != nullptr, &rows, &nwg);
    // XCD chunks of one XCD's resident work-groups (the resident set over 8 XCDs)
    const int chunk = max(1, tb_resident<S, R>(med != nullptr) / 8);
    if (med && ndesc == 1)
        tb2_step_kernel<S, R, true, 1><<<nwg, 64 * kTbWaves, 0, s>>>(
            (const S*)src, (S*)dst, (const S*)med, G, P, nstrips, rows, chunk);
    else if (med)
        tb2_step_kernel<S, R, true, 2><<<nwg, 64 * kTbWaves, 0, s>>>(
            (const S*)src, (S*)dst, (const S*)med, G, P, nstrips, rows, chunk);
    else if (ndesc == 1)
        tb2_step_kernel<S, R, false, 1><<<nwg, 64 * kTbWaves, 0, s>>>(
            (const S*)src, (S*)dst, nullptr, G, P, nstrips, rows, chunk);
    else
        tb2_step_kernel<S, R, false, 2><<<nwg, 64 * kTbWaves, 0, s>>>(
            (const S*)src, (S*)dst, nullptr, G, P, nstrips, rows, chunk);
    return hipGetLastError();
}

template <typename S, typename R>
void tb3_shape(const Geo& G, bool per_node_medium, int* rows, int* nseg, int* nwg) {
    if constexpr (std::is_same<S, float>::value && std::is_same<R, float>::value)
        tb3_shape_rows(G, tb3_resident<S, R>(per_node_medium), rows, nseg, nwg);
    else
        *rows = *nseg = *nwg = 0;
}

template <typename S, typename R>
hipError_t launch_tb3_step(const void* src, void* dst, const void* med, const Geo& G,
                           const Phys<R>& P, hipStream_t s) {
    if constexpr (std::is_same<S, float>::value && std::is_same<R, float>::value) {
        if (tb2_descs(G, sizeof(S)) != 1) return hipErrorInvalidValue;
        const int nstrips = (G.nx + kTb3Cols - 1) / kTb3Cols;
        int rows = 0, nseg = 0, nwg = 0;
        tb3_shape<S, R>(G, med != nullptr, &rows, &nseg, &nwg);
        // every segment holds at least one row (its sweep loop runs until it passes the last),
        // and on a walled y axis two segments of at least two
        if (nseg < 1 || nseg > G.ny || (G.wallS && (nseg < 2 || rows < 2)))
            return hipErrorInvalidValue;
        const int extra = G.ny - rows * nseg;   // segments one row taller
        const int chunk = max(1, tb3_resident<S, R>(med != nullptr) / 8);
        if (med)
            tb3_step_kernel<S, R, true><<<nwg, 64 * kTb3Waves, 0, s>>>(
                (const S*)src, (S*)dst, (const S*)med, G, P, nstrips, rows, extra, nseg, chunk);
        else
            tb3_step_kernel<S, R, false><<<nwg, 64 * kTb3Waves, 0, s>>>(
                (const S*)src, (S*)dst, nullptr, G, P, nstrips, rows, extra, nseg, chunk);
        return hipGetLastError();
    } else {
        (void)src, (void)dst, (void)med, (void)G, (void)P, (void)s;
        return hipErrorInvalidValue;
    }
}

// parity 0: the state is in the kAAOpp form (even step count); 1: kAAOwn (odd)
template <typename S, typename R>
hipError_t launch_aa_step(void* buf, const void* med, const Geo& G, const Phys<R>& P,
                          int parity, hipStream_t s) {
    const int tiles_x = (G.nx + kTileX - 1) / kTileX;
    const int nwg = tiles_x * G.ny;
    S* b = (S*)buf;
    const S* m = (const S*)med;
    if (parity == 0) {
        if (med)
            aa_step_kernel<S, R, true, kAAOpp><<<nwg, kTileX, 0, s>>>(b, m, G, P, tiles_x);
        else
            aa_step_kernel<S, R, false, kAAOpp><<<nwg, kTileX, 0, s>>>(b, m, G, P, tiles_x);
    } else {
        if (med)
            aa_step_kernel<S, R, true, kAAOwn><<<nwg, kTileX, 0, s>>>(b, m, G, P, tiles_x);
        else
            aa_step_kernel<S, R, false, kAAOwn><<<nwg, kTileX, 0, s>>>(b, m, G, P, tiles_x);
    }
    return hipGetLastError();
}

template <typename S, typename R, int L>
static hipError_t observe_l(const void* src, const void* med, const Geo& G, const Phys<R>& P,
                            void* ux, void* uy, void* p, void* T, double* part, int nparts,
                            double L_over_dT, double* out, hipStream_t s) {
    if (med)
        observe_kernel<S, R, true, L><<<nparts, 256, 0, s>>>(
            (const S*)src, (const S*)med, G, P, (S*)ux, (S*)uy, (S*)p, (S*)T, part);
    else
        observe_kernel<S, R, false, L><<<nparts, 256, 0, s>>>(
            (const S*)src, nullptr, G, P, (S*)ux, (S*)uy, (S*)p, (S*)T, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    nusselt_kernel<S, R, L><<<1, 256, 0, s>>>((const S*)src, G, P, L_over_dT, part, nparts, out);
    return hipGetLastError();
}

// layout: kPull, kAAOpp or kAAOwn, the form the state is in
template <typename S, typename R>
hipError_t launch_observe(const void* src, const void* med, const Geo& G, const Phys<R>& P,
                          int layout, void* ux, void* uy, void* p, void* T, double* part,
                          int nparts, double L_over_dT, double* out, hipStream_t s) {
    switch (layout) {
        case kPull:
            return observe_l<S, R, kPull>(src, med, G, P, ux, uy, p, T, part, nparts, L_over_dT,
                                          out, s);
        case kAAOpp:
            return observe_l<S, R, kAAOpp>(src, med, G, P, ux, uy, p, T, part, nparts,
                                           L_over_dT, out, s);
        case kAAOwn:
            return observe_l<S, R, kAAOwn>(src, med, G, P, ux, uy, p, T, part, nparts,
                                           L_over_dT, out, s);
        default: return hipErrorInvalidValue;
    }
}

template <typename S, typename R, int L>
static hipError_t stream_function_l(const void* src, const void* med, const Geo& G,
                                    const Phys<R>& P, void* psi, hipStream_t s) {
    const int nb = (G.nx + 63) / 64;
    if (med)
        stream_function_kernel<S, R, true, L><<<nb, 64, 0, s>>>((const S*)src, (const S*)med, G,
                                                                P, (S*)psi);
    else
        stream_function_kernel<S, R, false, L><<<nb, 64, 0, s>>>((const S*)src, nullptr, G, P,
                                                                 (S*)psi);
    return hipGetLastError();
}

template <typename S, typename R>
hipError_t launch_stream_function(const void* src, const void* med, const Geo& G,
                                  const Phys<R>& P, int layout, void* psi, hipStream_t s) {
    switch (layout) {
        case kPull: return stream_function_l<S, R, kPull>(src, med, G, P, psi, s);
        case kAAOpp: return stream_function_l<S, R, kAAOpp>(src, med, G, P, psi, s);
        case kAAOwn: return stream_function_l<S, R, kAAOwn>(src, med, G, P, psi, s);
        default: return hipErrorInvalidValue;
    }
}

template <typename R>
hipError_t launch_rest(void* dst, const Geo& G, double g0, double g1, hipStream_t s) {
    rest_kernel<R><<<1024, 256, 0, s>>>((R*)dst, G, R(g0), R(g1));
    return hipGetLastError();
}

template <typename R>
hipError_t launch_pitch_copy(void* dst, const void* src, const Geo& G, double v, hipStream_t s) {
    pitch_copy_kernel<R><<<1024, 256, 0, s>>>((R*)dst, (const R*)src, G, R(v));
    return hipGetLastError();
}

#define LBM_INSTANCES(S, R)                                                                      \
    template hipError_t launch_step<S, R>(const void*, void*, const void*, const Geo&,           \
                                          const Phys<R>&, hipStream_t);                          \
    template hipError_t launch_aa_step<S, R>(void*, const void*, const Geo&, const Phys<R>&,     \
                                             int, hipStream_t);                                  \
    template hipError_t launch_tb2_step<S, R>(const void*, void*, const void*, const Geo&,       \
                                              const Phys<R>&, hipStream_t);                      \
    template void prepare_tb2<S, R>();                                                           \
    template bool tb2_pays<S, R>(const Geo&, bool);                                              \
    template void tb2_shape<S, R>(const Geo&, bool, int*, int*);                                 \
    template bool tb3_pays<S, R>(const Geo&, bool);                                              \
    template void tb3_shape<S, R>(const Geo&, bool, int*, int*, int*);                           \
    template hipError_t launch_tb3_step<S, R>(const void*, void*, const void*, const Geo&,       \
                                              const Phys<R>&, hipStream_t);                      \
    template hipError_t launch_observe<S, R>(const void*, const void*, const Geo&,               \
                                             const Phys<R>&, int, void*, void*, void*, void*,    \
                                             double*, int, double, double*, hipStream_t);        \
    template hipError_t launch_stream_function<S, R>(const void*, const void*, const Geo&,       \
                                                     const Phys<R>&, int, void*, hipStream_t);
LBM_INSTANCES(float, float)
LBM_INSTANCES(double, double)
LBM_INSTANCES(float, double)
#undef LBM_INSTANCES
template hipError_t launch_rest<float>(void*, const Geo&, double, double, hipStream_t);
template hipError_t launch_rest<double>(void*, const Geo&, double, double, hipStream_t);
template hipError_t launch_pitch_copy<float>(void*, const void*, const Geo&, double, hipStream_t);
template hipError_t launch_pitch_copy<double>(void*, const void*, const Geo&, double,
                                              hipStream_t);

}  // namespace lbm
