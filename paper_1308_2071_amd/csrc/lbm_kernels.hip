// lbm_kernels.hip -- single-cavity kernels: the time step (one step per launch, two steps per
// launch, and the in-place AA-layout forms), the observables pass, the wall Nusselt reduction,
// the stream function and state initialisation.
#include "lbm_device.hpp"
#include "lbm_internal.hpp"

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
constexpr int kTbCols = 62;
constexpr int kTbWaves = 4;     // strips (wavefronts) per work-group
constexpr int kTbRounds = 6;    // aim: the work-groups fill about this many resident sets
constexpr int kTbMinRows = 8;

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

template <typename S, typename R, bool PN>
__global__ __launch_bounds__(64 * kTbWaves) void tb2_step_kernel(const S* __restrict__ src,
                                                                 S* __restrict__ dst,
                                                                 const S* __restrict__ med,
                                                                 Geo G, Phys<R> P, int nstrips,
                                                                 int rows) {
    const int lane = threadIdx.x & 63;
    // A work-group holds kTbWaves adjacent strips of one row segment, kept in step by a
    // barrier per row, so that the cache lines the neighbouring strips share are used while
    // resident.  Every wavefront runs the same rows; one past the last strip loads and stores
    // nothing.  Work-groups are dealt round-robin over the 8 XCDs; each XCD is given a
    // contiguous range of the logical work-groups (a bijection), so that neighbouring strips
    // and segments share its L2.
    int wg = blockIdx.x;
    {
        const int n = gridDim.x, per = n / 8, extra = n % 8;
        const int xcd = wg % 8, slot = wg / 8;
        wg = xcd * per + min(xcd, extra) + slot;
    }
    const int ngrp = (nstrips + kTbWaves - 1) / kTbWaves;
    const int strip = (wg % ngrp) * kTbWaves + (threadIdx.x >> 6), seg = wg / ngrp;
    const bool active = strip < nstrips;
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

// Wave-level reductions over the 64 lanes of a wavefront.
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    return v;
}
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_down(v, off, 64));
    return v;
}

// Macroscopic fields at the current time level, plus per-work-group partial results:
// part[3 * b + 0] = max |u|, part[3 * b + 1] = sum of stored f' (mass deviation),
// part[3 * b + 2] = 1 if a field is not finite.  Grid-stride over nodes.
template <typename S, typename R, bool PN, int L>
__global__ __launch_bounds__(256) void observe_kernel(const S* __restrict__ src,
                                                      const S* __restrict__ med, Geo G,
                                                      Phys<R> P, S* __restrict__ ux_out,
                                                      S* __restrict__ uy_out,
                                                      S* __restrict__ p_out,
                                                      S* __restrict__ T_out,
                                                      double* __restrict__ part) {
    const int n = G.nx * G.ny;
    double umax = 0.0, mass = 0.0, bad = 0.0;
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
        umax = fmax(umax, sp);
        if (!isfinite(sp) || !isfinite(double(p)) || !isfinite(double(T))) bad = 1.0;
        const int o = y * G.pitch + x;
        double s = 0.0;
#pragma unroll
        for (int i = 0; i < 9; ++i) s += double(src[i * G.plane + o]);
        mass += s;
    }
    __shared__ double red[3][4];
    umax = wave_max(umax);
    mass = wave_sum(mass);
    bad = wave_max(bad);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) {
        red[0][w] = umax;
        red[1][w] = mass;
        red[2][w] = bad;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double a = red[0][0], b = red[1][0], c = red[2][0];
        for (int i = 1; i < (int)(blockDim.x >> 6); ++i) {
            a = fmax(a, red[0][i]);
            b += red[1][i];
            c = fmax(c, red[2][i]);
        }
        part[3 * blockIdx.x + 0] = a;
        part[3 * blockIdx.x + 1] = b;
        part[3 * blockIdx.x + 2] = c;
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
// ny wall nodes; part[0..2] = partial results of observe_kernel (nparts work-groups).
// One work-group; writes out[0] nu_hot, out[1] nu_cold, out[2] max |u|, out[3] sum f',
// out[4] non-finite flag.
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
        double a = 0.0, b = 0.0, f = 0.0;
        for (int i = 0; i < nparts; ++i) {
            a = fmax(a, part[3 * i + 0]);
            b += part[3 * i + 1];
            f = fmax(f, part[3 * i + 2]);
        }
        out[2] = a;
        out[3] = b;
        out[4] = f;
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
            hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, tb2_step_kernel<S, R, PN>,
                                                         64 * kTbWaves, 0) != hipSuccess)
            return 0;
        return cus * per_cu;
    }();
    return n;
}

// Rows per segment of the two-step kernel.  Long segments amortise the two halo rows of the
// intermediate step; short-lived work-groups let vertically neighbouring segments run close
// together in time and keep the tail of the launch short.  Measured on the 4096^2 workload:
// about 6 rounds of the resident set (12 rows) is best, 1 round (69 rows) is 10 % slower.
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

// Queries the resident set of the two-step kernel once, outside any graph capture.
template <typename S, typename R>
void prepare_tb2() {
    (void)tb_resident<S, R>(true);
    (void)tb_resident<S, R>(false);
}

// Whether two steps per launch beat one: only with equal storage and arithmetic types (with
// FP64 arithmetic on FP32 storage the kernel holds 190 registers and runs at 2 waves per SIMD,
// 20 % slower than single steps) and with work-groups for at least a quarter of the resident
// set at 16-row segments (measured: 1024^2 gains 4 % in FP32 and 23 % in FP64, 4096^2 31 % and
// 35 %; on 256^2 the few long row loops are latency-bound and run 4x slower fused).
template <typename S, typename R>
bool tb2_pays(const Geo& G, bool per_node_medium) {
    if (!std::is_same<S, R>::value) return false;
    const int resident = tb_resident<S, R>(per_node_medium);
    const int nstrips = (G.nx + kTbCols - 1) / kTbCols;
    const long long groups =
        (long long)((nstrips + kTbWaves - 1) / kTbWaves) * ((G.ny + 15) / 16);
    return resident > 0 && 4 * groups >= resident;
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
    const int nstrips = (G.nx + kTbCols - 1) / kTbCols;
    int rows = 0, nwg = 0;
    tb2_shape<S, R>(G, med != nullptr, &rows, &nwg);
    if (med)
        tb2_step_kernel<S, R, true><<<nwg, 64 * kTbWaves, 0, s>>>(
            (const S*)src, (S*)dst, (const S*)med, G, P, nstrips, rows);
    else
        tb2_step_kernel<S, R, false><<<nwg, 64 * kTbWaves, 0, s>>>((const S*)src, (S*)dst,
                                                                   nullptr, G, P, nstrips, rows);
    return hipGetLastError();
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
