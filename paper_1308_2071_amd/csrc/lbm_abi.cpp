// lbm_abi.cpp -- the C ABI declared in include/lbm.h: argument checking, parameter derivation
// (Sec. 4 of arXiv:1308.2071), workspace layout, stream ordering, HIP-graph replay of the time
// loop, the adjoint's checkpoint-and-recompute schedule and the batched form.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "lbm.h"
#include "lbm_internal.hpp"

using namespace lbm;

namespace {

thread_local std::string g_err;

lbm_status fail(lbm_status s, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return s;
}

lbm_status hip_fail(hipError_t e, const char* what) {
    return fail(LBM_E_HIP, "%s: %s", what, hipGetErrorString(e));
}

#define HIP_TRY(expr, what)                         \
    do {                                            \
        hipError_t e_ = (expr);                     \
        if (e_ != hipSuccess) return hip_fail(e_, what); \
    } while (0)

constexpr size_t kAlign = 256;
size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

// Parameters of Sec. 4 derived from the problem statement.
struct Derived {
    double L, cs2, csT2, tau_v, tau_T, nu_e, nu, gbeta, dT, T0, K, Q;
};

Derived derive(const lbm_params& p) {
    Derived d;
    d.L = double(p.nx - 1);
    d.cs2 = 1.0 / 3.0;
    d.csT2 = (4.0 + p.varpi) / 10.0;
    // Eq. (37b)
    // with internal heating only (Ra = 0, Sec. 4.2) Ra_I takes Ra's place
    const double Ra_eff = p.Ra > 0 ? p.Ra : p.Ra_I;
    d.tau_v = p.tau_v > 0 ? p.tau_v : 0.5 + p.Ma * p.J * d.L * std::sqrt(p.Pr / Ra_eff) *
                                                std::sqrt(3.0);
    d.nu_e = d.cs2 * (d.tau_v - 0.5);  // Eq. (24)
    d.nu = d.nu_e / p.J;               // J = nu_e / nu
    // Pr = nu / alpha_e with alpha_e = sigma csT^2 (tau_T - 1/2) (Eq. (A9))
    d.tau_T = p.tau_T > 0 ? p.tau_T : 0.5 + d.nu / (p.sigma * d.csT2 * p.Pr);
    const bool sideheated = p.bc[LBM_WEST] == LBM_WALL_ISOTHERMAL &&
                            p.bc[LBM_EAST] == LBM_WALL_ISOTHERMAL &&
                            p.T_wall[LBM_WEST] != p.T_wall[LBM_EAST];
    d.dT = sideheated ? p.T_wall[LBM_WEST] - p.T_wall[LBM_EAST] : 1.0;
    d.T0 = sideheated ? 0.5 * (p.T_wall[LBM_WEST] + p.T_wall[LBM_EAST]) : p.T_init;
    // Ma = U / cs with U = sqrt(g beta dT L)
    d.gbeta = p.gbeta >= 0 ? p.gbeta : p.Ma * p.Ma * d.cs2 / (d.dT * d.L);
    d.K = p.Da > 0 ? p.Da * d.L * d.L : INFINITY;
    // Ra_I = g beta Q''' L^5 / (nu alpha_e^2) with alpha_e = sigma csT^2 (tau_T - 1/2)
    const double alpha = p.sigma * d.csT2 * (d.tau_T - 0.5);
    d.Q = p.Ra_I > 0 ? p.Ra_I * d.nu * alpha * alpha / (d.gbeta * std::pow(d.L, 5.0)) : p.Qv;
    return d;
}

bool walled(const lbm_params& p, int side) { return p.bc[side] != LBM_PERIODIC; }

// The interval T must stay in (LBM_DIV_TEMPERATURE): T_init and the isothermal walls' T,
// widened by the temperature scale dT and by the rise the heat source can cause at step n.
void temperature_bounds(const lbm_params& p, const Derived& d, int64_t n, double* lo,
                        double* hi) {
    double a = p.T_init, b = p.T_init;
    bool iso = false;
    for (int s = 0; s < 4; ++s)
        if (p.bc[s] == LBM_WALL_ISOTHERMAL) {
            iso = true;
            a = std::min(a, p.T_wall[s]);
            b = std::max(b, p.T_wall[s]);
        }
    const double Lmax = double(std::max(p.nx, p.ny) - 1);
    const double alpha = p.sigma * d.csT2 * (d.tau_T - 0.5);  // Eq. (A9)
    const double rise = iso ? std::fabs(d.Q) * Lmax * Lmax / (2.0 * alpha)
                            : std::fabs(d.Q) * double(n) / p.sigma;
    *lo = a - std::fabs(d.dT) - (d.Q < 0 ? rise : 0.0);
    *hi = b + std::fabs(d.dT) + (d.Q > 0 ? rise : 0.0);
}

// Fills the observables from the results r[0 .. kObsOut) of the observables pass (Nu_hot,
// Nu_cold, max |u|, sum f', non-finite flag, min T, max T, max |phi p - rho0 cs^2|) and
// decides the divergence flag (LBM_DIV_* in lbm.h).
void fill_obs(const lbm_params& p, const Derived& d, int64_t step, const double* r,
              lbm_obs* o) {
    const double n = double(p.nx) * p.ny;
    o->nu_hot = r[0];
    o->nu_cold = r[1];
    o->max_speed = r[2];
    o->mass_err = std::fabs(r[3]) / (n * p.rho0);
    o->step = step;
    o->T_min = r[5];
    o->T_max = r[6];
    o->phip_dev = r[7];
    double lo, hi;
    temperature_bounds(p, d, step, &lo, &hi);
    int why = 0;
    if (r[4] != 0.0 || !std::isfinite(r[0]) || !std::isfinite(r[1])) why |= LBM_DIV_NONFINITE;
    if (!(r[2] <= std::sqrt(d.cs2))) why |= LBM_DIV_SPEED;
    if (!(r[5] >= lo) || !(r[6] <= hi)) why |= LBM_DIV_TEMPERATURE;
    o->why = why;
    o->diverged = why != 0 ? 1 : 0;
}

// Bytes per stored value (populations, medium planes, fields) of a dtype.
size_t storage_bytes(int dtype) { return dtype == LBM_FP64 ? 8 : 4; }

lbm_status validate(const lbm_params& p) {
    if (p.dtype != LBM_FP32 && p.dtype != LBM_FP64 && p.dtype != LBM_FP32_F64)
        return fail(LBM_E_INVAL, "dtype %d is not LBM_FP32, LBM_FP64 or LBM_FP32_F64", p.dtype);
    for (int s = 0; s < 4; ++s)
        if (p.bc[s] < LBM_WALL_ISOTHERMAL || p.bc[s] > LBM_PERIODIC)
            return fail(LBM_E_INVAL, "bc[%d] = %d is not a side condition", s, p.bc[s]);
    if ((p.bc[LBM_WEST] == LBM_PERIODIC) != (p.bc[LBM_EAST] == LBM_PERIODIC))
        return fail(LBM_E_INVAL, "west and east sides must both be periodic or both walls");
    if ((p.bc[LBM_SOUTH] == LBM_PERIODIC) != (p.bc[LBM_NORTH] == LBM_PERIODIC))
        return fail(LBM_E_INVAL, "south and north sides must both be periodic or both walls");
    const int minx = walled(p, LBM_WEST) ? 5 : 2, miny = walled(p, LBM_SOUTH) ? 5 : 2;
    if (p.nx < minx || p.ny < miny)
        return fail(LBM_E_INVAL, "grid %d x %d too small (need >= %d x %d)", p.nx, p.ny, minx,
                    miny);
    const long long pitch = (p.nx + kPitchAlign - 1) / kPitchAlign * kPitchAlign;
    if (plane_elems(pitch, p.ny) * kPlanes >= (1LL << 31))
        return fail(LBM_E_INVAL, "grid %d x %d exceeds the 2^31-element state limit", p.nx, p.ny);
    if (!(p.rho0 > 0) || !(p.sigma > 0) || !(p.J > 0))
        return fail(LBM_E_INVAL, "rho0, sigma and J must be positive");
    if (!(p.varpi < 1) || !(p.varpi > -4))
        return fail(LBM_E_INVAL, "varpi = %g must lie in (-4, 1) (Eq. (29))", p.varpi);
    if (p.tau_v <= 0 && (!(p.Ra > 0 || p.Ra_I > 0) || !(p.Pr > 0) || !(p.Ma > 0)))
        return fail(LBM_E_INVAL, "Ra (or Ra_I), Pr and Ma must be positive to derive tau_v");
    if (p.Ra_I < 0 || !std::isfinite(p.Qv)) return fail(LBM_E_INVAL, "bad heat source");
    if (p.tau_T <= 0 && !(p.Pr > 0))
        return fail(LBM_E_INVAL, "Pr must be positive to derive tau_T");
    if (p.checkpoint_every < 0) return fail(LBM_E_INVAL, "checkpoint_every must be >= 0");
    if (p.layout != LBM_LAYOUT_PULL && p.layout != LBM_LAYOUT_AA)
        return fail(LBM_E_INVAL, "layout %d is not LBM_LAYOUT_PULL or LBM_LAYOUT_AA", p.layout);
    if (p.steps_per_launch != 0 && p.steps_per_launch != 1 && p.steps_per_launch != 2 &&
        p.steps_per_launch != 3 && p.steps_per_launch != kTileSteps &&
        p.steps_per_launch != kTinyTileSteps)
        return fail(LBM_E_INVAL, "steps_per_launch = %d is not 0, 1, 2, 3, %d or %d",
                    p.steps_per_launch, kTileSteps, kTinyTileSteps);
    if (p.steps_per_launch == 3 &&
        (p.dtype != LBM_FP32 ||
         plane_elems(pitch, p.ny) * kPlanes * (long long)storage_bytes(p.dtype) >= (1LL << 31)))
        return fail(LBM_E_UNSUPPORTED, "three steps per launch need FP32 and a state below 2 GiB");
    if (p.steps_per_launch == 2 &&
        plane_elems(pitch, p.ny) * (kPlanes / 2) * (long long)storage_bytes(p.dtype) >= (1LL << 31))
        return fail(LBM_E_UNSUPPORTED,
                    "two steps per launch need each half of the state (7 planes) below 2 GiB");
    if (p.layout == LBM_LAYOUT_AA && p.checkpoint_every > 0)
        return fail(LBM_E_UNSUPPORTED, "the AA layout has no adjoint tape");
    const Derived d = derive(p);
    if (!(d.tau_v > 0.5) || !std::isfinite(d.tau_v))
        return fail(LBM_E_INVAL, "tau_v = %.17g must exceed 1/2", d.tau_v);
    if (!(d.tau_T > 0.5) || !std::isfinite(d.tau_T))
        return fail(LBM_E_INVAL, "tau_T = %.17g must exceed 1/2", d.tau_T);
    if (!std::isfinite(d.gbeta)) return fail(LBM_E_INVAL, "g*beta is not finite");
    if (p.Ra_I > 0 && !(d.gbeta > 0)) return fail(LBM_E_INVAL, "Ra_I needs g*beta > 0");
    if (!std::isfinite(d.Q)) return fail(LBM_E_INVAL, "heat source is not finite");
    const double rates[5] = {p.s_e, p.s_eps, p.s_q, p.zeta3, p.zeta4};
    for (double r : rates)
        if (!(r > 0 && r < 2)) return fail(LBM_E_INVAL, "relaxation rate %g outside (0, 2)", r);
    return LBM_OK;
}

Geo make_geo(const lbm_params& p) {
    Geo G;
    G.nx = p.nx;
    G.ny = p.ny;
    G.pitch = (p.nx + kPitchAlign - 1) / kPitchAlign * kPitchAlign;
    G.plane = int(plane_elems(G.pitch, p.ny));
    G.wallW = walled(p, LBM_WEST);
    G.wallE = walled(p, LBM_EAST);
    G.wallS = walled(p, LBM_SOUTH);
    G.wallN = walled(p, LBM_NORTH);
    return G;
}

template <typename R>
Phys<R> make_phys(const lbm_params& p, const Derived& d, double phi_u) {
    Phys<R> P;
    P.rho0 = R(p.rho0);
    P.inv_rho0 = R(1.0 / p.rho0);
    P.gbeta = R(d.gbeta);
    P.ax = R(p.ext_accel[0]);
    P.ay = R(p.ext_accel[1]);
    P.nu = R(d.nu);
    P.s_e = R(p.s_e);
    P.s_eps = R(p.s_eps);
    P.s_q = R(p.s_q);
    P.s_v = R(1.0 / d.tau_v);
    P.os_e = R(1.0 - 0.5 * p.s_e);
    P.os_eps = R(1.0 - 0.5 * p.s_eps);
    P.os_q = R(1.0 - 0.5 * p.s_q);
    P.os_v = R(1.0 - 0.5 / d.tau_v);
    P.z_T = R(1.0 / d.tau_T);
    P.z3 = R(p.zeta3);
    P.z4 = R(p.zeta4);
    P.inv_sigma = R(1.0 / p.sigma);
    P.varpi = R(p.varpi);
    P.wt0 = R((1.0 - p.varpi) / 5.0);
    P.wt1 = R((4.0 + p.varpi) / 20.0);
    P.u_coef = R(1.0 / (p.sigma * d.csT2));
    P.T0 = R(d.T0);
    // heat source, Eqs. (30), (34), (36): Psi0 = Q/sigma, Psi3 = varpi Q/sigma
    P.hQs = R(0.5 * d.Q / p.sigma);
    P.psi3 = R((1.0 - 0.5 * p.zeta3) * p.varpi * d.Q / p.sigma);
    for (int s = 0; s < 4; ++s) {
        P.theta_wall[s] = R(p.T_wall[s] - d.T0);
        P.iso[s] = p.bc[s] == LBM_WALL_ISOTHERMAL;
    }
    P.forch = p.forchheimer ? 1 : 0;
    // uniform medium: phi_u and K = Da L^2
    const double Kinv = std::isinf(d.K) ? 0.0 : 1.0 / d.K;
    P.phi = R(phi_u);
    P.inv_phi = R(1.0 / phi_u);
    P.c_lin = R(phi_u * d.nu * Kinv);
    P.c_nl = R(p.forchheimer ? kErgun / std::sqrt(phi_u) * std::sqrt(Kinv) : 0.0);
    return P;
}

struct Layout {
    size_t state_bytes;   // one population buffer (14 planes)
    size_t off_buf[2];
    size_t off_med;       // 2 planes (phi, K), or none
    size_t off_part;      // observables partials + results
    size_t off_tape;      // checkpoints
    size_t n_ckpt;
    size_t off_seg;       // two banks of C states: the segment the adjoint is sweeping, and
                          // the one before it, recomputed meanwhile on a second stream
    size_t off_lam[2];
    size_t off_gacc;      // 2 FP64 planes
    size_t total;
};

Layout make_layout(const lbm_params& p, int64_t nsteps_max, bool med_planes) {
    const Geo G = make_geo(p);
    const size_t esz = storage_bytes(p.dtype);
    Layout L{};
    L.state_bytes = align_up(size_t(kPlanes) * G.plane * esz);
    size_t o = 0;
    L.off_buf[0] = o;
    o += L.state_bytes;
    L.off_buf[1] = o;
    if (p.layout == LBM_LAYOUT_AA)
        L.off_buf[1] = L.off_buf[0];  // one buffer, stepped in place
    else
        o += L.state_bytes;
    L.off_med = o;
    if (med_planes) o += align_up(2 * size_t(G.plane) * esz);
    L.off_part = o;
    o += align_up((kObsParts * kObserveWG + kObsOut) * sizeof(double));
    L.off_tape = o;
    if (p.checkpoint_every > 0) {
        const size_t C = size_t(p.checkpoint_every);
        L.n_ckpt = std::max<size_t>(1, (size_t(std::max<int64_t>(nsteps_max, 1)) + C - 1) / C);
        o += L.n_ckpt * L.state_bytes;
        L.off_seg = o;
        o += 2 * C * L.state_bytes;
        L.off_lam[0] = o;
        o += L.state_bytes;
        L.off_lam[1] = o;
        o += L.state_bytes;
        L.off_gacc = o;
        o += align_up(2 * size_t(G.plane) * sizeof(double));
    }
    L.total = o;
    return L;
}

}  // namespace

struct lbm_ctx {
    bool batch = false;
    lbm_params p{};
    Derived d{};
    Geo G{};
    Layout L{};
    hipStream_t stream = nullptr;
    char* ws = nullptr;
    bool med = false;
    int cur = 0;
    int64_t step = 0;
    int64_t nsteps_max = 0;
    double phi_u = 1.0;
    Phys<float> P32{};
    Phys<double> P64{};
    // graph replay of the time loop (per starting buffer)
    hipStream_t cap = nullptr;
    hipGraphExec_t gexec[2] = {nullptr, nullptr};
    int gsteps = 0;
    // adjoint: the stream that recomputes the next segment, and its events
    hipStream_t aux = nullptr;
    hipEvent_t ev_rec[2] = {nullptr, nullptr}, ev_bwd[2] = {nullptr, nullptr}, ev_go = nullptr;
    // batched form
    int ncav = 0;
    std::vector<lbm_params> bp;
    std::vector<Geo> bG;
    std::vector<Phys<float>> bP32;
    std::vector<Phys<double>> bP64;
    std::vector<long long> boff;      // element offset of each cavity in a state buffer
    std::vector<double> bLdT;         // L / dT per cavity
    size_t b_state_bytes = 0, b_off_buf[2] = {0, 0}, b_off_cav = 0, b_off_phys = 0;
    size_t b_off_tiles = 0, b_off_part = 0, b_max_tiles = 0;
    int b_wg = 4, b_npt = 1, b_nwg = 0, b_ntiles = 0;   // b_wg: rows per tile
    // two steps per launch: rows per segment (0: one step per launch) and work-groups
    size_t b_off_cav2 = 0, b_off_tbwg = 0, b_max_tbwg = 0;
    int b_tb_rows = 0, b_tb_nwg = 0, b_tb_waves = 4;

    void* buf(int i) const { return ws + L.off_buf[i]; }
    void* medp() const { return med ? ws + L.off_med : nullptr; }
    double* part() const { return (double*)(ws + L.off_part); }
    void* ckpt(size_t k) const { return ws + L.off_tape + k * L.state_bytes; }
    void* seg(int bank, size_t k) const {
        return ws + L.off_seg + (size_t(bank) * size_t(p.checkpoint_every) + k) * L.state_bytes;
    }
    void* lam(int i) const { return ws + L.off_lam[i]; }
    double* gacc(int i) const { return (double*)(ws + L.off_gacc) + size_t(i) * G.plane; }
};

namespace {

template <class T>
struct Tag {
    using type = T;
};

// Calls f(Tag<S>, Tag<R>) with the storage type S and the arithmetic type R of a dtype.
template <class F>
auto with_types(int dtype, F&& f) -> decltype(f(Tag<float>{}, Tag<float>{})) {
    if (dtype == LBM_FP64) return f(Tag<double>{}, Tag<double>{});
    if (dtype == LBM_FP32_F64) return f(Tag<float>{}, Tag<double>{});
    return f(Tag<float>{}, Tag<float>{});
}

// Kernel parameters in arithmetic type R: of the context, and of cavity i of a batch.
template <class R>
const Phys<R>& phys(const lbm_ctx* c);
template <>
const Phys<float>& phys<float>(const lbm_ctx* c) { return c->P32; }
template <>
const Phys<double>& phys<double>(const lbm_ctx* c) { return c->P64; }
template <class R>
const Phys<R>& bphys(const lbm_ctx* c, int i);
template <>
const Phys<float>& bphys<float>(const lbm_ctx* c, int i) { return c->bP32[i]; }
template <>
const Phys<double>& bphys<double>(const lbm_ctx* c, int i) { return c->bP64[i]; }

#define LBM_TYPES(st, rt)                  \
    using S = typename decltype(st)::type; \
    using R = typename decltype(rt)::type;

lbm_status check_ctx(const lbm_ctx* c, bool want_batch) {
    if (!c) return fail(LBM_E_INVAL, "null context");
    if (c->batch != want_batch)
        return fail(LBM_E_INVAL, want_batch ? "context is not a batch" : "context is a batch");
    return LBM_OK;
}

// One pull-layout step from src to dst.
hipError_t step_once(lbm_ctx* c, const void* src, void* dst, hipStream_t s) {
    return with_types(c->p.dtype, [&](auto st, auto rt) {
        LBM_TYPES(st, rt)
        return launch_step<S, R>(src, dst, c->medp(), c->G, phys<R>(c), s);
    });
}

// One step of the cavity's state from form `from`: the buffer index for the pull layout, the
// step parity for the AA layout (the state then lives in buf(0) == buf(1)).
hipError_t advance(lbm_ctx* c, int from, hipStream_t s) {
    if (c->p.layout != LBM_LAYOUT_AA) return step_once(c, c->buf(from), c->buf(1 - from), s);
    return with_types(c->p.dtype, [&](auto st, auto rt) {
        LBM_TYPES(st, rt)
        return launch_aa_step<S, R>(c->buf(0), c->medp(), c->G, phys<R>(c), from, s);
    });
}

// k > 1 steps in one launch from buffer `from` (pull layout only): the two- and three-step
// kernels for k = 2 and 3, the tiles in LDS for k = kTileSteps or kTinyTileSteps.
hipError_t advance_k(lbm_ctx* c, int k, int from, hipStream_t s) {
    return with_types(c->p.dtype, [&](auto st, auto rt) {
        LBM_TYPES(st, rt)
        if (k == 2)
            return launch_tb2_step<S, R>(c->buf(from), c->buf(1 - from), c->medp(), c->G,
                                         phys<R>(c), s);
        if (k == 3)
            return launch_tb3_step<S, R>(c->buf(from), c->buf(1 - from), c->medp(), c->G,
                                         phys<R>(c), s);
        return launch_tile_step<S, R>(c->buf(from), c->buf(1 - from), c->medp(), c->G,
                                      phys<R>(c), k, s);
    });
}

// Time steps per launch of the time loop: one with the AA layout; steps_per_launch when it
// asks for 1, 2, 3, kTileSteps or kTinyTileSteps; by default three (FP32) or two where that is
// measured to pay, else the tiles in LDS where a form of them does, else one.  With a tape,
// launches of several steps run only between checkpoints (lbm_step).
int launch_steps(const lbm_ctx* c) {
    if (c->p.layout != LBM_LAYOUT_PULL) return 1;
    if (c->p.steps_per_launch != 0) return c->p.steps_per_launch;
    return with_types(c->p.dtype, [&](auto st, auto rt) {
        LBM_TYPES(st, rt)
        if (tb3_pays<S, R>(c->G, c->med)) return 3;
        if (tb2_pays<S, R>(c->G, c->med)) return 2;
        const int t = tile_steps<S, R>(c->G, c->med);
        return t > 0 ? t : 1;
    });
}

// The PopLayout form the current state is in.
int pop_layout(const lbm_ctx* c) {
    if (c->p.layout != LBM_LAYOUT_AA) return kPull;
    return c->cur == 0 ? kAAOpp : kAAOwn;
}

// Capture kGraphSteps steps into an executable graph for the given starting buffer or parity:
// an even number of launches at every steps-per-launch count, so that the buffers, or the AA
// parity, end where they started.
constexpr int kGraphSteps = 48;
static_assert(kGraphSteps % 2 == 0 && kGraphSteps % 4 == 0 && kGraphSteps % 6 == 0 &&
                  kGraphSteps % (2 * kTileSteps) == 0 && kGraphSteps % (2 * kTinyTileSteps) == 0,
              "kGraphSteps must be an even number of launches of each form");

lbm_status ensure_graph(lbm_ctx* c, int start) {
    if (c->gexec[start]) return LBM_OK;
    if (!c->cap) HIP_TRY(hipStreamCreateWithFlags(&c->cap, hipStreamNonBlocking), "stream create");
    HIP_TRY(hipStreamBeginCapture(c->cap, hipStreamCaptureModeThreadLocal), "begin capture");
    hipError_t err = hipSuccess;
    int b = start;
    const int k = launch_steps(c);
    if (k > 1) {
        // kGraphSteps / k launches: an even number of buffer swaps
        for (int n = 0; n < kGraphSteps / k && err == hipSuccess; ++n) {
            err = advance_k(c, k, b, c->cap);
            b = 1 - b;
        }
    } else {
        for (int k = 0; k < kGraphSteps && err == hipSuccess; ++k) {
            err = advance(c, b, c->cap);
            b = 1 - b;
        }
    }
    hipGraph_t graph = nullptr;
    hipError_t e2 = hipStreamEndCapture(c->cap, &graph);
    if (err != hipSuccess) {
        if (graph) (void)hipGraphDestroy(graph);
        return hip_fail(err, "captured step launch");
    }
    if (e2 != hipSuccess) return hip_fail(e2, "end capture");
    hipError_t e3 = hipGraphInstantiate(&c->gexec[start], graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e3 != hipSuccess) {
        c->gexec[start] = nullptr;
        return hip_fail(e3, "graph instantiate");
    }
    c->gsteps = kGraphSteps;
    return LBM_OK;
}

}  // namespace

namespace {

// ---- batched form ------------------------------------------------------------------------

constexpr int kBatchGraphSteps = 32;   // even: a replay ends on the buffer it started from
constexpr int kBatchObsWG = 64;        // work-groups of one cavity's observables pass
constexpr int kBatchObsPer = kObsParts * kBatchObsWG + kObsOut;  // doubles per cavity
constexpr int kMinTileWidth = 64;      // narrowest tile of any supported launch shape

struct BatchLayout {
    std::vector<long long> off;
    size_t state_bytes, off_buf[2], off_cav, off_phys, off_tiles, off_part, max_tiles, total;
    size_t off_cav2, off_tbwg, max_tbwg;   // tables of the two-step form
};

// Work-groups of the batched two-step kernel for segments of `rows` rows, `waves` strips per
// work-group.
size_t batch_tb_groups(const std::vector<Geo>& G, int rows, int waves) {
    size_t n = 0;
    for (const Geo& g : G) {
        const size_t strips = size_t((g.nx + kTbCols - 1) / kTbCols);
        n += (strips + waves - 1) / waves * size_t((g.ny + rows - 1) / rows);
    }
    return n;
}

lbm_status batch_layout(int32_t n, const lbm_params* p, BatchLayout* L) {
    if (n <= 0) return fail(LBM_E_INVAL, "batch of %d cavities", n);
    const int dt = p[0].dtype;
    long long elems = 0;
    size_t tiles = 0;
    L->off.clear();
    for (int i = 0; i < n; ++i) {
        lbm_status s = validate(p[i]);
        if (s != LBM_OK) return fail(s, "cavity %d: %s", i, g_err.c_str());
        if (p[i].dtype != dt) return fail(LBM_E_INVAL, "cavity %d: dtypes differ in a batch", i);
        if (p[i].checkpoint_every != 0)
            return fail(LBM_E_UNSUPPORTED, "cavity %d: no adjoint tape in a batch", i);
        if (p[i].layout != LBM_LAYOUT_PULL)
            return fail(LBM_E_UNSUPPORTED, "cavity %d: a batch uses the pull layout", i);
        if (i == 0 && (p[0].steps_per_launch == 3 || p[0].steps_per_launch == kTileSteps ||
                       p[0].steps_per_launch == kTinyTileSteps))
            return fail(LBM_E_UNSUPPORTED, "a batch steps one or two steps per launch");
        const Geo G = make_geo(p[i]);
        if (p[0].steps_per_launch == 2 && tb2_descs(G, storage_bytes(dt)) != 1)
            return fail(LBM_E_UNSUPPORTED,
                        "cavity %d: two steps per launch need a state below 2 GiB", i);
        L->off.push_back(elems);
        elems += (long long)kPlanes * G.plane;
        elems = (elems + 63) / 64 * 64;  // 256-byte alignment in FP32
        tiles += size_t(G.ny) * size_t((G.nx + kMinTileWidth - 1) / kMinTileWidth);
    }
    if (elems >= (1LL << 31))
        return fail(LBM_E_INVAL, "batch state of %lld elements exceeds 2^31", elems);
    if (tiles >= (size_t(1) << 31)) return fail(LBM_E_INVAL, "too many tiles");
    const size_t esz = storage_bytes(dt);
    L->state_bytes = align_up(size_t(elems) * esz);
    size_t o = 0;
    L->off_buf[0] = o;
    o += L->state_bytes;
    L->off_buf[1] = o;
    o += L->state_bytes;
    L->off_cav = o;
    o += align_up(n * sizeof(BatchCavity));
    L->off_phys = o;
    o += align_up(n * std::max(sizeof(Phys<float>), sizeof(Phys<double>)));
    L->off_tiles = o;
    L->max_tiles = tiles;
    o += align_up(tiles * sizeof(int));
    std::vector<Geo> geos;
    for (int i = 0; i < n; ++i) geos.push_back(make_geo(p[i]));
    L->off_cav2 = o;
    o += align_up(n * sizeof(BatchCavity));
    L->off_tbwg = o;
    L->max_tbwg = batch_tb_groups(geos, kBatchTbMinRows, 1);  // the most: shortest rows, 1 strip
    o += align_up(L->max_tbwg * sizeof(int));
    L->off_part = o;
    o += align_up(size_t(n) * kBatchObsPer * sizeof(double));
    L->total = o;
    return LBM_OK;
}

hipError_t batch_rest(lbm_ctx* c) {
    const size_t esz = storage_bytes(c->p.dtype);
    for (int b = 0; b < 2; ++b) {
        char* base = c->ws + c->b_off_buf[b];
        for (int i = 0; i < c->ncav; ++i) {
            const lbm_params& p = c->bp[i];
            const Derived d = derive(p);
            const double g0 = (1.0 - p.varpi) / 5.0 * (p.T_init - d.T0);
            const double g1 = (4.0 + p.varpi) / 20.0 * (p.T_init - d.T0);
            void* dst = base + size_t(c->boff[i]) * esz;
            hipError_t e = esz == 8 ? launch_rest<double>(dst, c->bG[i], g0, g1, c->stream)
                                    : launch_rest<float>(dst, c->bG[i], g0, g1, c->stream);
            if (e != hipSuccess) return e;
        }
    }
    return hipSuccess;
}

// Tile queue for tiles of w nodes along x by h rows: fills the cavity table and the
// tile -> cavity table.
hipError_t batch_tables(lbm_ctx* c, int w, int h) {
    std::vector<BatchCavity> cav(c->ncav);
    std::vector<int> tc;
    tc.reserve(c->b_max_tiles);
    for (int i = 0; i < c->ncav; ++i) {
        cav[i].G = c->bG[i];
        cav[i].off = c->boff[i];
        cav[i].tile0 = int(tc.size());
        cav[i].tiles_x = (c->bG[i].nx + w - 1) / w;
        const size_t nt = size_t(cav[i].tiles_x) * size_t((c->bG[i].ny + h - 1) / h);
        tc.insert(tc.end(), nt, i);
    }
    if (tc.size() > c->b_max_tiles) return hipErrorInvalidValue;
    c->b_ntiles = int(tc.size());
    hipError_t e = hipMemcpy(c->ws + c->b_off_cav, cav.data(), cav.size() * sizeof(BatchCavity),
                             hipMemcpyHostToDevice);
    if (e != hipSuccess) return e;
    return hipMemcpy(c->ws + c->b_off_tiles, tc.data(), tc.size() * sizeof(int),
                     hipMemcpyHostToDevice);
}

template <typename R>
BatchTable<R> batch_table(const lbm_ctx* c) {
    BatchTable<R> T;
    T.cav = (const BatchCavity*)(c->ws + c->b_off_cav);
    T.phys = (const Phys<R>*)(c->ws + c->b_off_phys);
    T.tile_cav = (const int*)(c->ws + c->b_off_tiles);
    T.ncav = c->ncav;
    T.ntiles = c->b_ntiles;
    return T;
}

// Tables of the two-step form for segments of `rows` rows and `waves` strips per work-group:
// per cavity its first logical work-group (tile0) and strip groups (tiles_x), and the
// work-group -> cavity list.
hipError_t batch_tb_tables(lbm_ctx* c, int rows, int waves) {
    std::vector<BatchCavity> cav(c->ncav);
    std::vector<int> wc;
    for (int i = 0; i < c->ncav; ++i) {
        const Geo& G = c->bG[i];
        const int ngrp = ((G.nx + kTbCols - 1) / kTbCols + waves - 1) / waves;
        cav[i].G = G;
        cav[i].off = c->boff[i];
        cav[i].tile0 = int(wc.size());
        cav[i].tiles_x = ngrp;
        wc.insert(wc.end(), size_t(ngrp) * size_t((G.ny + rows - 1) / rows), i);
    }
    if (rows < kBatchTbMinRows || wc.size() > c->b_max_tbwg) return hipErrorInvalidValue;
    c->b_tb_nwg = int(wc.size());
    hipError_t e = hipMemcpy(c->ws + c->b_off_cav2, cav.data(), cav.size() * sizeof(BatchCavity),
                             hipMemcpyHostToDevice);
    if (e != hipSuccess) return e;
    return hipMemcpy(c->ws + c->b_off_tbwg, wc.data(), wc.size() * sizeof(int),
                     hipMemcpyHostToDevice);
}

template <typename R>
BatchTable<R> batch_tb_table(const lbm_ctx* c) {
    BatchTable<R> T;
    T.cav = (const BatchCavity*)(c->ws + c->b_off_cav2);
    T.phys = (const Phys<R>*)(c->ws + c->b_off_phys);
    T.tile_cav = (const int*)(c->ws + c->b_off_tbwg);
    T.ncav = c->ncav;
    T.ntiles = c->b_tb_nwg;
    return T;
}

// Two steps of every cavity in one launch, from buffer `from` to the other.
hipError_t batch_step2(lbm_ctx* c, int from, hipStream_t s) {
    const void* src = c->ws + c->b_off_buf[from];
    void* dst = c->ws + c->b_off_buf[1 - from];
    return with_types(c->p.dtype, [&](auto st, auto rt) {
        LBM_TYPES(st, rt)
        return launch_batch_tb2<S, R>(src, dst, batch_tb_table<R>(c), c->b_tb_rows,
                                      c->b_tb_waves, s);
    });
}

hipError_t batch_step_once(lbm_ctx* c, int from, hipStream_t s) {
    const void* src = c->ws + c->b_off_buf[from];
    void* dst = c->ws + c->b_off_buf[1 - from];
    return with_types(c->p.dtype, [&](auto st, auto rt) {
        LBM_TYPES(st, rt)
        return launch_batch_step<S, R>(src, dst, batch_table<R>(c), c->b_npt, c->b_wg, c->b_nwg,
                                       s);
    });
}

lbm_status ensure_batch_graph(lbm_ctx* c, int start) {
    if (c->gexec[start]) return LBM_OK;
    if (!c->cap) HIP_TRY(hipStreamCreateWithFlags(&c->cap, hipStreamNonBlocking), "stream create");
    HIP_TRY(hipStreamBeginCapture(c->cap, hipStreamCaptureModeThreadLocal), "begin capture");
    hipError_t err = hipSuccess;
    int b = start;
    if (c->b_tb_rows > 0) {
        // kBatchGraphSteps / 2 two-step launches: an even number of buffer swaps
        for (int k = 0; k < kBatchGraphSteps / 2 && err == hipSuccess; ++k) {
            err = batch_step2(c, b, c->cap);
            b = 1 - b;
        }
    } else {
        for (int k = 0; k < kBatchGraphSteps && err == hipSuccess; ++k) {
            err = batch_step_once(c, b, c->cap);
            b = 1 - b;
        }
    }
    hipGraph_t graph = nullptr;
    hipError_t e2 = hipStreamEndCapture(c->cap, &graph);
    if (err != hipSuccess) {
        if (graph) (void)hipGraphDestroy(graph);
        return hip_fail(err, "captured batch launch");
    }
    if (e2 != hipSuccess) return hip_fail(e2, "end capture");
    hipError_t e3 = hipGraphInstantiate(&c->gexec[start], graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e3 != hipSuccess) {
        c->gexec[start] = nullptr;
        return hip_fail(e3, "graph instantiate");
    }
    return LBM_OK;
}

// Cache key: device architecture, dtype and the list of cavity shapes.
std::string batch_key(const lbm_ctx* c) {
    hipDeviceProp_t prop;
    int dev = 0;
    std::string arch = "unknown";
    if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess)
        arch = prop.gcnArchName;
    for (char& ch : arch)
        if (ch == ' ' || ch == ':') ch = '_';
    uint64_t h = 1469598103934665603ULL;  // FNV-1a over the shapes
    auto mix = [&h](uint64_t v) {
        for (int k = 0; k < 8; ++k) {
            h ^= (v >> (8 * k)) & 0xff;
            h *= 1099511628211ULL;
        }
    };
    mix(uint64_t(c->ncav));
    for (const Geo& G : c->bG) {
        mix(uint64_t(G.nx));
        mix(uint64_t(G.ny));
    }
    char buf[128];
    snprintf(buf, sizeof buf, "v3|%s|%s|%016llx", arch.c_str(),
             c->p.dtype == LBM_FP64 ? "fp64" : c->p.dtype == LBM_FP32_F64 ? "fp32_f64" : "fp32",
             (unsigned long long)h);
    return buf;
}

// A cache line: key, rows per tile, 64-node segments per work-item, work-groups (0: one tile
// per work-group), rows per segment of the two-step form (0: one step per launch) and its
// strips per work-group.
bool cache_lookup(const char* path, const std::string& key, int* wg, int* npt, int* nwg,
                  int* tb_rows, int* tb_waves) {
    FILE* f = std::fopen(path, "r");
    if (!f) return false;
    char line[512], k[256];
    int a, b, d, t, w;
    bool found = false;
    while (std::fgets(line, sizeof line, f))
        if (std::sscanf(line, "%255s %d %d %d %d %d", k, &a, &b, &d, &t, &w) == 6 && key == k) {
            *wg = a;
            *npt = b;
            *nwg = d;
            *tb_rows = t;
            *tb_waves = w;
            found = true;
        }
    std::fclose(f);
    return found;
}

void cache_store(const char* path, const std::string& key, int wg, int npt, int nwg,
                 int tb_rows, int tb_waves) {
    FILE* f = std::fopen(path, "a");
    if (!f) return;
    std::fprintf(f, "%s %d %d %d %d %d\n", key.c_str(), wg, npt, nwg, tb_rows, tb_waves);
    std::fclose(f);
}

// Times `launches` launches of `step` (alternating buffers) after 3 untimed ones; ms per step.
template <class Step>
hipError_t time_steps(lbm_ctx* c, hipEvent_t e0, hipEvent_t e1, int steps_per_launch,
                      Step&& step, float* ms_per_step) {
    hipError_t e = hipSuccess;
    int from = 0;
    for (int k = 0; k < 3 && e == hipSuccess; ++k, from = 1 - from) e = step(from);
    if (e == hipSuccess) e = hipEventRecord(e0, c->stream);
    for (int k = 0; k < 10 && e == hipSuccess; ++k, from = 1 - from) e = step(from);
    if (e == hipSuccess) e = hipEventRecord(e1, c->stream);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    *ms_per_step = ms / float(10 * steps_per_launch);
    return e;
}

// Autotuner, on the batch itself.  The one-step kernel: every supported tile shape (rows per
// work-group x 64-node segments per work-item), with one tile per work-group and with chunked
// persistent grids of 2..16 work-groups per CU.  The two-step kernel: segments of 2, 3, 4, 5,
// 6, 8 and 12 rows with 1, 2 or 4 strips per work-group (short segments keep the launch's
// tail short; on the 64-cavity workload 3 rows and one strip won, 61.4k against 60.3k MLUPS
// for the best of 6 rows and up).  It keeps the fastest per step (the
// one-step shape is kept either way, for odd step counts), unless steps_per_launch of the
// first cavity forces one or two steps per launch.  The result is cached per (device, dtype,
// cavity shapes, that setting) in tune_cache_path.
lbm_status batch_tune(lbm_ctx* c, const char* path) {
    int cu = 256;
    int dev = 0;
    if (hipGetDevice(&dev) == hipSuccess)
        (void)hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, dev);
    const int spl = c->bp[0].steps_per_launch;
    const std::string key = batch_key(c) + "|s" + std::to_string(spl);
    int rows, npt, nwg, tbr, tbw;
    c->b_tb_rows = 0;
    c->b_tb_nwg = 0;
    if (path && cache_lookup(path, key, &rows, &npt, &nwg, &tbr, &tbw)) {
        c->b_wg = rows;
        c->b_npt = npt;
        HIP_TRY(batch_tables(c, 64 * npt, rows), "tile tables");
        c->b_nwg = nwg > 0 ? nwg : c->b_ntiles;
        if (tbr > 0) {
            HIP_TRY(batch_tb_tables(c, tbr, tbw), "two-step tables");
            c->b_tb_rows = tbr;
            c->b_tb_waves = tbw;
        }
        return LBM_OK;
    }
    if (!path) {
        c->b_wg = 4;
        c->b_npt = 1;
        HIP_TRY(batch_tables(c, 64, 4), "tile tables");
        c->b_nwg = c->b_ntiles;
        if (spl == 2) {
            HIP_TRY(batch_tb_tables(c, 12, 4), "two-step tables");
            c->b_tb_rows = 12;
            c->b_tb_waves = 4;
        }
        return LBM_OK;
    }
    const int shapes[10][2] = {{1, 1}, {1, 2}, {1, 4}, {2, 1}, {2, 2}, {2, 4},
                               {4, 1}, {4, 2}, {4, 4}, {8, 1}};
    const int per_cu[5] = {0, 2, 4, 8, 16};  // 0: one tile per work-group
    const int tb_rows[7] = {kBatchTbMinRows, 3, 4, 5, 6, 8, 12};
    const int tb_waves[3] = {1, 2, 4};
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0), "event");
    HIP_TRY(hipEventCreate(&e1), "event");
    float best = 1e30f, best_tb = 1e30f;
    int br = 4, bn = 1, bg = 0, btr = 0, btw = 4;
    lbm_status st = LBM_OK;
    for (const auto& sh : shapes) {
        hipError_t e = batch_tables(c, 64 * sh[1], sh[0]);
        if (e != hipSuccess) { st = hip_fail(e, "tile tables"); break; }
        for (int pc : per_cu) {
            c->b_wg = sh[0];
            c->b_npt = sh[1];
            c->b_nwg = pc == 0 ? c->b_ntiles : std::min(c->b_ntiles, pc * cu);
            float ms = 0;
            e = time_steps(
                c, e0, e1, 1, [&](int from) { return batch_step_once(c, from, c->stream); }, &ms);
            if (e != hipSuccess) { st = hip_fail(e, "autotune"); break; }
            if (ms < best) {
                best = ms;
                br = sh[0];
                bn = sh[1];
                bg = pc == 0 ? 0 : c->b_nwg;
            }
        }
        if (st != LBM_OK) break;
    }
    bool fit = true;  // the two-step kernel needs each cavity's state below 2 GiB
    for (int i = 0; i < c->ncav; ++i)
        fit = fit && tb2_descs(c->bG[i], storage_bytes(c->p.dtype)) == 1;
    if (st == LBM_OK && spl != 1 && fit) {
        for (int tr : tb_rows) {
            for (int tw : tb_waves) {
                hipError_t e = batch_tb_tables(c, tr, tw);
                if (e != hipSuccess) { st = hip_fail(e, "two-step tables"); break; }
                c->b_tb_rows = tr;
                c->b_tb_waves = tw;
                float ms = 0;
                e = time_steps(c, e0, e1, 2,
                               [&](int from) { return batch_step2(c, from, c->stream); }, &ms);
                if (e != hipSuccess) { st = hip_fail(e, "autotune"); break; }
                if (ms < best_tb) {
                    best_tb = ms;
                    btr = tr;
                    btw = tw;
                }
            }
            if (st != LBM_OK) break;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    c->b_tb_rows = 0;
    if (st != LBM_OK) return st;
    c->b_wg = br;
    c->b_npt = bn;
    HIP_TRY(batch_tables(c, 64 * bn, br), "tile tables");
    c->b_nwg = bg > 0 ? bg : c->b_ntiles;
    const int use_tr = (btr > 0 && (spl == 2 || best_tb < best)) ? btr : 0;
    c->b_tb_nwg = 0;
    if (use_tr > 0) {
        HIP_TRY(batch_tb_tables(c, use_tr, btw), "two-step tables");
        c->b_tb_rows = use_tr;
        c->b_tb_waves = btw;
    }
    cache_store(path, key, br, bn, bg, use_tr, btw);
    return LBM_OK;
}

}  // namespace

namespace {

// Fills context c for the validated parameters p over the workspace (at least L.total bytes)
// and puts the cavity at rest: the medium planes (when phi or K is given) and both state
// buffers are written, so nothing in the workspace needs to start at zero.  Synchronises.
lbm_status setup_ctx(lbm_ctx* c, const lbm_params& p, const Layout& L, int64_t nmax,
                     const void* phi, const void* K, double phi_uniform, void* workspace,
                     void* hip_stream) {
    const bool med = phi != nullptr || K != nullptr;
    c->p = p;
    c->d = derive(p);
    c->G = make_geo(p);
    c->L = L;
    c->stream = (hipStream_t)hip_stream;
    c->ws = (char*)workspace;
    c->med = med;
    c->nsteps_max = nmax;
    c->phi_u = phi ? 1.0 : phi_uniform;
    c->P32 = make_phys<float>(p, c->d, c->phi_u);
    c->P64 = make_phys<double>(p, c->d, c->phi_u);
    const double g0 = (1.0 - p.varpi) / 5.0 * (p.T_init - c->d.T0);
    const double g1 = (4.0 + p.varpi) / 20.0 * (p.T_init - c->d.T0);
    hipError_t e = with_types(p.dtype, [&](auto st, auto rt) {
        LBM_TYPES(st, rt)
        prepare_tb2<S, R>();
        hipError_t e1 = hipSuccess;
        if (med) {
            char* mp = c->ws + L.off_med;
            const size_t plane_bytes = size_t(c->G.plane) * sizeof(S);
            // an infinite K (Da <= 0) is stored as a large finite value: drag ~ 1/K vanishes
            const double Kv = std::isinf(c->d.K) ? (sizeof(S) == 8 ? 1e300 : 1e30) : c->d.K;
            e1 = launch_pitch_copy<S>(mp, phi, c->G, phi_uniform, c->stream);
            if (e1 == hipSuccess)
                e1 = launch_pitch_copy<S>(mp + plane_bytes, K, c->G, Kv, c->stream);
        }
        // both buffers, so that the row padding (never written by a step) is defined too
        for (int b = 0; b < 2 && e1 == hipSuccess; ++b)
            e1 = launch_rest<S>(c->buf(b), c->G, g0, g1, c->stream);
        return e1;
    });
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(e, "cavity set-up");
    return LBM_OK;
}

// Observables of the context's current state (see lbm_observables).  Synchronises.
lbm_status observe_ctx(lbm_ctx* c, lbm_obs* o, void* ux, void* uy, void* p, void* T) {
    double* part = c->part();
    double* res = part + kObsParts * kObserveWG;
    const double LdT = c->d.L / c->d.dT;
    hipError_t e = with_types(c->p.dtype, [&](auto st, auto rt) {
        LBM_TYPES(st, rt)
        return launch_observe<S, R>(c->buf(c->cur), c->medp(), c->G, phys<R>(c), pop_layout(c),
                                    ux, uy, p, T, part, kObserveWG, LdT, res, c->stream);
    });
    if (e != hipSuccess) return hip_fail(e, "observables launch");
    double h[kObsOut];
    HIP_TRY(hipMemcpyAsync(h, res, sizeof h, hipMemcpyDeviceToHost, c->stream), "readback");
    HIP_TRY(hipStreamSynchronize(c->stream), "synchronize");
    fill_obs(c->p, c->d, c->step, h, o);
    if (o->diverged)
        return fail(LBM_E_DIVERGED, "diverged at step %lld (reasons %d)", (long long)c->step,
                    o->why);
    return LBM_OK;
}

// ---- device memory for lbm_run_noalloc --------------------------------------------------------
// The one entry point that allocates nothing keeps its cavity (two state buffers, the medium
// planes and the observables' partial results) in this array.  Each GPU the library runs on
// holds its own copy, at its own address, from the module's load until the process ends.  In
// host code the array's name is only a stand-in for the symbol: device addresses come from
// hipGetSymbolAddress, per device.
constexpr size_t kNoAllocBytes = size_t(64) << 20;
constexpr int kMaxDevices = 64;
static __device__ __align__(256) char scratch[kNoAllocBytes];

// The current device's address of `scratch`, looked up once per device with that device
// current and kept.
lbm_status scratch_address(void** out) {
    static std::mutex mu;
    static void* addr[kMaxDevices] = {};
    int dev = -1;
    HIP_TRY(hipGetDevice(&dev), "hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices)
        return fail(LBM_E_UNSUPPORTED, "device %d beyond the %d the library tracks", dev,
                    kMaxDevices);
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[dev]) {
        void* ptr = nullptr;
        HIP_TRY(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)");
        if (!ptr) return fail(LBM_E_HIP, "hipGetSymbolAddress(scratch) returned NULL");
        addr[dev] = ptr;
    }
    *out = addr[dev];
    return LBM_OK;
}

}  // namespace

extern "C" {

const char* lbm_status_string(lbm_status s) {
    switch (s) {
        case LBM_OK: return "LBM_OK";
        case LBM_E_INVAL: return "LBM_E_INVAL";
        case LBM_E_NOMEM: return "LBM_E_NOMEM";
        case LBM_E_HIP: return "LBM_E_HIP";
        case LBM_E_DIVERGED: return "LBM_E_DIVERGED";
        case LBM_E_STATE: return "LBM_E_STATE";
        case LBM_E_UNSUPPORTED: return "LBM_E_UNSUPPORTED";
        default: return "LBM_E_UNKNOWN";
    }
}

const char* lbm_last_error(void) { return g_err.c_str(); }

lbm_status lbm_default_params(lbm_params* p) {
    if (!p) return fail(LBM_E_INVAL, "null params");
    std::memset(p, 0, sizeof(*p));
    p->nx = 64;
    p->ny = 64;
    p->bc[LBM_WEST] = LBM_WALL_ISOTHERMAL;
    p->bc[LBM_EAST] = LBM_WALL_ISOTHERMAL;
    p->bc[LBM_SOUTH] = LBM_WALL_ADIABATIC;
    p->bc[LBM_NORTH] = LBM_WALL_ADIABATIC;
    p->T_wall[LBM_WEST] = 1.0;
    p->T_wall[LBM_EAST] = 0.0;
    p->Ra = 1e3;
    p->Pr = 1.0;
    p->Da = 1e-2;
    p->J = 1.0;
    p->Ma = 0.1;
    p->sigma = 1.0;
    p->varpi = -2.0;
    p->rho0 = 1.0;
    p->s_e = 1.1;
    p->s_eps = 1.1;
    p->s_q = 1.2;
    p->zeta3 = 1.5;
    p->zeta4 = 1.5;
    p->forchheimer = 1;
    p->T_init = 0.5;
    p->tau_v = -1.0;
    p->tau_T = -1.0;
    p->gbeta = -1.0;
    p->Ra_I = 0.0;
    p->Qv = 0.0;
    p->dtype = LBM_FP32;
    p->checkpoint_every = 0;
    p->layout = LBM_LAYOUT_PULL;
    p->steps_per_launch = 0;
    g_err.clear();
    return LBM_OK;
}

lbm_status lbm_derived(const lbm_params* p, double* out) {
    if (!p || !out) return fail(LBM_E_INVAL, "null argument");
    const Derived d = derive(*p);
    const double v[10] = {d.L, d.tau_v, d.tau_T, d.nu_e, d.nu, d.gbeta, d.dT, d.T0, d.K, d.Q};
    std::memcpy(out, v, sizeof v);
    return LBM_OK;
}

lbm_status lbm_workspace_size(const lbm_params* p, int64_t nsteps_max, size_t* bytes) {
    if (!p || !bytes) return fail(LBM_E_INVAL, "null argument");
    lbm_status s = validate(*p);
    if (s != LBM_OK) return s;
    if (p->checkpoint_every > 0 && nsteps_max <= 0)
        return fail(LBM_E_INVAL, "a tape needs nsteps_max > 0");
    *bytes = make_layout(*p, nsteps_max, true).total;
    return LBM_OK;
}

lbm_status lbm_init(lbm_ctx** out, const lbm_params* p, const void* phi, const void* K,
                    double phi_uniform, void* workspace, size_t ws_bytes, void* hip_stream) {
    if (!out || !p) return fail(LBM_E_INVAL, "null argument");
    *out = nullptr;
    lbm_status s = validate(*p);
    if (s != LBM_OK) return s;
    if (!phi && !(phi_uniform > 0 && phi_uniform <= 1))
        return fail(LBM_E_INVAL, "phi_uniform = %g outside (0, 1]", phi_uniform);
    if (!workspace) return fail(LBM_E_INVAL, "null workspace");
    if (reinterpret_cast<uintptr_t>(workspace) % kAlign)
        return fail(LBM_E_INVAL, "workspace is not %zu-byte aligned", kAlign);
    const bool med = phi != nullptr || K != nullptr;
    // the tape's length comes from the workspace size: as many checkpoints as fit
    Layout L = make_layout(*p, 1, med);
    int64_t nmax = 0;
    if (p->checkpoint_every > 0) {
        const size_t fixed = L.total - L.n_ckpt * L.state_bytes;
        if (ws_bytes < L.total)
            return fail(LBM_E_NOMEM, "workspace of %zu bytes < %zu needed", ws_bytes, L.total);
        const size_t nck = (ws_bytes - fixed) / L.state_bytes;
        nmax = int64_t(nck) * p->checkpoint_every;
        L = make_layout(*p, nmax, med);
    }
    if (ws_bytes < L.total)
        return fail(LBM_E_NOMEM, "workspace of %zu bytes < %zu needed", ws_bytes, L.total);
    lbm_ctx* c = new (std::nothrow) lbm_ctx();
    if (!c) return fail(LBM_E_NOMEM, "host allocation failed");
    s = setup_ctx(c, *p, L, nmax, phi, K, phi_uniform, workspace, hip_stream);
    if (s != LBM_OK) {
        delete c;
        return s;
    }
    *out = c;
    return LBM_OK;
}

lbm_status lbm_step(lbm_ctx* c, int64_t nsteps) {
    lbm_status s = check_ctx(c, false);
    if (s != LBM_OK) return s;
    if (nsteps < 0) return fail(LBM_E_INVAL, "nsteps < 0");
    const int C = c->p.checkpoint_every;
    if (C > 0 && c->step + nsteps > c->nsteps_max)
        return fail(LBM_E_STATE, "tape holds %lld steps; %lld + %lld requested",
                    (long long)c->nsteps_max, (long long)c->step, (long long)nsteps);
    int64_t left = nsteps;
    if (C == 0 && left >= 2 * kGraphSteps) {
        s = ensure_graph(c, c->cur);
        if (s != LBM_OK) return s;
        while (left >= kGraphSteps) {
            HIP_TRY(hipGraphLaunch(c->gexec[c->cur], c->stream), "graph launch");
            left -= kGraphSteps;
            c->step += kGraphSteps;
        }
    }
    // k steps per launch where they fit: with a tape, between checkpoints (the state at every
    // multiple of C goes to its checkpoint first)
    const int k = launch_steps(c);
    while (left > 0) {
        if (C > 0 && c->step % C == 0)
            HIP_TRY(hipMemcpyAsync(c->ckpt(size_t(c->step / C)), c->buf(c->cur),
                                   c->L.state_bytes, hipMemcpyDeviceToDevice, c->stream),
                    "checkpoint copy");
        const int64_t room = C > 0 ? C - c->step % C : left;   // steps to the next checkpoint
        if (k > 1 && left >= k && room >= k) {
            HIP_TRY(advance_k(c, k, c->cur, c->stream), "step launch");
            c->step += k;
            left -= k;
        } else {
            HIP_TRY(advance(c, c->cur, c->stream), "step launch");
            c->step += 1;
            left -= 1;
        }
        c->cur = 1 - c->cur;
    }
    return LBM_OK;
}

lbm_status lbm_observables(lbm_ctx* c, lbm_obs* o, void* ux, void* uy, void* p, void* T) {
    lbm_status s = check_ctx(c, false);
    if (s != LBM_OK) return s;
    if (!o) return fail(LBM_E_INVAL, "null lbm_obs");
    return observe_ctx(c, o, ux, uy, p, T);
}

lbm_status lbm_stream_function(lbm_ctx* c, void* psi) {
    lbm_status s = check_ctx(c, false);
    if (s != LBM_OK) return s;
    if (!psi) return fail(LBM_E_INVAL, "null psi");
    hipError_t e = with_types(c->p.dtype, [&](auto st, auto rt) {
        LBM_TYPES(st, rt)
        return launch_stream_function<S, R>(c->buf(c->cur), c->medp(), c->G, phys<R>(c),
                                            pop_layout(c), psi, c->stream);
    });
    if (e != hipSuccess) return hip_fail(e, "stream function launch");
    HIP_TRY(hipStreamSynchronize(c->stream), "synchronize");
    return LBM_OK;
}

lbm_status lbm_state_size(const lbm_ctx* c, size_t* bytes) {
    lbm_status s = check_ctx(c, false);
    if (s != LBM_OK) return s;
    if (!bytes) return fail(LBM_E_INVAL, "null argument");
    *bytes = c->L.state_bytes + 64;
    return LBM_OK;
}

// Saved layout: 64-byte header {magic, dtype, nx, ny, pitch, step, layout, plane stride} then
// the raw buffer.
lbm_status lbm_save(lbm_ctx* c, void* host_buf, size_t bytes) {
    lbm_status s = check_ctx(c, false);
    if (s != LBM_OK) return s;
    if (!host_buf || bytes < c->L.state_bytes + 64)
        return fail(LBM_E_INVAL, "buffer of %zu bytes < %zu", bytes, c->L.state_bytes + 64);
    int64_t hdr[8] = {0x4C424D50, c->p.dtype, c->p.nx, c->p.ny, c->G.pitch, c->step, c->p.layout,
                      c->G.plane};
    std::memcpy(host_buf, hdr, sizeof hdr);
    HIP_TRY(hipMemcpyAsync((char*)host_buf + 64, c->buf(c->cur), c->L.state_bytes,
                           hipMemcpyDeviceToHost, c->stream),
            "save copy");
    HIP_TRY(hipStreamSynchronize(c->stream), "synchronize");
    return LBM_OK;
}

lbm_status lbm_load(lbm_ctx* c, const void* host_buf, size_t bytes) {
    lbm_status s = check_ctx(c, false);
    if (s != LBM_OK) return s;
    if (c->p.checkpoint_every > 0)
        return fail(LBM_E_UNSUPPORTED, "loading a state into a context with a tape");
    if (!host_buf || bytes < c->L.state_bytes + 64)
        return fail(LBM_E_INVAL, "buffer of %zu bytes < %zu", bytes, c->L.state_bytes + 64);
    int64_t hdr[8];
    std::memcpy(hdr, host_buf, sizeof hdr);
    if (hdr[0] != 0x4C424D50 || hdr[1] != c->p.dtype || hdr[2] != c->p.nx || hdr[3] != c->p.ny ||
        hdr[4] != c->G.pitch || hdr[6] != c->p.layout || hdr[7] != c->G.plane || hdr[5] < 0)
        return fail(LBM_E_INVAL, "saved state does not match this context");
    HIP_TRY(hipMemcpyAsync(c->buf(c->cur), (const char*)host_buf + 64, c->L.state_bytes,
                           hipMemcpyHostToDevice, c->stream),
            "load copy");
    HIP_TRY(hipStreamSynchronize(c->stream), "synchronize");
    c->step = hdr[5];
    if (c->p.layout == LBM_LAYOUT_AA) c->cur = int(c->step % 2);  // the form the state is in
    return LBM_OK;
}

lbm_status lbm_grad(lbm_ctx* c, double dJ, void* dJ_dphi, void* dJ_dK) {
    lbm_status s = check_ctx(c, false);
    if (s != LBM_OK) return s;
    if (c->p.checkpoint_every <= 0)
        return fail(LBM_E_STATE, "no adjoint tape (checkpoint_every = 0)");
    if (!std::isfinite(dJ)) return fail(LBM_E_INVAL, "dJ is not finite");
    const size_t esz = storage_bytes(c->p.dtype);
    const size_t nel = c->L.state_bytes / esz;
    const int64_t N = c->step;
    const int64_t C = c->p.checkpoint_every;
    hipStream_t st = c->stream;
    double* gphi = c->gacc(0);
    double* gK = c->gacc(1);
    HIP_TRY(launch_fill_f64(gphi, 2 * size_t(c->G.plane), st), "zero gradients");
    for (int b = 0; b < 2; ++b)
        HIP_TRY(esz == 8 ? launch_fill<double>(c->lam(b), nel, st)
                         : launch_fill<float>(c->lam(b), nel, st),
                "zero adjoint");
    int lc = 0;  // buffer holding the adjoint of the latest state
    if (N > 0) {
        if (!c->aux) {
            HIP_TRY(hipStreamCreateWithFlags(&c->aux, hipStreamNonBlocking), "stream create");
            for (int b = 0; b < 2; ++b) {
                HIP_TRY(hipEventCreateWithFlags(&c->ev_rec[b], hipEventDisableTiming), "event");
                HIP_TRY(hipEventCreateWithFlags(&c->ev_bwd[b], hipEventDisableTiming), "event");
            }
            HIP_TRY(hipEventCreateWithFlags(&c->ev_go, hipEventDisableTiming), "event");
        }
        hipStream_t aux = c->aux;
        const double LdT = c->d.L / c->d.dT;
        HIP_TRY(with_types(c->p.dtype,
                           [&](auto stt, auto rt) {
                               LBM_TYPES(stt, rt)
                               return launch_adjoint_seed<S, R>(c->buf(c->cur), c->lam(lc), c->G,
                                                                phys<R>(c), LdT, st);
                           }),
                "adjoint seed");
        const int64_t nseg = (N + C - 1) / C;
        // X^{n0} .. X^{n0+len-1} of segment sg, recomputed from its checkpoint into bank sg % 2
        auto recompute = [&](int64_t sg) -> hipError_t {
            const int bank = int(sg & 1);
            const int64_t len = std::min<int64_t>(C, N - sg * C);
            hipError_t e = hipMemcpyAsync(c->seg(bank, 0), c->ckpt(size_t(sg)),
                                          c->L.state_bytes, hipMemcpyDeviceToDevice, aux);
            for (int64_t k = 1; k < len && e == hipSuccess; ++k)
                e = step_once(c, c->seg(bank, size_t(k - 1)), c->seg(bank, size_t(k)), aux);
            if (e == hipSuccess) e = hipEventRecord(c->ev_rec[bank], aux);
            return e;
        };
        // The backward sweep of segment sg (on the caller's stream) overlaps the recompute of
        // segment sg - 1 (on aux); a bank is recomputed only after the sweep that last read it.
        auto sweep = [&]() -> lbm_status {
            HIP_TRY(hipEventRecord(c->ev_go, st), "event");
            HIP_TRY(hipStreamWaitEvent(aux, c->ev_go, 0), "stream wait");
            HIP_TRY(recompute(nseg - 1), "recompute launch");
            for (int64_t sg = nseg - 1; sg >= 0; --sg) {
                const int bank = int(sg & 1);
                const int64_t len = std::min<int64_t>(C, N - sg * C);
                if (sg > 0) {
                    if (sg + 1 < nseg)
                        HIP_TRY(hipStreamWaitEvent(aux, c->ev_bwd[1 - bank], 0), "stream wait");
                    HIP_TRY(recompute(sg - 1), "recompute launch");
                }
                HIP_TRY(hipStreamWaitEvent(st, c->ev_rec[bank], 0), "stream wait");
                for (int64_t k = len - 1; k >= 0; --k) {
                    const void* X = c->seg(bank, size_t(k));
                    HIP_TRY(with_types(c->p.dtype,
                                       [&](auto stt, auto rt) {
                                           LBM_TYPES(stt, rt)
                                           return launch_adjoint_step<S, R>(
                                               X, c->lam(lc), c->lam(1 - lc), c->medp(), gphi,
                                               gK, c->G, phys<R>(c), st);
                                       }),
                            "adjoint step launch");
                    lc = 1 - lc;
                }
                HIP_TRY(hipEventRecord(c->ev_bwd[bank], st), "event");
            }
            return LBM_OK;
        };
        const lbm_status st_out = sweep();
        if (st_out != LBM_OK) {
            // leave no work in flight on the second stream
            (void)hipStreamSynchronize(aux);
            (void)hipStreamSynchronize(st);
            return st_out;
        }
    }
    if (dJ_dphi)
        HIP_TRY(launch_unpitch_scale((double*)dJ_dphi, gphi, c->G, dJ, st), "gradient copy");
    if (dJ_dK)
        HIP_TRY(launch_unpitch_scale((double*)dJ_dK, gK, c->G, dJ, st), "gradient copy");
    HIP_TRY(hipStreamSynchronize(st), "synchronize");
    return LBM_OK;
}

lbm_status lbm_destroy(lbm_ctx* c) {
    if (!c) return LBM_OK;
    hipError_t e = c->stream ? hipStreamSynchronize(c->stream) : hipDeviceSynchronize();
    if (c->aux) (void)hipStreamSynchronize(c->aux);
    for (int i = 0; i < 2; ++i)
        if (c->gexec[i]) (void)hipGraphExecDestroy(c->gexec[i]);
    if (c->cap) (void)hipStreamDestroy(c->cap);
    for (int i = 0; i < 2; ++i) {
        if (c->ev_rec[i]) (void)hipEventDestroy(c->ev_rec[i]);
        if (c->ev_bwd[i]) (void)hipEventDestroy(c->ev_bwd[i]);
    }
    if (c->ev_go) (void)hipEventDestroy(c->ev_go);
    if (c->aux) (void)hipStreamDestroy(c->aux);
    delete c;
    if (e != hipSuccess) return hip_fail(e, "lbm_destroy");
    return LBM_OK;
}

lbm_status lbm_batch_workspace_size(int32_t n, const lbm_params* p, size_t* bytes) {
    if (!p || !bytes) return fail(LBM_E_INVAL, "null argument");
    BatchLayout L;
    lbm_status s = batch_layout(n, p, &L);
    if (s != LBM_OK) return s;
    *bytes = L.total;
    return LBM_OK;
}

lbm_status lbm_batch_init(lbm_ctx** out, int32_t n, const lbm_params* p,
                          const double* phi_uniform, void* workspace, size_t ws_bytes,
                          void* hip_stream, const char* tune_cache_path) {
    if (!out || !p || !phi_uniform) return fail(LBM_E_INVAL, "null argument");
    *out = nullptr;
    BatchLayout L;
    lbm_status s = batch_layout(n, p, &L);
    if (s != LBM_OK) return s;
    for (int i = 0; i < n; ++i)
        if (!(phi_uniform[i] > 0 && phi_uniform[i] <= 1))
            return fail(LBM_E_INVAL, "phi_uniform[%d] = %g outside (0, 1]", i, phi_uniform[i]);
    if (!workspace) return fail(LBM_E_INVAL, "null workspace");
    if (reinterpret_cast<uintptr_t>(workspace) % kAlign)
        return fail(LBM_E_INVAL, "workspace is not %zu-byte aligned", kAlign);
    if (ws_bytes < L.total)
        return fail(LBM_E_NOMEM, "workspace of %zu bytes < %zu needed", ws_bytes, L.total);
    lbm_ctx* c = new (std::nothrow) lbm_ctx();
    if (!c) return fail(LBM_E_NOMEM, "host allocation failed");
    c->batch = true;
    c->p = p[0];
    c->ncav = n;
    c->stream = (hipStream_t)hip_stream;
    c->ws = (char*)workspace;
    c->b_state_bytes = L.state_bytes;
    c->b_off_buf[0] = L.off_buf[0];
    c->b_off_buf[1] = L.off_buf[1];
    c->b_off_cav = L.off_cav;
    c->b_off_phys = L.off_phys;
    c->b_off_tiles = L.off_tiles;
    c->b_off_part = L.off_part;
    c->b_max_tiles = L.max_tiles;
    c->b_off_cav2 = L.off_cav2;
    c->b_off_tbwg = L.off_tbwg;
    c->b_max_tbwg = L.max_tbwg;
    c->bp.assign(p, p + n);
    c->boff = L.off;
    for (int i = 0; i < n; ++i) {
        const Derived d = derive(p[i]);
        c->bG.push_back(make_geo(p[i]));
        c->bP32.push_back(make_phys<float>(p[i], d, phi_uniform[i]));
        c->bP64.push_back(make_phys<double>(p[i], d, phi_uniform[i]));
        c->bLdT.push_back(d.L / d.dT);
    }
    // the parameter table in the arithmetic type
    const bool r64 = p[0].dtype != LBM_FP32;
    hipError_t e = r64 ? hipMemcpy(c->ws + L.off_phys, c->bP64.data(), n * sizeof(Phys<double>),
                                   hipMemcpyHostToDevice)
                       : hipMemcpy(c->ws + L.off_phys, c->bP32.data(), n * sizeof(Phys<float>),
                                   hipMemcpyHostToDevice);
    if (e == hipSuccess) e = batch_rest(c);
    if (e != hipSuccess) {
        delete c;
        return hip_fail(e, "lbm_batch_init");
    }
    with_types(p[0].dtype, [&](auto st, auto rt) {
        LBM_TYPES(st, rt)
        prepare_batch_tb2<S, R>();
        return 0;
    });
    s = batch_tune(c, tune_cache_path);
    if (s == LBM_OK) {
        hipError_t e2 = batch_rest(c);  // tuning stepped the cavities: back to rest
        if (e2 == hipSuccess) e2 = hipStreamSynchronize(c->stream);
        if (e2 != hipSuccess) s = hip_fail(e2, "lbm_batch_init");
    }
    if (s != LBM_OK) {
        lbm_destroy(c);
        return s;
    }
    c->step = 0;
    c->cur = 0;
    *out = c;
    return LBM_OK;
}

lbm_status lbm_batch_step(lbm_ctx* c, int64_t nsteps) {
    lbm_status s = check_ctx(c, true);
    if (s != LBM_OK) return s;
    if (nsteps < 0) return fail(LBM_E_INVAL, "nsteps < 0");
    int64_t left = nsteps;
    if (left >= kBatchGraphSteps) {
        s = ensure_batch_graph(c, c->cur);
        if (s != LBM_OK) return s;
        while (left >= kBatchGraphSteps) {
            HIP_TRY(hipGraphLaunch(c->gexec[c->cur], c->stream), "graph launch");
            left -= kBatchGraphSteps;
            c->step += kBatchGraphSteps;
        }
    }
    if (c->b_tb_rows > 0) {
        for (; left >= 2; left -= 2) {
            HIP_TRY(batch_step2(c, c->cur, c->stream), "batch step launch");
            c->cur = 1 - c->cur;
            c->step += 2;
        }
    }
    for (; left > 0; --left) {
        HIP_TRY(batch_step_once(c, c->cur, c->stream), "batch step launch");
        c->cur = 1 - c->cur;
        c->step += 1;
    }
    return LBM_OK;
}

lbm_status lbm_batch_observables(lbm_ctx* c, lbm_obs* o) {
    lbm_status s = check_ctx(c, true);
    if (s != LBM_OK) return s;
    if (!o) return fail(LBM_E_INVAL, "null lbm_obs");
    const int n = c->ncav;
    const size_t esz = storage_bytes(c->p.dtype);
    double* part0 = (double*)(c->ws + c->b_off_part);
    const size_t per = kBatchObsPer;
    char* base = c->ws + c->b_off_buf[c->cur];
    for (int i = 0; i < n; ++i) {
        const void* src = base + size_t(c->boff[i]) * esz;
        double* part = part0 + i * per;
        double* res = part + kObsParts * kBatchObsWG;
        hipError_t e = with_types(c->p.dtype, [&](auto st, auto rt) {
            LBM_TYPES(st, rt)
            return launch_observe<S, R>(src, nullptr, c->bG[i], bphys<R>(c, i), kPull, nullptr,
                                        nullptr, nullptr, nullptr, part, kBatchObsWG, c->bLdT[i],
                                        res, c->stream);
        });
        if (e != hipSuccess) return hip_fail(e, "batch observables launch");
    }
    std::vector<double> h(size_t(n) * per);
    HIP_TRY(hipMemcpyAsync(h.data(), part0, h.size() * sizeof(double), hipMemcpyDeviceToHost,
                           c->stream),
            "readback");
    HIP_TRY(hipStreamSynchronize(c->stream), "synchronize");
    bool any = false;
    for (int i = 0; i < n; ++i) {
        const double* r = h.data() + i * per + kObsParts * kBatchObsWG;
        fill_obs(c->bp[i], derive(c->bp[i]), c->step, r, &o[i]);
        any = any || o[i].diverged;
    }
    if (any) return fail(LBM_E_DIVERGED, "a cavity diverged at step %lld", (long long)c->step);
    return LBM_OK;
}

lbm_status lbm_batch_fields(lbm_ctx* c, int32_t i, void* ux, void* uy, void* p, void* T) {
    lbm_status s = check_ctx(c, true);
    if (s != LBM_OK) return s;
    if (i < 0 || i >= c->ncav) return fail(LBM_E_INVAL, "cavity %d of %d", i, c->ncav);
    const size_t esz = storage_bytes(c->p.dtype);
    const void* src = c->ws + c->b_off_buf[c->cur] + size_t(c->boff[i]) * esz;
    double* part = (double*)(c->ws + c->b_off_part) + size_t(i) * kBatchObsPer;
    double* res = part + kObsParts * kBatchObsWG;
    hipError_t e = with_types(c->p.dtype, [&](auto st, auto rt) {
        LBM_TYPES(st, rt)
        return launch_observe<S, R>(src, nullptr, c->bG[i], bphys<R>(c, i), kPull, ux, uy, p, T,
                                    part, kBatchObsWG, c->bLdT[i], res, c->stream);
    });
    if (e != hipSuccess) return hip_fail(e, "batch fields launch");
    HIP_TRY(hipStreamSynchronize(c->stream), "synchronize");
    return LBM_OK;
}

lbm_status lbm_step_shape(const lbm_ctx* c, int32_t* out) {
    lbm_status s = check_ctx(c, false);
    if (s != LBM_OK) return s;
    if (!out) return fail(LBM_E_INVAL, "null argument");
    const int k = launch_steps(c);
    out[0] = k;
    out[1] = c->p.layout;
    out[2] = 0;
    out[3] = (c->G.nx + kTileX - 1) / kTileX * c->G.ny;
    if (k == kTileSteps || k == kTinyTileSteps) {
        const int ts = tile_side(k);
        out[2] = ts;
        out[3] = (c->G.nx + ts - 1) / ts * ((c->G.ny + ts - 1) / ts);
    }
    if (k == 2 || k == 3)
        (void)with_types(c->p.dtype, [&](auto st, auto rt) {
            LBM_TYPES(st, rt)
            int rows = 0, nseg = 0, nwg = 0;
            if (k == 2)
                tb2_shape<S, R>(c->G, c->med, &rows, &nwg);
            else
                tb3_shape<S, R>(c->G, c->med, &rows, &nseg, &nwg);
            out[2] = rows;
            out[3] = nwg;
            return 0;
        });
    return LBM_OK;
}

lbm_status lbm_batch_shape(const lbm_ctx* c, int32_t* out) {
    lbm_status s = check_ctx(c, true);
    if (s != LBM_OK) return s;
    if (!out) return fail(LBM_E_INVAL, "null argument");
    out[0] = c->b_npt;
    out[1] = 64 * c->b_wg;
    out[2] = c->b_nwg;
    out[3] = kBatchGraphSteps;
    out[4] = c->b_tb_rows > 0 ? 2 : 1;
    out[5] = c->b_tb_rows;
    out[6] = c->b_tb_nwg;
    out[7] = c->b_tb_rows > 0 ? c->b_tb_waves : 0;
    return LBM_OK;
}

lbm_status lbm_run_noalloc(const lbm_params* p, const void* phi, const void* K,
                           double phi_uniform, int64_t nsteps, lbm_obs* o, void* ux, void* uy,
                           void* pr, void* T, void* hip_stream) {
    if (!p || !o) return fail(LBM_E_INVAL, "null argument");
    lbm_status s = validate(*p);
    if (s != LBM_OK) return s;
    if (p->checkpoint_every != 0)
        return fail(LBM_E_UNSUPPORTED, "lbm_run_noalloc keeps no adjoint tape");
    if (nsteps < 0) return fail(LBM_E_INVAL, "nsteps < 0");
    if (!phi && !(phi_uniform > 0 && phi_uniform <= 1))
        return fail(LBM_E_INVAL, "phi_uniform = %g outside (0, 1]", phi_uniform);
    const Layout L = make_layout(*p, 1, phi != nullptr || K != nullptr);
    if (L.total > kNoAllocBytes)
        return fail(LBM_E_NOMEM,
                    "a %d x %d cavity needs %zu bytes of device memory; lbm_run_noalloc holds "
                    "at most %zu",
                    p->nx, p->ny, L.total, kNoAllocBytes);
    void* ws = nullptr;
    s = scratch_address(&ws);
    if (s != LBM_OK) return s;
    lbm_ctx c;  // on the stack: no host allocation either
    s = setup_ctx(&c, *p, L, 0, phi, K, phi_uniform, ws, hip_stream);
    if (s != LBM_OK) return s;
    int64_t left = nsteps;
    const int k = launch_steps(&c);
    if (k > 1) {
        for (; left >= k; left -= k) {
            HIP_TRY(advance_k(&c, k, c.cur, c.stream), "step launch");
            c.cur = 1 - c.cur;
            c.step += k;
        }
    }
    for (; left > 0; --left) {
        HIP_TRY(advance(&c, c.cur, c.stream), "step launch");
        c.cur = 1 - c.cur;
        c.step += 1;
    }
    return observe_ctx(&c, o, ux, uy, pr, T);
}

}  // extern "C"
