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
    double L, cs2, csT2, tau_v, tau_T, nu_e, nu, gbeta, dT, T0, K;
};

Derived derive(const lbm_params& p) {
    Derived d;
    d.L = double(p.nx - 1);
    d.cs2 = 1.0 / 3.0;
    d.csT2 = (4.0 + p.varpi) / 10.0;
    // Eq. (37b)
    d.tau_v = p.tau_v > 0 ? p.tau_v : 0.5 + p.Ma * p.J * d.L * std::sqrt(p.Pr / p.Ra) *
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
    return d;
}

bool walled(const lbm_params& p, int side) { return p.bc[side] != LBM_PERIODIC; }

lbm_status validate(const lbm_params& p) {
    if (p.dtype != LBM_FP32 && p.dtype != LBM_FP64)
        return fail(LBM_E_INVAL, "dtype %d is neither LBM_FP32 nor LBM_FP64", p.dtype);
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
    if (pitch * (long long)p.ny * kPlanes >= (1LL << 31))
        return fail(LBM_E_INVAL, "grid %d x %d exceeds the 2^31-element state limit", p.nx, p.ny);
    if (!(p.rho0 > 0) || !(p.sigma > 0) || !(p.J > 0))
        return fail(LBM_E_INVAL, "rho0, sigma and J must be positive");
    if (!(p.varpi < 1) || !(p.varpi > -4))
        return fail(LBM_E_INVAL, "varpi = %g must lie in (-4, 1) (Eq. (29))", p.varpi);
    if (p.tau_v <= 0 && (!(p.Ra > 0) || !(p.Pr > 0) || !(p.Ma > 0)))
        return fail(LBM_E_INVAL, "Ra, Pr and Ma must be positive to derive tau_v");
    if (p.tau_T <= 0 && !(p.Pr > 0))
        return fail(LBM_E_INVAL, "Pr must be positive to derive tau_T");
    if (p.checkpoint_every < 0) return fail(LBM_E_INVAL, "checkpoint_every must be >= 0");
    const Derived d = derive(p);
    if (!(d.tau_v > 0.5) || !std::isfinite(d.tau_v))
        return fail(LBM_E_INVAL, "tau_v = %.17g must exceed 1/2", d.tau_v);
    if (!(d.tau_T > 0.5) || !std::isfinite(d.tau_T))
        return fail(LBM_E_INVAL, "tau_T = %.17g must exceed 1/2", d.tau_T);
    if (!std::isfinite(d.gbeta)) return fail(LBM_E_INVAL, "g*beta is not finite");
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
    G.plane = G.pitch * p.ny;
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
    size_t off_seg;       // C states of one segment
    size_t off_lam[2];
    size_t off_gacc;      // 2 FP64 planes
    size_t total;
};

Layout make_layout(const lbm_params& p, int64_t nsteps_max, bool med_planes) {
    const Geo G = make_geo(p);
    const size_t esz = p.dtype == LBM_FP64 ? 8 : 4;
    Layout L{};
    L.state_bytes = align_up(size_t(kPlanes) * G.plane * esz);
    size_t o = 0;
    L.off_buf[0] = o;
    o += L.state_bytes;
    L.off_buf[1] = o;
    o += L.state_bytes;
    L.off_med = o;
    if (med_planes) o += align_up(2 * size_t(G.plane) * esz);
    L.off_part = o;
    o += align_up((3 * kObserveWG + 16) * sizeof(double));
    L.off_tape = o;
    if (p.checkpoint_every > 0) {
        const size_t C = size_t(p.checkpoint_every);
        L.n_ckpt = std::max<size_t>(1, (size_t(std::max<int64_t>(nsteps_max, 1)) + C - 1) / C);
        o += L.n_ckpt * L.state_bytes;
        L.off_seg = o;
        o += C * L.state_bytes;
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
    // batched form
    int ncav = 0;
    std::vector<lbm_params> bp;
    std::vector<double> bphi;
    std::vector<BatchCavity> bcav;
    size_t b_off_cav = 0, b_off_phys = 0, b_off_obs = 0;
    int b_ntiles = 0;
    int b_shape[4] = {0, 0, 0, 0};

    void* buf(int i) const { return ws + L.off_buf[i]; }
    void* medp() const { return med ? ws + L.off_med : nullptr; }
    double* part() const { return (double*)(ws + L.off_part); }
    void* ckpt(size_t k) const { return ws + L.off_tape + k * L.state_bytes; }
    void* seg(size_t k) const { return ws + L.off_seg + k * L.state_bytes; }
    void* lam(int i) const { return ws + L.off_lam[i]; }
    double* gacc(int i) const { return (double*)(ws + L.off_gacc) + size_t(i) * G.plane; }
};

namespace {

lbm_status check_ctx(const lbm_ctx* c, bool want_batch) {
    if (!c) return fail(LBM_E_INVAL, "null context");
    if (c->batch != want_batch)
        return fail(LBM_E_INVAL, want_batch ? "context is not a batch" : "context is a batch");
    return LBM_OK;
}

hipError_t step_once(lbm_ctx* c, const void* src, void* dst, hipStream_t s) {
    if (c->p.dtype == LBM_FP64) return launch_step<double>(src, dst, c->medp(), c->G, c->P64, s);
    return launch_step<float>(src, dst, c->medp(), c->G, c->P32, s);
}

// Capture kGraphSteps launches (an even count, so the buffers end where they started) into an
// executable graph for the given starting buffer.
constexpr int kGraphSteps = 64;

lbm_status ensure_graph(lbm_ctx* c, int start) {
    if (c->gexec[start]) return LBM_OK;
    if (!c->cap) HIP_TRY(hipStreamCreateWithFlags(&c->cap, hipStreamNonBlocking), "stream create");
    HIP_TRY(hipStreamBeginCapture(c->cap, hipStreamCaptureModeThreadLocal), "begin capture");
    hipError_t err = hipSuccess;
    int b = start;
    for (int k = 0; k < kGraphSteps && err == hipSuccess; ++k) {
        err = step_once(c, c->buf(b), c->buf(1 - b), c->cap);
        b = 1 - b;
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
    p->dtype = LBM_FP32;
    p->checkpoint_every = 0;
    g_err.clear();
    return LBM_OK;
}

lbm_status lbm_derived(const lbm_params* p, double* out) {
    if (!p || !out) return fail(LBM_E_INVAL, "null argument");
    const Derived d = derive(*p);
    const double v[9] = {d.L, d.tau_v, d.tau_T, d.nu_e, d.nu, d.gbeta, d.dT, d.T0, d.K};
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
    c->p = *p;
    c->d = derive(*p);
    c->G = make_geo(*p);
    c->L = L;
    c->stream = (hipStream_t)hip_stream;
    c->ws = (char*)workspace;
    c->med = med;
    c->nsteps_max = nmax;
    c->phi_u = phi ? 1.0 : phi_uniform;
    c->P32 = make_phys<float>(*p, c->d, c->phi_u);
    c->P64 = make_phys<double>(*p, c->d, c->phi_u);
    const double g0 = (1.0 - p->varpi) / 5.0 * (p->T_init - c->d.T0);
    const double g1 = (4.0 + p->varpi) / 20.0 * (p->T_init - c->d.T0);
    hipError_t e = hipSuccess;
    const bool f64 = p->dtype == LBM_FP64;
    if (med) {
        char* mp = c->ws + L.off_med;
        const size_t plane_bytes = size_t(c->G.plane) * (f64 ? 8 : 4);
        const double Kv = std::isinf(c->d.K) ? 1e300 : c->d.K;
        if (f64) {
            e = launch_pitch_copy<double>(mp, phi, c->G, phi_uniform, c->stream);
            if (e == hipSuccess)
                e = launch_pitch_copy<double>(mp + plane_bytes, K, c->G, Kv, c->stream);
        } else {
            e = launch_pitch_copy<float>(mp, phi, c->G, phi_uniform, c->stream);
            if (e == hipSuccess)
                e = launch_pitch_copy<float>(mp + plane_bytes, K, c->G, std::isinf(c->d.K) ? 1e30
                                                                                          : Kv,
                                             c->stream);
        }
    }
    // both buffers, so that the row padding (never written by a step) is defined too
    for (int b = 0; b < 2 && e == hipSuccess; ++b)
        e = f64 ? launch_rest<double>(c->buf(b), c->G, g0, g1, c->stream)
                : launch_rest<float>(c->buf(b), c->G, g0, g1, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) {
        delete c;
        return hip_fail(e, "lbm_init");
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
    for (; left > 0; --left) {
        if (C > 0 && c->step % C == 0)
            HIP_TRY(hipMemcpyAsync(c->ckpt(size_t(c->step / C)), c->buf(c->cur),
                                   c->L.state_bytes, hipMemcpyDeviceToDevice, c->stream),
                    "checkpoint copy");
        HIP_TRY(step_once(c, c->buf(c->cur), c->buf(1 - c->cur), c->stream), "step launch");
        c->cur = 1 - c->cur;
        c->step += 1;
    }
    return LBM_OK;
}

lbm_status lbm_observables(lbm_ctx* c, lbm_obs* o, void* ux, void* uy, void* p, void* T) {
    lbm_status s = check_ctx(c, false);
    if (s != LBM_OK) return s;
    if (!o) return fail(LBM_E_INVAL, "null lbm_obs");
    double* part = c->part();
    double* res = part + 3 * kObserveWG;
    const double LdT = c->d.L / c->d.dT;
    hipError_t e = c->p.dtype == LBM_FP64
                       ? launch_observe<double>(c->buf(c->cur), c->medp(), c->G, c->P64, ux, uy,
                                                p, T, part, kObserveWG, LdT, res, c->stream)
                       : launch_observe<float>(c->buf(c->cur), c->medp(), c->G, c->P32, ux, uy,
                                               p, T, part, kObserveWG, LdT, res, c->stream);
    if (e != hipSuccess) return hip_fail(e, "observables launch");
    double h[5];
    HIP_TRY(hipMemcpyAsync(h, res, sizeof h, hipMemcpyDeviceToHost, c->stream), "readback");
    HIP_TRY(hipStreamSynchronize(c->stream), "synchronize");
    const double n = double(c->p.nx) * c->p.ny;
    o->nu_hot = h[0];
    o->nu_cold = h[1];
    o->max_speed = h[2];
    o->mass_err = std::fabs(h[3]) / (n * c->p.rho0);
    o->step = c->step;
    o->diverged = (h[4] != 0.0 || !(h[2] <= std::sqrt(1.0 / 3.0)) || !std::isfinite(h[0]) ||
                   !std::isfinite(h[1]))
                      ? 1
                      : 0;
    o->pad_ = 0;
    if (o->diverged) return fail(LBM_E_DIVERGED, "diverged at step %lld", (long long)c->step);
    return LBM_OK;
}

lbm_status lbm_state_size(const lbm_ctx* c, size_t* bytes) {
    lbm_status s = check_ctx(c, false);
    if (s != LBM_OK) return s;
    if (!bytes) return fail(LBM_E_INVAL, "null argument");
    *bytes = c->L.state_bytes + 64;
    return LBM_OK;
}

// Saved layout: 64-byte header {magic, dtype, nx, ny, pitch, step} then the raw buffer.
lbm_status lbm_save(lbm_ctx* c, void* host_buf, size_t bytes) {
    lbm_status s = check_ctx(c, false);
    if (s != LBM_OK) return s;
    if (!host_buf || bytes < c->L.state_bytes + 64)
        return fail(LBM_E_INVAL, "buffer of %zu bytes < %zu", bytes, c->L.state_bytes + 64);
    int64_t hdr[8] = {0x4C424D50, c->p.dtype, c->p.nx, c->p.ny, c->G.pitch, c->step, 0, 0};
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
        hdr[4] != c->G.pitch)
        return fail(LBM_E_INVAL, "saved state does not match this context");
    HIP_TRY(hipMemcpyAsync(c->buf(c->cur), (const char*)host_buf + 64, c->L.state_bytes,
                           hipMemcpyHostToDevice, c->stream),
            "load copy");
    HIP_TRY(hipStreamSynchronize(c->stream), "synchronize");
    c->step = hdr[5];
    return LBM_OK;
}

lbm_status lbm_grad(lbm_ctx* c, double dJ, void* dJ_dphi, void* dJ_dK) {
    lbm_status s = check_ctx(c, false);
    if (s != LBM_OK) return s;
    (void)dJ;
    (void)dJ_dphi;
    (void)dJ_dK;
    if (c->p.checkpoint_every <= 0) return fail(LBM_E_STATE, "no adjoint tape (checkpoint_every = 0)");
    return fail(LBM_E_UNSUPPORTED, "adjoint not built");
}

lbm_status lbm_destroy(lbm_ctx* c) {
    if (!c) return LBM_OK;
    hipError_t e = c->stream ? hipStreamSynchronize(c->stream) : hipDeviceSynchronize();
    for (int i = 0; i < 2; ++i)
        if (c->gexec[i]) (void)hipGraphExecDestroy(c->gexec[i]);
    if (c->cap) (void)hipStreamDestroy(c->cap);
    delete c;
    if (e != hipSuccess) return hip_fail(e, "lbm_destroy");
    return LBM_OK;
}

lbm_status lbm_batch_workspace_size(int32_t n, const lbm_params* p, size_t* bytes) {
    (void)n;
    (void)p;
    (void)bytes;
    return fail(LBM_E_UNSUPPORTED, "batched form not built");
}

lbm_status lbm_batch_init(lbm_ctx** out, int32_t n, const lbm_params* p,
                          const double* phi_uniform, void* workspace, size_t ws_bytes,
                          void* hip_stream, const char* tune_cache_path) {
    (void)out; (void)n; (void)p; (void)phi_uniform; (void)workspace; (void)ws_bytes;
    (void)hip_stream; (void)tune_cache_path;
    return fail(LBM_E_UNSUPPORTED, "batched form not built");
}

lbm_status lbm_batch_step(lbm_ctx* c, int64_t nsteps) {
    (void)c; (void)nsteps;
    return fail(LBM_E_UNSUPPORTED, "batched form not built");
}

lbm_status lbm_batch_observables(lbm_ctx* c, lbm_obs* o) {
    (void)c; (void)o;
    return fail(LBM_E_UNSUPPORTED, "batched form not built");
}

lbm_status lbm_batch_shape(const lbm_ctx* c, int32_t* out) {
    (void)c; (void)out;
    return fail(LBM_E_UNSUPPORTED, "batched form not built");
}

}  // extern "C"
