// lbm_adjoint.hip -- discrete adjoint of the fused time step: the exact vector-Jacobian product
// of one step of the forward map (streaming, wall reconstruction, macroscopic recovery,
// collision; Eqs. (18), (35), (36), (22), (21), (23), (4), (17), (34) of arXiv:1308.2071), plus
// the accumulation of dJ/dphi and dJ/dK at every node, and the seed of J = Nu_hot (Eq. (38)).
//
// Race freedom without atomics: in the forward pull, node x reads slot (i, x - e_i) of the
// previous state, and the map x -> (i, x - e_i) is a bijection; a wall node reads nothing of its
// own slots but the slots of its inward neighbour x_f.  So the thread of node x writes the
// adjoint of exactly its own slots: its own collision's contribution plus the contributions of
// every wall node whose inward neighbour is x, which the wall nodes' threads hand over through
// LDS.  Wall threads write zeros to their own slots.
#include "lbm_device.hpp"
#include "lbm_internal.hpp"

namespace lbm {

// Adjoints of the macroscopic quantities a collision consumes.
template <typename R>
struct MacAdj {
    R theta, ux, uy, P, Fx, Fy, ip;
};

// Reverse of collide(): given the adjoints lf, lg of the post-collision populations, adds the
// adjoints of the post-streaming populations to af, ag and of the macroscopics to A.
template <typename R>
__device__ __forceinline__ void collide_vjp(const R f[9], const R g[5], const Mac<R>& m,
                                            const Med<R>& md, const Phys<R>& P, const R lf[9],
                                            const R lg[5], R af[9], R ag[5], MacAdj<R>& A) {
    const R r0 = P.rho0, ux = m.ux, uy = m.uy, Fx = m.Fx, Fy = m.Fy;
    const R rip = r0 * md.inv_phi;
    const R uu = ux * ux + uy * uy;
    // f+ = M^T a  =>  adjoint of a = M lf (rows 1..8 of Eq. (11)), then the 1/|row|^2 scaling
    const R s14 = (lf[1] + lf[2]) + (lf[3] + lf[4]);
    const R s58 = (lf[5] + lf[6]) + (lf[7] + lf[8]);
    const R qx = (lf[5] - lf[6]) - (lf[7] - lf[8]);
    const R qy = (lf[5] + lf[6]) - (lf[7] + lf[8]);
    const R lA1 = (R(2) * s58 - s14 - R(4) * lf[0]) * R(1.0 / 36.0);
    const R lA2 = (s58 - R(2) * s14 + R(4) * lf[0]) * R(1.0 / 36.0);
    const R lA3 = ((lf[1] - lf[3]) + qx) * R(1.0 / 6.0);
    const R lA4 = (qx - R(2) * (lf[1] - lf[3])) * R(1.0 / 12.0);
    const R lA5 = ((lf[2] - lf[4]) + qy) * R(1.0 / 6.0);
    const R lA6 = (qy - R(2) * (lf[2] - lf[4])) * R(1.0 / 12.0);
    const R lA7 = ((lf[1] - lf[2]) + (lf[3] - lf[4])) * R(0.25);
    const R lA8 = ((lf[5] - lf[6]) + (lf[7] - lf[8])) * R(0.25);
    // relaxation (Eq. (17))
    const R lm1 = (R(1) - P.s_e) * lA1, lm2 = (R(1) - P.s_eps) * lA2;
    const R lm4 = (R(1) - P.s_q) * lA4, lm6 = (R(1) - P.s_q) * lA6;
    const R lm7 = (R(1) - P.s_v) * lA7, lm8 = (R(1) - P.s_v) * lA8;
    const R le = P.s_e * lA1, leps = P.s_eps * lA2;
    const R lpxx = P.s_v * lA7, lpxy = P.s_v * lA8;
    const R lS1 = P.os_e * lA1 - P.os_eps * lA2;
    const R lS7 = P.os_v * lA7, lS8 = P.os_v * lA8;
    R lux = r0 * lA3 - P.s_q * r0 * lA4;
    R luy = r0 * lA5 - P.s_q * r0 * lA6;
    R lFx = R(0.5) * r0 * lA3 - P.os_q * r0 * lA4;
    R lFy = R(0.5) * r0 * lA5 - P.os_q * r0 * lA6;
    // equilibrium moments (Eq. (16)) and forcing (Eq. (19))
    A.P += R(6) * le - R(9) * leps;
    const R lRU = R(3) * (le - leps);           // adjoint of rip * uu
    R lrip = lRU * uu;
    R luu = lRU * rip;
    lrip += lpxx * (ux * ux - uy * uy) + lpxy * ux * uy;
    lux += R(2) * rip * ux * lpxx + rip * uy * lpxy;
    luy += -R(2) * rip * uy * lpxx + rip * ux * lpxy;
    const R uF = ux * Fx + uy * Fy;
    const R luF = R(6) * rip * lS1;
    lrip += R(6) * uF * lS1 + R(2) * (ux * Fx - uy * Fy) * lS7 + (ux * Fy + uy * Fx) * lS8;
    lux += luF * Fx + R(2) * rip * Fx * lS7 + rip * Fy * lS8;
    luy += luF * Fy - R(2) * rip * Fy * lS7 + rip * Fx * lS8;
    lFx += luF * ux + R(2) * rip * ux * lS7 + rip * uy * lS8;
    lFy += luF * uy - R(2) * rip * uy * lS7 + rip * ux * lS8;
    lux += R(2) * ux * luu;
    luy += R(2) * uy * luu;
    A.ip += r0 * lrip;
    // moments m' = M f' (rows 1, 2, 4, 6, 7, 8)
    af[0] += R(-4) * lm1 + R(4) * lm2;
    af[1] += -lm1 - R(2) * lm2 - R(2) * lm4 + lm7;
    af[2] += -lm1 - R(2) * lm2 - R(2) * lm6 - lm7;
    af[3] += -lm1 - R(2) * lm2 + R(2) * lm4 + lm7;
    af[4] += -lm1 - R(2) * lm2 + R(2) * lm6 - lm7;
    af[5] += R(2) * lm1 + lm2 + lm4 + lm6 + lm8;
    af[6] += R(2) * lm1 + lm2 - lm4 + lm6 - lm8;
    af[7] += R(2) * lm1 + lm2 - lm4 - lm6 + lm8;
    af[8] += R(2) * lm1 + lm2 + lm4 - lm6 - lm8;

    // thermal (Eq. (34)): g+ = N^T b  =>  adjoint of b = N lg
    const R lb0 = (lg[0] + lg[1]) + (lg[2] + lg[3]) + lg[4];
    const R lb1 = lg[1] - lg[3];
    const R lb2 = lg[2] - lg[4];
    const R lb3 = (lg[1] + lg[2]) + (lg[3] + lg[4]) - R(4) * lg[0];
    const R lb4 = (lg[1] - lg[2]) + (lg[3] - lg[4]);
    const R T = P.T0 + m.theta;
    const R ln1 = R(0.5) * (R(1) - P.z_T) * lb1;
    const R ln2 = R(0.5) * (R(1) - P.z_T) * lb2;
    const R ln3 = R(0.05) * (R(1) - P.z3) * lb3;
    const R ln4 = R(0.25) * (R(1) - P.z4) * lb4;
    const R kz = R(0.5) * P.z_T * P.inv_sigma;
    lux += kz * T * lb1;
    luy += kz * T * lb2;
    A.theta += R(0.2) * lb0 + R(0.05) * P.z3 * P.varpi * lb3 + kz * (ux * lb1 + uy * lb2);
    ag[0] += R(-4) * ln3;
    ag[1] += ln1 + ln3 + ln4;
    ag[2] += ln2 + ln3 - ln4;
    ag[3] += -ln1 + ln3 + ln4;
    ag[4] += -ln2 + ln3 - ln4;
    A.ux += lux;
    A.uy += luy;
    A.Fx += lFx;
    A.Fy += lFy;
}

// Reverse of fluid_macros(): adds to af, ag and to the medium adjoints lphi, lK.
template <typename R>
__device__ __forceinline__ void macros_vjp(const R f[9], const R g[5], R phi, R K,
                                           const Med<R>& md, const Phys<R>& P,
                                           const MacAdj<R>& A0, R af[9], R ag[5], R& lphi,
                                           R& lK) {
    // forward recompute, exactly as the forward step computes it
    const Vel<R> v = velocity<R>(f, g, md, P);
    const R Gx = v.Gx, Gy = v.Gy, hphi = R(0.5) * phi;
    const R vx = v.vx, vy = v.vy, l0 = v.l0, l1 = v.l1, vm = v.vm, q = v.q;
    const R inv_den = R(1) / v.den;
    const R ux = v.ux, uy = v.uy, uu = v.uu, um = v.um, drag = v.drag;
    // reverse
    R lux = A0.ux, luy = A0.uy, lth = A0.theta, lip = A0.ip;
    R lGx = phi * A0.Fx, lGy = phi * A0.Fy;
    lphi += Gx * A0.Fx + Gy * A0.Fy;
    const R ldrag = -(ux * A0.Fx + uy * A0.Fy);
    lux -= drag * A0.Fx;
    luy -= drag * A0.Fy;
    R lclin = ldrag, lcnl = um * ldrag;
    const R lum = md.c_nl * ldrag;
    if (um > R(0)) {                  // d|u|/du, taken as 0 at u = 0
        lux += lum * ux / um;
        luy += lum * uy / um;
    }
    // P = 0.6 (sum18 - (2/3) rho0 uu / phi)
    const R lsum18 = R(0.6) * A0.P;
    const R luu = R(-0.4) * P.rho0 * md.inv_phi * A0.P;
    lip += R(-0.4) * P.rho0 * uu * A0.P;
    lux += R(2) * ux * luu;
    luy += R(2) * uy * luu;
    // u = v / den, den = l0 + sqrt(l0^2 + l1 |v|)
    R lvx = lux * inv_den, lvy = luy * inv_den;
    const R lden = -(lux * ux + luy * uy) * inv_den;
    const R lq = lden;
    const R ll0 = lden + lq * l0 / q;
    const R ll1 = lq * vm / (R(2) * q);
    const R lvm = lq * l1 / (R(2) * q);
    if (vm > R(0)) {                  // d|v|/dv, taken as 0 at v = 0
        lvx += lvm * vx / vm;
        lvy += lvm * vy / vm;
    }
    lclin += R(0.25) * ll0;
    lcnl += R(0.5) * ll1;
    // v = j / rho0 + phi G / 2
    lphi += R(0.5) * (Gx * lvx + Gy * lvy);
    lGx += hphi * lvx;
    lGy += hphi * lvy;
    const R ljx = lvx * P.inv_rho0, ljy = lvy * P.inv_rho0;
    lth += P.gbeta * lGy;
    (void)lGx;
    // medium: ip = 1/phi, c_lin = phi nu / K, c_nl = C phi^(-1/2) K^(-1/2)
    lphi += -md.inv_phi * md.inv_phi * lip;
    lphi += md.c_lin * md.inv_phi * lclin;
    lK += -md.c_lin / K * lclin;
    lphi += R(-0.5) * md.c_nl * md.inv_phi * lcnl;
    lK += R(-0.5) * md.c_nl / K * lcnl;
    // populations
    af[1] += ljx + lsum18;
    af[2] += ljy + lsum18;
    af[3] += -ljx + lsum18;
    af[4] += -ljy + lsum18;
    af[5] += ljx + ljy + lsum18;
    af[6] += -ljx + ljy + lsum18;
    af[7] += -ljx - ljy + lsum18;
    af[8] += ljx - ljy + lsum18;
#pragma unroll
    for (int i = 0; i < 5; ++i) ag[i] += lth;
}

// Reverse of nee_wall() with respect to the neighbour's macroscopics: given the adjoints lfb,
// lgb of the rebuilt wall populations, adds to A the adjoints of the neighbour's ux, uy, 1/phi
// and theta.  The neighbour's pulled populations receive lfb and lgb unchanged.  Returns
// sum_i wt_i lgb_i, the adjoint of the wall temperature theta_b through the rebuilt g.
template <typename R>
__device__ __forceinline__ R nee_vjp(const Mac<R>& mf, const Med<R>& mdf, const Phys<R>& P,
                                     const R lfb[9], const R lgb[5], MacAdj<R>& A) {
    const R ux = mf.ux, uy = mf.uy, ip = mdf.inv_phi, r0 = P.rho0;
    // f_b,i = f_f,i - rho0 s_i(u; phi): s_i = w_i [3 e.u + 4.5 (e.u)^2 ip - 1.5 uu ip]
    const R ex[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
    const R ey[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
    const R w[9] = {R(4.0 / 9.0), R(1.0 / 9.0), R(1.0 / 9.0), R(1.0 / 9.0), R(1.0 / 9.0),
                    R(1.0 / 36.0), R(1.0 / 36.0), R(1.0 / 36.0), R(1.0 / 36.0)};
    const R uu = ux * ux + uy * uy;
    R lux = 0, luy = 0, lip = 0;
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        const R eu = ex[i] * ux + ey[i] * uy;
        const R c = -r0 * w[i] * lfb[i];
        lux += c * (R(3) * ex[i] + R(9) * eu * ex[i] * ip - R(3) * ux * ip);
        luy += c * (R(3) * ey[i] + R(9) * eu * ey[i] * ip - R(3) * uy * ip);
        lip += c * (R(4.5) * eu * eu - R(1.5) * uu);
    }
    // g_b,i = g_f,i + wt_i (theta_b - theta_f) - wt1 T_f u_coef (e_i . u)   (i >= 1)
    const R sw = P.wt0 * lgb[0] + P.wt1 * ((lgb[1] + lgb[2]) + (lgb[3] + lgb[4]));
    A.theta -= sw;                           // via theta_f
    const R k = P.wt1 * P.u_coef;
    const R Tf = P.T0 + mf.theta;
    const R dx = lgb[1] - lgb[3], dy = lgb[2] - lgb[4];
    lux -= k * Tf * dx;
    luy -= k * Tf * dy;
    A.theta -= k * (ux * dx + uy * dy);      // via T_f
    A.ux += lux;
    A.uy += luy;
    A.ip += lip;
    return sw;
}

template <typename R>
__device__ __forceinline__ bool on_wall(const Geo& G, int x, int y) {
    return (G.wallW && x == 0) || (G.wallE && x == G.nx - 1) || (G.wallS && y == 0) ||
           (G.wallN && y == G.ny - 1);
}

// Work-group tiles of the backward step: kAdjTX x kAdjTY nodes, one work-item each, one
// wavefront per row.  Every wall node shares its tile with its inward neighbour: where the
// last tile along a walled axis would be one node wide, it starts one node earlier and the tile
// before it ends there (a walled axis has at least five nodes).
constexpr int kAdjTX = 64, kAdjTY = 4, kAdjThreads = kAdjTX * kAdjTY;
// What a wall node hands its inward neighbour: the adjoints of the neighbour's 14 pulled
// populations and of its ux, uy, 1/phi, theta and P.
constexpr int kHandoff = 19;

struct AdjTiles {
    int nx_tiles, ny_tiles;
    int last_x0, last_y0;   // first column and first row of the last tile along x and y
};

// Nodes [a, b) of tile t of T along an axis of n nodes.
__device__ __forceinline__ void adj_span(int t, int T, int side, int last0, int n, int& a,
                                         int& b) {
    a = t == T - 1 ? last0 : t * side;
    b = t == T - 1 ? n : min((t + 1) * side, last0);
}

// One backward step.  state: the forward state X^n (post-collision populations entering step
// n); lam_in: adjoint of X^{n+1}; lam_out: adjoint of X^n (written); gphi, gK: FP64 gradient
// planes [ny][pitch] accumulated in place.  S: storage type of state, adjoint and medium;
// R: arithmetic type.
//
// A fluid node's work-item reverses its own collision and macroscopics.  A wall node's
// work-item runs the same gather, macroscopics and collision VJP on the wall node's own
// reconstructed state (so both kinds of node stay in step), adds its dJ/dphi (through
// F_b = phi_b G_b), writes zeros to its own slots (the forward step never reads them) and hands
// its inward neighbour, through LDS, what flows back through the reconstruction.  After one
// barrier the neighbour adds up to three hand-offs (two sides and their corner) in a fixed
// order before reversing its own macroscopics.
template <typename S, typename R, bool PN>
__global__ __launch_bounds__(kAdjThreads) void adjoint_step_kernel(
    const S* __restrict__ state, const S* __restrict__ lam_in, S* __restrict__ lam_out,
    const S* __restrict__ med, double* __restrict__ gphi, double* __restrict__ gK, Geo G,
    Phys<R> P, AdjTiles T) {
    __shared__ R handoff[kHandoff][kAdjThreads];
    const int tx = blockIdx.x % T.nx_tiles, ty = blockIdx.x / T.nx_tiles;
    int x0, x1, y0, y1;
    adj_span(tx, T.nx_tiles, kAdjTX, T.last_x0, G.nx, x0, x1);
    adj_span(ty, T.ny_tiles, kAdjTY, T.last_y0, G.ny, y0, y1);
    const int me = threadIdx.x;
    const int x = x0 + me % kAdjTX, y = y0 + me / kAdjTX;
    const bool active = x < x1 && y < y1;
    const bool onW = G.wallW && x == 0, onE = G.wallE && x == G.nx - 1;
    const bool onS = G.wallS && y == 0, onN = G.wallN && y == G.ny - 1;
    const bool wall = onW || onE || onS || onN;
    const int o = y * G.pitch + x;
    const int xm = (x == 0) ? G.nx - 1 : x - 1;
    const int xp = (x == G.nx - 1) ? 0 : x + 1;
    const int ym = (y == 0) ? G.ny - 1 : y - 1;
    const int yp = (y == G.ny - 1) ? 0 : y + 1;
    // slot owned by this node for population i: (i, x - e_i); valid unless it leaves a walled
    // side of the domain
    const int sx[9] = {x, xm, x, xp, x, xm, xp, xp, xm};
    const int sy[9] = {y, y, ym, y, yp, ym, ym, yp, yp};

    R f[9], g[5], af[9], ag[5], phi = 0, K = 0;
    Med<R> md{};
    MacAdj<R> A{};
    // the gradient planes are read before the barrier, which global loads do not cross, so
    // that their latency hides behind the step's arithmetic
    double gphi0 = 0, gK0 = 0;
    if (active) {
        gphi0 = gphi[o];
        if (!wall) gK0 = gK[o];
        // the node whose pulled populations this node's state is built from: itself, or its
        // inward neighbour (the diagonal one at a corner)
        const int px = x + (onW ? 1 : 0) - (onE ? 1 : 0);
        const int py = y + (onS ? 1 : 0) - (onN ? 1 : 0);
        pull<R, S>(state, G, px, py, f, g);
        if constexpr (PN) {
            const int op = py * G.pitch + px;
            phi = R(med[op]);
            K = R(med[G.plane + op]);
            md = medium_from<R>(phi, K, P);
        } else {
            phi = P.phi;
            K = P.c_lin > R(0) ? phi * P.nu / P.c_lin : R(INFINITY);
            md = Med<R>{P.phi, P.inv_phi, P.c_lin, P.c_nl};
        }
        const Mac<R> m = fluid_macros<R>(f, g, md, P);
        R lout[14];
#pragma unroll
        for (int i = 0; i < 14; ++i) lout[i] = R(lam_in[i * G.plane + o]);
        Mac<R> mc = m;
        Med<R> mdc = md;
        R theta_b = 0, phi_b = 0;
        if (wall) {
            // the wall node's state: rebuilt from its neighbour's, at rest, with its own phi
            theta_b = wall_theta<R>(onW, onE, onS, onN, m.theta, P);
            nee_wall<R>(f, g, m, md, theta_b, P);
            phi_b = PN ? R(med[o]) : P.phi;
            mc.theta = theta_b;
            mc.ux = R(0);
            mc.uy = R(0);
            mc.Fx = phi_b * P.ax;
            mc.Fy = phi_b * (P.ay + P.gbeta * theta_b);
            mdc = Med<R>{phi_b, R(1) / phi_b, R(0), R(0)};
        }
#pragma unroll
        for (int i = 0; i < 9; ++i) af[i] = R(0);
#pragma unroll
        for (int i = 0; i < 5; ++i) ag[i] = R(0);
        collide_vjp<R>(f, g, mc, mdc, P, lout, lout + 9, af, ag, A);
        if (wall) {
            // at rest the collision depends on 1/phi_b only through terms in u = 0, so phi_b
            // acts through F_b alone; theta_b through the collision, F_b and the rebuilt g
            const R Gy = P.ay + P.gbeta * theta_b;
            const R lphib = P.ax * A.Fx + Gy * A.Fy;
            const R lthb = A.theta + phi_b * P.gbeta * A.Fy;
            MacAdj<R> H{};
            const R sw = nee_vjp<R>(m, md, P, af, ag, H);
            const bool adiabatic = !((onW && P.iso[0]) || (onE && P.iso[1]) ||
                                     (onS && P.iso[2]) || (onN && P.iso[3]));
            if (adiabatic) H.theta += lthb + sw;    // theta_b = theta_f on an adiabatic side
#pragma unroll
            for (int i = 0; i < 9; ++i) handoff[i][me] = af[i];
#pragma unroll
            for (int i = 0; i < 5; ++i) handoff[9 + i][me] = ag[i];
            handoff[14][me] = H.ux;
            handoff[15][me] = H.uy;
            handoff[16][me] = H.ip;
            handoff[17][me] = H.theta;
            handoff[18][me] = A.P;
            const bool okx_m = !onW, okx_p = !onE, oky_m = !onS, oky_p = !onN;
            const bool ok[9] = {true, okx_m, oky_m, okx_p, oky_p, okx_m && oky_m,
                                okx_p && oky_m, okx_p && oky_p, okx_m && oky_p};
#pragma unroll
            for (int i = 0; i < 9; ++i)
                if (ok[i]) lam_out[i * G.plane + sy[i] * G.pitch + sx[i]] = S(0);
#pragma unroll
            for (int i = 0; i < 5; ++i)
                if (ok[i]) lam_out[(9 + i) * G.plane + sy[i] * G.pitch + sx[i]] = S(0);
            gphi[o] = gphi0 + double(lphib);
        }
    }
    __syncthreads();
    if (!active || wall) return;

    // hand-offs of the wall nodes whose inward neighbour this node is, in a fixed order
    const bool nearW = G.wallW && x == 1, nearE = G.wallE && x == G.nx - 2;
    const bool nearS = G.wallS && y == 1, nearN = G.wallN && y == G.ny - 2;
    if (nearW || nearE || nearS || nearN) {
        const bool has[8] = {nearW,          nearE,          nearS,          nearN,
                             nearW && nearS, nearE && nearS, nearW && nearN, nearE && nearN};
        const int dxs[8] = {-1, 1, 0, 0, -1, 1, -1, 1};
        const int dys[8] = {0, 0, -1, 1, -1, -1, 1, 1};
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            if (!has[k]) continue;
            const int j = me + dys[k] * kAdjTX + dxs[k];
#pragma unroll
            for (int i = 0; i < 9; ++i) af[i] += handoff[i][j];
#pragma unroll
            for (int i = 0; i < 5; ++i) ag[i] += handoff[9 + i][j];
            A.ux += handoff[14][j];
            A.uy += handoff[15][j];
            A.ip += handoff[16][j];
            A.theta += handoff[17][j];
            A.P += handoff[18][j];
        }
    }
    R lphi = 0, lK = 0;
    macros_vjp<R>(f, g, phi, K, md, P, A, af, ag, lphi, lK);
#pragma unroll
    for (int i = 0; i < 9; ++i) lam_out[i * G.plane + sy[i] * G.pitch + sx[i]] = S(af[i]);
#pragma unroll
    for (int i = 0; i < 5; ++i) lam_out[(9 + i) * G.plane + sy[i] * G.pitch + sx[i]] = S(ag[i]);
    gphi[o] = gphi0 + double(lphi);
    gK[o] = gK0 + double(lK);
}

// Seed: adjoint of X^N for J = Nu_hot(T at time N).  T(x) = T0 + sum_i g_i(x - e_i) at a fluid
// node; at a wall node T is the wall value (isothermal side) or the inward neighbour's T.  One
// work-item per node of the first six columns; all other slots must already be zero.
template <typename R>
__device__ __forceinline__ double nu_weight(const Geo& G, int x, int y, double scale) {
    if (x > 4) return 0.0;
    const double c[5] = {-25.0, 48.0, -36.0, 16.0, -3.0};
    const double w = (y == 0 || y == G.ny - 1) ? 0.5 : 1.0;
    return scale * w * c[x] / 12.0;
}

template <typename S, typename R>
__global__ void adjoint_seed_kernel(S* __restrict__ lam, Geo G, Phys<R> P, double scale) {
    const int ncol = G.nx < 6 ? G.nx : 6;
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= ncol * G.ny) return;
    const int y = k / ncol, x = k - y * ncol;
    if (on_wall<R>(G, x, y)) return;
    double c = nu_weight<R>(G, x, y, scale);
    const int dxs[8] = {-1, 1, 0, 0, -1, 1, -1, 1};
    const int dys[8] = {0, 0, -1, 1, -1, -1, 1, 1};
    for (int d = 0; d < 8; ++d) {
        const int xb = x + dxs[d], yb = y + dys[d];
        if (xb < 0 || xb >= G.nx || yb < 0 || yb >= G.ny) continue;
        const bool bW = G.wallW && xb == 0, bE = G.wallE && xb == G.nx - 1;
        const bool bS = G.wallS && yb == 0, bN = G.wallN && yb == G.ny - 1;
        if (!(bW || bE || bS || bN)) continue;
        if (xb + (bW ? 1 : 0) - (bE ? 1 : 0) != x || yb + (bS ? 1 : 0) - (bN ? 1 : 0) != y)
            continue;
        const bool adiabatic = !((bW && P.iso[0]) || (bE && P.iso[1]) || (bS && P.iso[2]) ||
                                 (bN && P.iso[3]));
        if (adiabatic) c += nu_weight<R>(G, xb, yb, scale);
    }
    if (c == 0.0) return;
    const int xm = (x == 0) ? G.nx - 1 : x - 1;
    const int xp = (x == G.nx - 1) ? 0 : x + 1;
    const int ym = (y == 0) ? G.ny - 1 : y - 1;
    const int yp = (y == G.ny - 1) ? 0 : y + 1;
    const int sx[5] = {x, xm, x, xp, x};
    const int sy[5] = {y, y, ym, y, yp};
#pragma unroll
    for (int i = 0; i < 5; ++i) lam[(9 + i) * G.plane + sy[i] * G.pitch + sx[i]] = S(c);
}

template <typename R>
__global__ void fill_zero_kernel(R* __restrict__ p, size_t n) {
    for (size_t k = blockIdx.x * size_t(blockDim.x) + threadIdx.x; k < n;
         k += size_t(gridDim.x) * blockDim.x)
        p[k] = R(0);
}

__global__ void unpitch_scale_kernel(double* __restrict__ dst, const double* __restrict__ src,
                                     Geo G, double scale) {
    const int n = G.nx * G.ny;
    for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < n; k += gridDim.x * blockDim.x) {
        const int y = k / G.nx, x = k - y * G.nx;
        dst[k] = scale * src[y * G.pitch + x];
    }
}

template <typename S, typename R>
hipError_t launch_adjoint_seed(const void* state, void* lam, const Geo& G, const Phys<R>& P,
                               double L_over_dT, hipStream_t s) {
    (void)state;
    const int ncol = G.nx < 6 ? G.nx : 6;
    const int n = ncol * G.ny;
    const double scale = -L_over_dT / double(G.ny - 1);
    adjoint_seed_kernel<S, R><<<(n + 255) / 256, 256, 0, s>>>((S*)lam, G, P, scale);
    return hipGetLastError();
}

template <typename S, typename R>
hipError_t launch_adjoint_step(const void* state, const void* lam_in, void* lam_out,
                               const void* med, double* gphi, double* gK, const Geo& G,
                               const Phys<R>& P, hipStream_t s) {
    AdjTiles T;
    T.nx_tiles = (G.nx + kAdjTX - 1) / kAdjTX;
    T.ny_tiles = (G.ny + kAdjTY - 1) / kAdjTY;
    T.last_x0 = (T.nx_tiles - 1) * kAdjTX;
    T.last_y0 = (T.ny_tiles - 1) * kAdjTY;
    if (G.wallE && G.nx - T.last_x0 == 1) T.last_x0 = G.nx - 2;
    if (G.wallN && G.ny - T.last_y0 == 1) T.last_y0 = G.ny - 2;
    const int nwg = T.nx_tiles * T.ny_tiles;
    if (med)
        adjoint_step_kernel<S, R, true><<<nwg, kAdjThreads, 0, s>>>(
            (const S*)state, (const S*)lam_in, (S*)lam_out, (const S*)med, gphi, gK, G, P, T);
    else
        adjoint_step_kernel<S, R, false><<<nwg, kAdjThreads, 0, s>>>(
            (const S*)state, (const S*)lam_in, (S*)lam_out, nullptr, gphi, gK, G, P, T);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_fill(void* dst, size_t n, hipStream_t s) {
    fill_zero_kernel<R><<<1024, 256, 0, s>>>((R*)dst, n);
    return hipGetLastError();
}

hipError_t launch_fill_f64(double* dst, size_t n, hipStream_t s) {
    fill_zero_kernel<double><<<1024, 256, 0, s>>>(dst, n);
    return hipGetLastError();
}

hipError_t launch_unpitch_scale(double* dst, const double* src, const Geo& G, double scale,
                                hipStream_t s) {
    unpitch_scale_kernel<<<1024, 256, 0, s>>>(dst, src, G, scale);
    return hipGetLastError();
}

#define LBM_ADJ_INSTANCES(S, R)                                                                  \
    template hipError_t launch_adjoint_seed<S, R>(const void*, void*, const Geo&,                \
                                                  const Phys<R>&, double, hipStream_t);          \
    template hipError_t launch_adjoint_step<S, R>(const void*, const void*, void*, const void*,  \
                                                  double*, double*, const Geo&, const Phys<R>&,  \
                                                  hipStream_t);
LBM_ADJ_INSTANCES(float, float)
LBM_ADJ_INSTANCES(double, double)
LBM_ADJ_INSTANCES(float, double)
#undef LBM_ADJ_INSTANCES
template hipError_t launch_fill<float>(void*, size_t, hipStream_t);
template hipError_t launch_fill<double>(void*, size_t, hipStream_t);

}  // namespace lbm
