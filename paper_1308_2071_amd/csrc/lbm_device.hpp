// lbm_device.hpp -- per-node arithmetic of the coupled D2Q9 / D2Q5 porous-media MRT lattice
// Boltzmann step (Liu, He, Li, Tao, arXiv:1308.2071), shared by the plain, batched and adjoint
// kernels.
//
// Storage: populations are kept as deviations from the rest state, f'_i = f_i - w_i rho0 and
// g'_i = g_i - wt_i T0 (T0 the buoyancy reference temperature).  Every operation of the step
// is affine in the populations, so the step is computed on deviations exactly; in FP32 this
// keeps ~7 significant digits on the O(Ma^2) physics instead of on the O(1) rest values.
// With deviations, m' = M f' and the rest moments rho0 (1, -2, 1, 0, ..., 0) drop out; the
// pressure enters through P = phi p - rho0 cs^2.
//
// Layout: 14 planes [f0..f8, g0..g4], each [ny][pitch] with x fastest, G.plane elements apart.
//
// Precision: S is the storage type of the populations and the medium planes, R the type the
// arithmetic runs in.  (S, R) = (float, float), (double, double), or (float, double): FP32
// storage with FP64 arithmetic, where each stored deviation is rounded once per step and none
// of the ~300 operations in between are.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

namespace lbm {

constexpr int kPlanes = 14;
// 1.75 / sqrt(150): Eq. (5) gives phi F_phi = 1.75/sqrt(150) * phi^(-1/2).
constexpr double kErgun = 0.14288690166235207;

struct Geo {
    int nx, ny, pitch;
    int plane;             // elements from one plane to the next: ny * pitch plus a pad
    int wallW, wallE, wallS, wallN;  // side is a wall (not periodic)
};

// Population plane i of a state buffer.  The pointer is uniform over the work-group; nodes
// index it with an unsigned 32-bit offset (a plane holds fewer than 2^31 elements), which lets
// the compiler address every plane from one scalar base and one vector offset per position.
template <typename T>
__device__ __forceinline__ T* plane(T* base, int i, int P) {
    return base + size_t(i) * size_t(P);
}

// Element at a 32-bit byte offset from a uniform base.  A state holds fewer than 2^31
// elements over 14 planes, so a plane is below 1.3 GB even in FP64 and the byte offset of any
// node in it fits 32 bits; computed there, each access can use the scalar-base plus 32-bit
// vector-offset address form.
template <typename T>
__device__ __forceinline__ T& at(T* base, unsigned byte_off) {
    return *reinterpret_cast<T*>(reinterpret_cast<
        typename std::conditional<std::is_const<T>::value, const char*, char*>::type>(base) +
                                 byte_off);
}

template <typename R>
struct Phys {
    R rho0, inv_rho0;
    R gbeta, ax, ay;       // g*beta and the extra body acceleration (Eq. (4), G)
    R nu;                  // fluid viscosity in the Darcy term of Eq. (4)
    R s_e, s_eps, s_q, s_v;        // Eq. (20)
    R os_e, os_eps, os_q, os_v;    // 1 - s/2
    R z_T, z3, z4;                 // Eq. (31): zeta1 = zeta2 = z_T
    R inv_sigma, varpi;
    R wt0, wt1;            // Eq. (37a) weights
    R u_coef;              // 1 / (sigma csT^2)
    R T0;
    R hQs;                 // Q'''/(2 sigma): T = sum g + hQs (Eq. (36))
    R psi3;                // (1 - zeta3/2) varpi Q'''/sigma (Eqs. (30), (34))
    R theta_wall[4];       // T_wall - T0 per side
    int iso[4];            // side is isothermal
    int forch;             // Forchheimer term on
    // uniform medium (used when there are no per-node planes)
    R phi, inv_phi, c_lin, c_nl;
};

// Medium coefficients of one node: phi, 1/phi, c_lin = phi nu / K, c_nl = phi F_phi / sqrt(K).
template <typename R>
struct Med {
    R phi, inv_phi, c_lin, c_nl;
};

// Macroscopic state of one node: theta = T - T0, u, P = phi p - rho0 cs^2, F (Eq. (4)), and
// |v|^2 of Eq. (22) (a wall node carries its inward neighbour's), which the divergence check
// reads: once |v|^2 overflows, Eq. (21) returns u = 0 and u alone no longer shows the blow-up.
template <typename R>
struct Mac {
    R theta, ux, uy, P, Fx, Fy, vv;
};

// Arithmetic forms.  The build does not contract a * b + c on its own (-ffp-contract=off), so
// that every kernel computing a node rounds exactly alike; where a fused multiply-add is
// wanted it is written out (fma), the same in every kernel.  Products by 2, 4, 0.25 and 0.5
// are exact, so fma(2, a, b) rounds like 2 * a + b did.
//
// rsq_1ulp, sqrt_1ulp: in FP32 the hardware reciprocal square root and square root (within
// 1 ulp) instead of the correctly rounded sequences (~15 instructions each).  They are used
// only where one rounding more cannot act as a common gain: the medium coefficients of a
// per-node medium (Eq. (5), different at every node), |v| inside Eq. (21)'s root (a small
// correction to l0^2) and |u| in Eq. (4)'s Forchheimer term.  FP64 keeps sqrt.
__device__ __forceinline__ float rsq_1ulp(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ double rsq_1ulp(double x) { return 1.0 / sqrt(x); }
__device__ __forceinline__ float sqrt_1ulp(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ double sqrt_1ulp(double x) { return sqrt(x); }

template <typename R>
__device__ __forceinline__ Med<R> medium_from(R phi, R K, const Phys<R>& P) {
    Med<R> m;
    const R rK = rsq_1ulp(K);
    m.phi = phi;
    m.inv_phi = R(1) / phi;
    m.c_lin = phi * P.nu * (rK * rK);
    m.c_nl = P.forch ? R(kErgun) * rsq_1ulp(phi) * rK : R(0);
    return m;
}

template <typename R, bool PN, typename S = R>
__device__ __forceinline__ Med<R> load_medium(const S* __restrict__ med, int idx, int plane,
                                              const Phys<R>& P) {
    if constexpr (PN) {
        const unsigned o = unsigned(idx) * unsigned(sizeof(S));
        return medium_from<R>(R(at(med, o)), R(at(lbm::plane(med, 1, plane), o)), P);
    } else {
        return Med<R>{P.phi, P.inv_phi, P.c_lin, P.c_nl};
    }
}

// Population layouts.
//   kPull  two buffers.  The state holds the post-collision f+_i(x) at slot (i, x); a step
//          gathers f_i(x) = f+_i(x - e_i) (streaming as a pull) and writes slot (i, x) of the
//          other buffer.
//   AA pattern, one buffer, two alternating forms of the same step:
//   kAAOpp the state holds f+_i(x) at slot (opp(i), x) (after an even number of steps; the
//          rest state, symmetric in i <-> opp(i), is both).  The step gathers f_i(x) from
//          (opp(i), x - e_i) and writes f+_i(x) to (i, x + e_i), its streamed position.
//   kAAOwn the state holds the streamed f_i(x) at slot (i, x) (after an odd number of steps).
//          The step gathers in place and writes f+_i(x) to (opp(i), x).
// In both AA forms the slots a node's step writes are exactly the slots it read, so one
// buffer suffices.
enum PopLayout { kPull = 0, kAAOpp = 1, kAAOwn = 2 };

// Streaming, Eqs. (18) and (35): the populations arriving at (x, y), i.e. those that left
// (x - ex_i, y - ey_i) after the previous collision, as the layout L stores them.  Indices
// wrap, which is only ever used on periodic axes: on a walled axis the node is interior, so
// x-1 and x+1 stay in range.
template <typename R, typename S = R, int L = kPull>
__device__ __forceinline__ void pull(const S* __restrict__ src, const Geo& G, int x, int y,
                                     R f[9], R g[5]) {
    constexpr unsigned B = sizeof(S);
    const unsigned xm = (x == 0) ? G.nx - 1 : x - 1;
    const unsigned xp = (x == G.nx - 1) ? 0 : x + 1;
    const unsigned rm = unsigned((y == 0) ? G.ny - 1 : y - 1) * unsigned(G.pitch);
    const unsigned rp = unsigned((y == G.ny - 1) ? 0 : y + 1) * unsigned(G.pitch);
    const unsigned r0 = unsigned(y) * unsigned(G.pitch);
    const unsigned xx = unsigned(x);
    const int P = G.plane;
    if constexpr (L == kAAOwn) {
        const unsigned o = (r0 + xx) * B;
#pragma unroll
        for (int i = 0; i < 9; ++i) f[i] = R(at(plane(src, i, P), o));
#pragma unroll
        for (int i = 0; i < 5; ++i) g[i] = R(at(plane(src, 9 + i, P), o));
        return;
    }
    // plane holding direction i: i itself (kPull) or opp(i) (kAAOpp); D2Q9 opposites
    // 1 <-> 3, 2 <-> 4, 5 <-> 7, 6 <-> 8, D2Q5 likewise for 1..4
    constexpr bool O = (L == kAAOpp);
    const unsigned c00 = (r0 + xx) * B, cw = (r0 + xm) * B, ce = (r0 + xp) * B;
    const unsigned cs = (rm + xx) * B, cn = (rp + xx) * B;
    const unsigned csw = (rm + xm) * B, cse = (rm + xp) * B;
    const unsigned cne = (rp + xp) * B, cnw = (rp + xm) * B;
    f[0] = R(at(plane(src, 0, P), c00));
    f[1] = R(at(plane(src, O ? 3 : 1, P), cw));
    f[2] = R(at(plane(src, O ? 4 : 2, P), cs));
    f[3] = R(at(plane(src, O ? 1 : 3, P), ce));
    f[4] = R(at(plane(src, O ? 2 : 4, P), cn));
    f[5] = R(at(plane(src, O ? 7 : 5, P), csw));
    f[6] = R(at(plane(src, O ? 8 : 6, P), cse));
    f[7] = R(at(plane(src, O ? 5 : 7, P), cne));
    f[8] = R(at(plane(src, O ? 6 : 8, P), cnw));
    g[0] = R(at(plane(src, 9, P), c00));
    g[1] = R(at(plane(src, O ? 12 : 10, P), cw));
    g[2] = R(at(plane(src, O ? 13 : 11, P), cs));
    g[3] = R(at(plane(src, O ? 10 : 12, P), ce));
    g[4] = R(at(plane(src, O ? 11 : 13, P), cn));
}

// x / d for a small integer d, correctly rounded: the product with r = RN(1/d) is within one
// ulp of x/d, the residual x - q d is exact with a fused multiply-add, and one more fused step
// q + (x - q d) r rounds to RN(x/d) (Markstein, IBM J. Res. Dev. 34 (1990)).  A bare product
// x r would carry the relative error of r, the same sign at every node and step.
template <typename R>
__device__ __forceinline__ R div_const(R x, R d, R r) {
    const R q = x * r;
    const R e = fma(-q, d, x);
    return fma(e, r, q);
}

// The velocity part of the macroscopic recovery at a fluid node, shared by fluid_macros and
// the adjoint's recompute so that both see the same values: theta = T - T0 (Eq. (36)), G
// (Eq. (4)), v (Eq. (22)), l0, l1, |v|, the root q and den = l0 + q of Eq. (21), u = v / den,
// |u|^2, |u| and the drag coefficient of Eq. (4).
template <typename R>
struct Vel {
    R theta, Gx, Gy, vx, vy, l0, l1, vv, vm, q, den, ux, uy, uu, um, drag;
};

template <typename R>
__device__ __forceinline__ Vel<R> velocity(const R f[9], const R g[5], const Med<R>& md,
                                           const Phys<R>& P) {
    Vel<R> v;
    v.theta = ((g[0] + g[1]) + (g[2] + g[3]) + g[4]) + P.hQs;
    v.Gx = P.ax;
    v.Gy = fma(P.gbeta, v.theta, P.ay);
    const R jx = (f[1] - f[3]) + (f[5] - f[6]) - (f[7] - f[8]);
    const R jy = (f[2] - f[4]) + (f[5] + f[6]) - (f[7] + f[8]);
    const R hphi = R(0.5) * md.phi;
    v.vx = fma(hphi, v.Gx, jx * P.inv_rho0);
    v.vy = fma(hphi, v.Gy, jy * P.inv_rho0);
    v.l0 = fma(R(0.25), md.c_lin, R(0.5));
    v.l1 = R(0.5) * md.c_nl;
    v.vv = fma(v.vx, v.vx, v.vy * v.vy);
    v.vm = sqrt_1ulp(v.vv);
    v.q = sqrt(fma(v.l0, v.l0, v.l1 * v.vm));
    v.den = v.l0 + v.q;
    // divide rather than multiply by a rounded reciprocal: in a uniform medium the denominator
    // is nearly the same at every node, so the reciprocal's rounding would act as one common
    // gain on the momentum, step after step
    v.ux = v.vx / v.den;
    v.uy = v.vy / v.den;
    v.uu = fma(v.ux, v.ux, v.uy * v.uy);
    v.um = sqrt_1ulp(v.uu);
    v.drag = fma(md.c_nl, v.um, md.c_lin);
    return v;
}

// Eqs. (36), (22), (21), (23), (4) at a fluid node, on deviation populations.
template <typename R>
__device__ __forceinline__ Mac<R> fluid_macros(const R f[9], const R g[5], const Med<R>& md,
                                               const Phys<R>& P) {
    const Vel<R> v = velocity<R>(f, g, md, P);
    Mac<R> m;
    // phi p = cs^2/(1 - w0) [sum_{i>=1} f_i + rho0 s0(u)], s0 = -w0 |u|^2 / (2 phi cs^2).
    // The level of phi p is a free mode of the step (a gauge that no equation restores), so
    // each rounding on its path that repeats step after step moves it for good.  The sum and
    // the factor are taken in FP64 in every precision and rounded once: in the 256^2 workload
    // the FP32 level moved by 1.2e-4 of p's range in 50k steps with them in FP32, 7.3e-5 this
    // way, at no measurable cost.  cs^2/(1 - w0) = 3/5 is a correctly rounded division by 5:
    // a product with the rounded 0.6 is a common gain on the level (in FP32 it moved it by
    // 3.0e-4 of the range).
    const double sum18 = ((double(f[1]) + double(f[2])) + (double(f[3]) + double(f[4]))) +
                         ((double(f[5]) + double(f[6])) + (double(f[7]) + double(f[8])));
    m.P = R(div_const(3.0 * fma(-2.0 / 3.0 * double(P.rho0), double(v.uu) * double(md.inv_phi),
                                sum18),
                      5.0, 1.0 / 5.0));
    m.theta = v.theta;
    m.ux = v.ux;
    m.uy = v.uy;
    m.Fx = fma(-v.drag, v.ux, md.phi * v.Gx);
    m.Fy = fma(-v.drag, v.uy, md.phi * v.Gy);
    m.vv = v.vv;
    return m;
}

// Non-equilibrium extrapolation at a wall node whose inward neighbour x_f holds (f, g) with
// macroscopics mf and medium mdf.  All populations are replaced by the wall equilibrium
// (u = 0, phi_b p_b = phi_f p_f, T_b) plus the neighbour's non-equilibrium part.  Because the
// pressure parts of the two equilibria cancel, f_b,i = f_f,i - rho0 s_i(u_f; phi_f).
template <typename R>
__device__ __forceinline__ void nee_wall(R f[9], R g[5], const Mac<R>& mf, const Med<R>& mdf,
                                         R theta_b, const Phys<R>& P) {
    const R ux = mf.ux, uy = mf.uy;
    const R ip = mdf.inv_phi;
    const R uu = ux * ux + uy * uy;
    const R r0 = P.rho0;
    // rho0 s_i(u) = rho0 w_i [3 e.u + 4.5 (e.u)^2 / phi - 1.5 |u|^2 / phi]   (Eq. (14))
    const R base = R(1.5) * uu * ip;
    const R c1 = r0 * R(1.0 / 9.0), c5 = r0 * R(1.0 / 36.0);
    f[0] -= r0 * R(4.0 / 9.0) * (-base);
    f[1] -= c1 * (R(3) * ux + R(4.5) * ux * ux * ip - base);
    f[2] -= c1 * (R(3) * uy + R(4.5) * uy * uy * ip - base);
    f[3] -= c1 * (R(-3) * ux + R(4.5) * ux * ux * ip - base);
    f[4] -= c1 * (R(-3) * uy + R(4.5) * uy * uy * ip - base);
    const R a = ux + uy, b = uy - ux;
    f[5] -= c5 * (R(3) * a + R(4.5) * a * a * ip - base);
    f[6] -= c5 * (R(3) * b + R(4.5) * b * b * ip - base);
    f[7] -= c5 * (R(-3) * a + R(4.5) * a * a * ip - base);
    f[8] -= c5 * (R(-3) * b + R(4.5) * b * b * ip - base);
    // g_b = wt T_b + g_f - wt T_f (1 + e.u_f / (sigma csT^2))            (Eq. (37a))
    const R dth = theta_b - mf.theta;
    const R Tf = P.T0 + mf.theta;
    const R k = P.wt1 * Tf * P.u_coef;
    g[0] += P.wt0 * dth;
    g[1] += P.wt1 * dth - k * ux;
    g[2] += P.wt1 * dth - k * uy;
    g[3] += P.wt1 * dth + k * ux;
    g[4] += P.wt1 * dth + k * uy;
}

// Collision in moment space, Eq. (17) with s0 = s3 = s5 = 1 (Sec. 4) and Eq. (34) with
// zeta0 = 1 and the heat source of Eq. (30); f, g hold post-streaming deviations on entry and
// post-collision deviations on exit.
template <typename R>
__device__ __forceinline__ void collide(R f[9], R g[5], const Mac<R>& m, const Med<R>& md,
                                        const Phys<R>& P) {
    // m' = M f' (rows of Eq. (11)); m0', m3', m5' are not needed: s0 = s3 = s5 = 1
    const R s14 = (f[1] + f[2]) + (f[3] + f[4]);
    const R p56 = f[5] + f[6], p78 = f[7] + f[8];
    const R d56 = f[5] - f[6], d78 = f[7] - f[8];
    const R s58 = p56 + p78;
    const R qx = d56 - d78;
    const R qy = p56 - p78;
    const R m1 = fma(R(-4), f[0], fma(R(2), s58, -s14));
    const R m2 = fma(R(4), f[0], fma(R(-2), s14, s58));
    const R m4 = fma(R(-2), f[1] - f[3], qx);
    const R m6 = fma(R(-2), f[2] - f[4], qy);
    const R m7 = (f[1] - f[2]) + (f[3] - f[4]);
    const R m8 = d56 + d78;
    // equilibrium moments (Eq. (16) less the rest state) and forcing (Eq. (19))
    const R r0 = P.rho0, ux = m.ux, uy = m.uy;
    const R rip = r0 * md.inv_phi;
    const R uu = fma(ux, ux, uy * uy);
    const R ruu = R(3) * rip * uu;
    const R e_eq = fma(R(6), m.P, ruu);
    const R eps_eq = fma(R(-9), m.P, -ruu);
    const R pxx_eq = rip * fma(ux, ux, -(uy * uy));
    const R pxy_eq = rip * ux * uy;
    const R S1 = R(6) * rip * fma(ux, m.Fx, uy * m.Fy);
    const R S7 = R(2) * rip * fma(ux, m.Fx, -(uy * m.Fy));
    const R S8 = rip * fma(ux, m.Fy, uy * m.Fx);
    const R rFx = r0 * m.Fx, rFy = r0 * m.Fy;
    // relaxation m - s (m - m_eq) + (1 - s/2) S, then division by |row|^2 for
    // M^-1 = M^T diag(1/|row|^2); the divisions by 36, 6 and 12 are correctly rounded (not
    // products with the rounded reciprocal, whose error is one common gain on energy and
    // momentum that accumulates step after step)
    const R a1 = div_const(fma(P.os_e, S1, fma(-P.s_e, m1 - e_eq, m1)), R(36), R(1.0 / 36.0));
    const R a2 =
        div_const(fma(-P.os_eps, S1, fma(-P.s_eps, m2 - eps_eq, m2)), R(36), R(1.0 / 36.0));
    const R a3 = div_const(fma(R(0.5), rFx, r0 * ux), R(6), R(1.0 / 6.0));
    const R a4 = div_const(fma(-P.os_q, rFx, fma(-P.s_q, fma(r0, ux, m4), m4)), R(12),
                           R(1.0 / 12.0));
    const R a5 = div_const(fma(R(0.5), rFy, r0 * uy), R(6), R(1.0 / 6.0));
    const R a6 = div_const(fma(-P.os_q, rFy, fma(-P.s_q, fma(r0, uy, m6), m6)), R(12),
                           R(1.0 / 12.0));
    const R a7 = fma(P.os_v, S7, fma(-P.s_v, m7 - pxx_eq, m7)) * R(0.25);
    const R a8 = fma(P.os_v, S8, fma(-P.s_v, m8 - pxy_eq, m8)) * R(0.25);
    // f' = M^T a (columns of Eq. (11)); a0 = 0 because the post-collision m0' is 0
    const R c14 = fma(R(-2), a2, -a1);
    const R c58 = fma(R(2), a1, a2);
    f[0] = R(4) * (a2 - a1);
    const R x4 = fma(R(-2), a4, a3), y6 = fma(R(-2), a6, a5);
    f[1] = (c14 + x4) + a7;
    f[2] = (c14 + y6) - a7;
    f[3] = (c14 - x4) + a7;
    f[4] = (c14 - y6) - a7;
    const R px = a3 + a4, py = a5 + a6;
    f[5] = ((c58 + px) + py) + a8;
    f[6] = ((c58 - px) + py) - a8;
    f[7] = ((c58 - px) - py) + a8;
    f[8] = ((c58 + px) - py) - a8;

    // thermal: n' = N g' (rows of Eq. (28)); with zeta0 = 1, n0'+ = theta + Q'''/(2 sigma)
    // (the source term of Eq. (34) with Psi0 = Q'''/sigma, Eq. (30))
    const R Ts = (P.T0 + m.theta) * P.inv_sigma;
    const R n1 = g[1] - g[3];
    const R n2 = g[2] - g[4];
    const R n3 = fma(R(-4), g[0], (g[1] + g[2]) + (g[3] + g[4]));
    const R n4 = (g[1] - g[2]) + (g[3] - g[4]);
    const R b0 = div_const(m.theta + P.hQs, R(5), R(1.0 / 5.0));
    const R b1 = fma(-P.z_T, fma(-ux, Ts, n1), n1) * R(0.5);
    const R b2 = fma(-P.z_T, fma(-uy, Ts, n2), n2) * R(0.5);
    const R b3 = div_const(fma(-P.z3, fma(-P.varpi, m.theta, n3), n3) + P.psi3, R(20),
                           R(1.0 / 20.0));
    const R b4 = fma(-P.z4, n4, n4) * R(0.25);
    // g' = N^T b (columns of Eq. (28))
    const R b03 = b0 + b3;
    g[0] = fma(R(-4), b3, b0);
    g[1] = b03 + (b1 + b4);
    g[2] = b03 + (b2 - b4);
    g[3] = b03 - (b1 - b4);
    g[4] = b03 - (b2 + b4);
}

// Wall temperature rule: an isothermal side fixes T; at a corner of two isothermal sides the
// mean is used; on adiabatic sides T_b = T_f (zero normal gradient).
template <typename R>
__device__ __forceinline__ R wall_theta(bool onW, bool onE, bool onS, bool onN, R theta_f,
                                        const Phys<R>& P) {
    // selects, not indexing: a runtime index into P would force a register copy of it into
    // private memory
    const bool isoX = (onW && P.iso[0]) || (onE && P.iso[1]);
    const bool isoY = (onS && P.iso[2]) || (onN && P.iso[3]);
    const R tX = onW ? P.theta_wall[0] : P.theta_wall[1];
    const R tY = onS ? P.theta_wall[2] : P.theta_wall[3];
    if (isoX && isoY) return R(0.5) * (tX + tY);
    if (isoX) return tX;
    if (isoY) return tY;
    return theta_f;
}

// Macroscopics of a wall node (on the sides flagged onW..onN) whose inward neighbour holds the
// pulled populations f, g with macroscopics mf and medium mdf; f, g are overwritten with the
// wall node's reconstructed populations; mdb is the wall node's own medium.
template <typename R>
__device__ __forceinline__ Mac<R> wall_state(bool onW, bool onE, bool onS, bool onN, R f[9],
                                             R g[5], const Mac<R>& mf, const Med<R>& mdf,
                                             const Med<R>& mdb, const Phys<R>& P) {
    const R theta_b = wall_theta<R>(onW, onE, onS, onN, mf.theta, P);
    nee_wall<R>(f, g, mf, mdf, theta_b, P);
    Mac<R> m;
    m.theta = theta_b;
    m.ux = R(0);
    m.uy = R(0);
    m.P = mf.P;
    m.Fx = mdb.phi * P.ax;
    m.Fy = mdb.phi * (P.ay + P.gbeta * theta_b);
    m.vv = mf.vv;
    return m;
}

// Post-streaming, post-wall-reconstruction state of node (x, y): populations, macroscopics and
// medium.  Wall nodes gather around their inward neighbour (the diagonal one at corners).
template <typename R, bool PN, typename S = R, int L = kPull>
__device__ __forceinline__ void node_state(const S* __restrict__ src, const S* __restrict__ med,
                                           const Geo& G, const Phys<R>& P, int x, int y, R f[9],
                                           R g[5], Mac<R>& m, Med<R>& md) {
    const bool onW = G.wallW && x == 0;
    const bool onE = G.wallE && x == G.nx - 1;
    const bool onS = G.wallS && y == 0;
    const bool onN = G.wallN && y == G.ny - 1;
    if (!(onW || onE || onS || onN)) {
        pull<R, S, L>(src, G, x, y, f, g);
        md = load_medium<R, PN, S>(med, y * G.pitch + x, G.plane, P);
        m = fluid_macros<R>(f, g, md, P);
        return;
    }
    const int xf = x + (onW ? 1 : 0) - (onE ? 1 : 0);
    const int yf = y + (onS ? 1 : 0) - (onN ? 1 : 0);
    pull<R, S, L>(src, G, xf, yf, f, g);
    const Med<R> mdf = load_medium<R, PN, S>(med, yf * G.pitch + xf, G.plane, P);
    const Mac<R> mf = fluid_macros<R>(f, g, mdf, P);
    md = load_medium<R, PN, S>(med, y * G.pitch + x, G.plane, P);
    m = wall_state<R>(onW, onE, onS, onN, f, g, mf, mdf, md, P);
}

// For a fluid node (x, y) that holds its pulled populations f, g, macroscopics m and medium md:
// reconstructs and collides every wall node whose inward neighbour it is (up to three: two
// sides and their corner) and hands each to store(xb, yb, fb, gb).  The arithmetic is
// node_state's and collide's, so a wall node stepped this way equals one stepped by its own
// work-item.
template <typename R, bool PN, typename S, typename Store>
__device__ __forceinline__ void step_wall_neighbours(const S* __restrict__ med, const Geo& G,
                                                     const Phys<R>& P, int x, int y,
                                                     const R f[9], const R g[5],
                                                     const Mac<R>& m, const Med<R>& md,
                                                     Store&& store) {
    const bool nearW = G.wallW && x == 1, nearE = G.wallE && x == G.nx - 2;
    const bool nearS = G.wallS && y == 1, nearN = G.wallN && y == G.ny - 2;
    if (!(nearW || nearE || nearS || nearN)) return;
    for (int k = 0; k < 8; ++k) {
        // the 8 neighbours: W, E, S, N, then SW, SE, NW, NE (arithmetic, not a table: an
        // indexed local array would live in scratch memory)
        const int dx = k < 2 ? 2 * k - 1 : (k < 4 ? 0 : 2 * ((k - 4) & 1) - 1);
        const int dy = k < 2 ? 0 : (k < 4 ? 2 * (k - 2) - 1 : 2 * ((k - 4) >> 1) - 1);
        const int xb = x + dx, yb = y + dy;
        if (xb < 0 || xb >= G.nx || yb < 0 || yb >= G.ny) continue;
        const bool bW = G.wallW && xb == 0, bE = G.wallE && xb == G.nx - 1;
        const bool bS = G.wallS && yb == 0, bN = G.wallN && yb == G.ny - 1;
        if (!(bW || bE || bS || bN)) continue;
        if (xb + (bW ? 1 : 0) - (bE ? 1 : 0) != x || yb + (bS ? 1 : 0) - (bN ? 1 : 0) != y)
            continue;
        R fb[9], gb[5];
#pragma unroll
        for (int i = 0; i < 9; ++i) fb[i] = f[i];
#pragma unroll
        for (int i = 0; i < 5; ++i) gb[i] = g[i];
        const Med<R> mdb = load_medium<R, PN, S>(med, yb * G.pitch + xb, G.plane, P);
        const Mac<R> mb = wall_state<R>(bW, bE, bS, bN, fb, gb, m, md, mdb, P);
        collide<R>(fb, gb, mb, mdb, P);
        store(xb, yb, fb, gb);
    }
}

// AA-pattern store of the post-collision populations of node (x, y).  After a kAAOpp gather
// each goes to its streamed position (i, x + e_i) (wrapping on periodic axes; a target beyond
// a walled side is dropped, as nothing would read it); after a kAAOwn gather to (opp(i), x).
template <typename S, typename R, int L>
__device__ __forceinline__ void aa_store(S* __restrict__ buf, const Geo& G, int x, int y,
                                         const R f[9], const R g[5]) {
    const int P = G.plane;
    const unsigned r0 = unsigned(y) * unsigned(G.pitch);
    const unsigned xx = unsigned(x);
    if constexpr (L == kAAOwn) {
        const unsigned o = r0 + xx;
        // f+_i goes to plane opp(i)
        const int opp9[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};
        const int opp5[5] = {0, 3, 4, 1, 2};
#pragma unroll
        for (int i = 0; i < 9; ++i) plane(buf, opp9[i], P)[o] = S(f[i]);
#pragma unroll
        for (int i = 0; i < 5; ++i) plane(buf, 9 + opp5[i], P)[o] = S(g[i]);
    } else {
        const bool okE = !(G.wallE && x == G.nx - 1), okW = !(G.wallW && x == 0);
        const bool okN = !(G.wallN && y == G.ny - 1), okS = !(G.wallS && y == 0);
        const unsigned xm = (x == 0) ? G.nx - 1 : x - 1;
        const unsigned xp = (x == G.nx - 1) ? 0 : x + 1;
        const unsigned rm = unsigned((y == 0) ? G.ny - 1 : y - 1) * unsigned(G.pitch);
        const unsigned rp = unsigned((y == G.ny - 1) ? 0 : y + 1) * unsigned(G.pitch);
        plane(buf, 0, P)[r0 + xx] = S(f[0]);
        plane(buf, 9, P)[r0 + xx] = S(g[0]);
        if (okE) {
            plane(buf, 1, P)[r0 + xp] = S(f[1]);
            plane(buf, 10, P)[r0 + xp] = S(g[1]);
        }
        if (okN) {
            plane(buf, 2, P)[rp + xx] = S(f[2]);
            plane(buf, 11, P)[rp + xx] = S(g[2]);
        }
        if (okW) {
            plane(buf, 3, P)[r0 + xm] = S(f[3]);
            plane(buf, 12, P)[r0 + xm] = S(g[3]);
        }
        if (okS) {
            plane(buf, 4, P)[rm + xx] = S(f[4]);
            plane(buf, 13, P)[rm + xx] = S(g[4]);
        }
        if (okE && okN) plane(buf, 5, P)[rp + xp] = S(f[5]);
        if (okW && okN) plane(buf, 6, P)[rp + xm] = S(f[6]);
        if (okW && okS) plane(buf, 7, P)[rm + xm] = S(f[7]);
        if (okE && okS) plane(buf, 8, P)[rm + xp] = S(f[8]);
    }
}

}  // namespace lbm
