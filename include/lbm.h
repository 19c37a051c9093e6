/*
 * lbm.h -- C ABI of liblbmpm.so, the MI355X (gfx950) implementation of the coupled D2Q9 flow /
 * D2Q5 temperature multiple-relaxation-time lattice Boltzmann model for convection heat transfer
 * in porous media at the REV scale (Q. Liu, Y.-L. He, Q. Li, W.-Q. Tao, arXiv:1308.2071).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Every function returns an lbm_status; nothing throws or aborts across the ABI.  A failed
 *    call leaves a human-readable message in lbm_last_error() (thread-local).
 *  - Argument checking happens before any device call, so LBM_E_INVAL never leaves work queued.
 *  - Device memory is owned by the caller.  The library never allocates device memory: the
 *    caller passes a workspace of at least lbm_workspace_size() bytes (256-byte aligned) that
 *    stays valid until lbm_destroy().  Host memory for the context itself is malloc'd.
 *  - All device work is enqueued on the caller's HIP stream (a hipStream_t passed as void*;
 *    NULL = the null stream).  lbm_step is asynchronous; lbm_observables, lbm_grad, lbm_save
 *    and lbm_load synchronise the stream before returning.
 *  - Asynchronous HIP faults surface as LBM_E_HIP at the next synchronising call.
 *  - A context is used by one host thread at a time.
 *  - Fields are row-major [ny][nx] (x fastest), one value per lattice node, wall nodes included;
 *    node (x, y) sits at x*dx, y*dx with dx = dt = 1 (Sec. 4).
 *
 * State semantics
 * ---------------
 *  The state between steps is the post-collision population field.  One time step is
 *  streaming (Eqs. (18), (35)) -> non-equilibrium extrapolation at wall nodes (Sec. 4, the
 *  paper's ref. [43]) -> macroscopic recovery (Eqs. (36), (22), (21), (23), (4)) -> collision in
 *  moment space (Eqs. (17), (34)).  Observables at time n are the macroscopic fields after the
 *  n-th streaming and wall reconstruction.  At n = 0 every post-collision population is at
 *  rest equilibrium, f_i = w_i rho0 and g_i = wt_i T_init (Eq. (13) with u = 0 and
 *  phi*p = rho0 cs^2; Eq. (37a) with u = 0).
 */
#ifndef LBM_H
#define LBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t lbm_status;
#define LBM_OK 0
#define LBM_E_INVAL (-1)       /* bad argument; nothing was enqueued                        */
#define LBM_E_NOMEM (-2)       /* workspace too small, or host allocation failed            */
#define LBM_E_HIP (-3)         /* a HIP call failed (launch, copy, or an earlier async fault) */
#define LBM_E_DIVERGED (-4)    /* the run diverged (see lbm_obs.why); state still readable   */
#define LBM_E_STATE (-5)       /* call not valid in the context's current state             */
#define LBM_E_UNSUPPORTED (-6) /* valid request the library does not implement             */

/* Precision: storage of the populations, medium planes and fields, and the arithmetic of
 * every per-node operation.  LBM_FP32_F64 stores FP32 (the bytes of LBM_FP32) and computes each
 * step in FP64, rounding each stored value once per step; device arrays passed to or returned
 * by the library (phi, K, fields) are FP32 for it. */
#define LBM_FP32 0       /* FP32 storage, FP32 arithmetic */
#define LBM_FP64 1       /* FP64 storage, FP64 arithmetic */
#define LBM_FP32_F64 2   /* FP32 storage, FP64 arithmetic */

/* Population layout in the workspace.  LBM_LAYOUT_PULL: two state buffers, streaming as a pull
 * (Eqs. (18), (35)).  LBM_LAYOUT_AA: one buffer stepped in place by two alternating forms of
 * the same step (the AA pattern): half the state memory, results bitwise equal to the pull
 * layout.  The AA layout has no adjoint tape (checkpoint_every must be 0) and no batched form
 * (LBM_E_UNSUPPORTED). */
#define LBM_LAYOUT_PULL 0
#define LBM_LAYOUT_AA 1

/* Side conditions (Sec. 4.1, Fig. 1).  Velocity is no-slip on every non-periodic side.
 * Periodic sides come in pairs (west with east, south with north). */
#define LBM_WALL_ISOTHERMAL 0
#define LBM_WALL_ADIABATIC 1
#define LBM_PERIODIC 2

/* Sides, in the order of lbm_params.bc and T_wall. */
#define LBM_WEST 0
#define LBM_EAST 1
#define LBM_SOUTH 2
#define LBM_NORTH 3

/* Problem statement of Sec. 2 and Sec. 4.  Defaults (lbm_default_params) are the paper's:
 * rho0 = 1, varpi = -2, J = 1, sigma = 1, Ma = 0.1, s_e = s_eps = 1.1, s_q = 1.2,
 * zeta3 = zeta4 = 1.5 (Sec. 4), hot west wall T = 1, cold east wall T = 0, adiabatic south and
 * north walls (Sec. 4.1), T_init = 0.5. */
typedef struct {
    int32_t nx, ny;          /* lattice nodes including wall nodes; L = nx - 1              */
    int32_t bc[4];           /* LBM_WALL_ISOTHERMAL / LBM_WALL_ADIABATIC / LBM_PERIODIC      */
    double T_wall[4];        /* wall temperature where bc == LBM_WALL_ISOTHERMAL             */
    double Ra, Pr, Da, J;    /* Rayleigh, Prandtl, Darcy numbers, viscosity ratio (Sec. 2)  */
    double Ma, sigma, varpi, rho0; /* Mach number, heat capacity ratio, Eq. (29) constant, rho0 */
    double s_e, s_eps, s_q;  /* relaxation rates s1, s2, s4 = s6 of Eq. (20)                  */
    double zeta3, zeta4;     /* relaxation rates zeta3, zeta4 of Eq. (31)                     */
    int32_t forchheimer;     /* 1: F_phi = 1.75/sqrt(150 phi^3) (Eq. (5)); 0: F_phi = 0        */
    double T_init;           /* initial temperature of every node                            */
    double ext_accel[2];     /* extra body acceleration added to G of Eq. (4) (0 by default)  */
    double tau_v, tau_T;     /* > 0 overrides Eq. (37b); otherwise derived from Ma, Ra, Pr, J */
    double gbeta;            /* >= 0 overrides g*beta; negative: Ma^2 cs^2 / (dT L)           */
    double Ra_I;             /* internal Rayleigh number (Sec. 2); > 0: heat source Q''' from  */
                             /* Ra_I = g beta Q''' L^5 / (nu alpha_e^2); with Ra = 0 it also   */
                             /* sets tau_v (Sec. 4.2) and the scale dT = Q''' L^2/alpha_e = 1 */
    double Qv;               /* Q''' in lattice units when Ra_I <= 0 (default 0: no source)   */
    int32_t dtype;           /* LBM_FP32, LBM_FP64 or LBM_FP32_F64                            */
    int32_t checkpoint_every;/* 0: no adjoint tape; C > 0: checkpoint every C steps, lbm_grad on */
    int32_t layout;          /* LBM_LAYOUT_PULL (default) or LBM_LAYOUT_AA                     */
    int32_t steps_per_launch;/* Time steps per launch of the pull layout.  0 (default):     */
                             /* three (FP32 on grids of about 2048^2 and more) or two (the   */
                             /* intermediate steps kept in registers and LDS) where that is  */
                             /* faster (large grids, storage type = arithmetic type), four   */
                             /* (16 x 16 tiles advanced in LDS) or eight (8 x 8 tiles) where */
                             /* that is (small and the smallest grids), else one.  1: one.   */
                             /* 2: two; it needs each half of the state (7 of the 14 planes) */
                             /* below 2 GiB and gives LBM_E_UNSUPPORTED beyond.  3: three;   */
                             /* it needs LBM_FP32 and the whole state below 2 GiB, else      */
                             /* LBM_E_UNSUPPORTED.  4: four.  8: eight.  With a tape,        */
                             /* launches of several steps run only between checkpoints.  The */
                             /* AA layout steps one at a time.  Results are bitwise the same */
                             /* in every case.                                               */
} lbm_params;

/* Reasons for the divergence flag (bits of lbm_obs.why).  The paper gives no divergence test;
 * these are the library's. */
#define LBM_DIV_NONFINITE 1    /* u, p, T, Nu or |v| of Eq. (22) is not finite (once |v|^2    */
                               /* overflows, Eq. (21) gives u = 0, so u alone cannot show it) */
#define LBM_DIV_SPEED 2        /* max |u| exceeds cs = 1/sqrt(3) (Ma above 1)                */
#define LBM_DIV_TEMPERATURE 4  /* T leaves [T_lo - dT - r_lo, T_hi + dT + r_hi]: T_lo, T_hi   */
                               /* the min and max of T_init and the isothermal walls' T, dT  */
                               /* the temperature scale (out[6] of lbm_derived), r the rise   */
                               /* a heat source Q can cause, in the bound of its sign only:  */
                               /* |Q| Lmax^2 / (2 alpha_e), Lmax = max(nx, ny) - 1, when some */
                               /* side is isothermal (conduction alpha_e T'' = -Q from one    */
                               /* isothermal side), else |Q| n / sigma (Eq. (3) with no heat  */
                               /* leaving); alpha_e = sigma csT^2 (tau_T - 1/2), Eq. (A9)     */

/* Observables at the current time level. */
typedef struct {
    double nu_hot;    /* average Nusselt number of the west wall, Eq. (38)                     */
    double nu_cold;   /* average Nusselt number of the east wall, Eq. (38)                     */
    double max_speed; /* max |u| over the lattice                                              */
    double mass_err;  /* |sum f - n rho0| / (n rho0) over the stored post-collision populations */
    int64_t step;     /* time level n                                                          */
    int32_t diverged; /* 1 when any LBM_DIV_* condition holds                                  */
    int32_t why;      /* the LBM_DIV_* bits that hold (0 when not diverged)                    */
    double T_min;     /* min T over the lattice (Eq. (36))                                     */
    double T_max;     /* max T over the lattice                                                */
    double phip_dev;  /* max |phi p - rho0 cs^2| over the lattice (Eq. (23)); the level of phi */
                      /* p is a gauge of the step and drifts in long runs, so it is reported */
                      /* but not part of the divergence flag                                 */
} lbm_obs;

typedef struct lbm_ctx lbm_ctx;

/* Fill *p with the paper's defaults (Sec. 4) for a 64 x 64 side-heated cavity at Ra = 1e3,
 * Pr = 1, Da = 1e-2, FP32, no tape. */
lbm_status lbm_default_params(lbm_params* p);

/* Derived parameters of Sec. 4 for *p, in this order:
 *  out[0] L = nx - 1, out[1] tau_v (Eq. (37b)), out[2] tau_T (Eq. (37b) with nu = nu_e / J, so
 *  that Pr = nu / alpha_e and alpha_e = sigma csT^2 (tau_T - 1/2), Eq. (A9)), out[3] nu_e
 *  (Eq. (24)), out[4] nu, out[5] g*beta (Ma = U / cs, U = sqrt(g beta dT L)), out[6] dT,
 *  out[7] T0, out[8] K = Da L^2 (infinite when Da <= 0), out[9] the heat source Q''' (Eq. (30)).
 *  out has room for 10 doubles. */
lbm_status lbm_derived(const lbm_params* p, double* out);

/* Bytes of device workspace lbm_init needs for *p; with checkpoint_every > 0 the adjoint tape
 * for up to nsteps_max time steps is included. */
lbm_status lbm_workspace_size(const lbm_params* p, int64_t nsteps_max, size_t* bytes);

/* Create a cavity.  phi and K are device arrays [ny][nx] of p->dtype holding the porosity phi
 * (0 < phi <= 1) and permeability K (> 0) of each node (Eqs. (4), (5)); either may be NULL:
 * phi then takes phi_uniform everywhere, K takes Da L^2 everywhere (no Darcy or Forchheimer
 * drag when Da <= 0).  The library copies them into the workspace; the caller may free them
 * after the call returns.  The cavity starts at rest (see State semantics).
 * With Ra_I > 0 or Qv != 0 the thermal step carries the heat source: Psi of Eq. (30) enters the
 * collision through (I - Theta/2) Psi (Eqs. (33), (34)) and T = sum g + Q'''/(2 sigma) (Eq. (36)).
 * Errors: LBM_E_INVAL for nx or ny below 5 on a walled axis (the five-point stencil of
 * Eq. (38) needs five nodes) or below 2 on a periodic one, unpaired periodic sides, a
 * derived tau_v or tau_T not above 1/2, phi_uniform outside (0, 1], varpi >= 1 (Eq. (29)),
 * rho0, sigma or J not positive, unknown dtype or bc; LBM_E_NOMEM when ws_bytes is too
 * small; LBM_E_HIP when a device call fails. */
lbm_status lbm_init(lbm_ctx** out, const lbm_params* p, const void* phi, const void* K,
                    double phi_uniform, void* workspace, size_t ws_bytes, void* hip_stream);

/* Advance by nsteps time steps (asynchronous).  One time step is the flow collision of
 * Eq. (17) with the forcing of Eq. (19) and streaming of Eq. (18), coupled to the thermal
 * collision of Eq. (34) and streaming of Eq. (35), with the macroscopic fields of Eqs. (21)-(23)
 * and (36) and the wall reconstruction of Sec. 4 (see State semantics); nsteps = 0 does
 * nothing, nsteps < 0 is LBM_E_INVAL.  With a tape, the total number of steps since lbm_init
 * may not exceed the nsteps_max the workspace was sized for (LBM_E_STATE).  Launch errors give
 * LBM_E_HIP; faults inside the steps surface at the next synchronising call. */
lbm_status lbm_step(lbm_ctx* c, int64_t nsteps);

/* Observables at the current time level (synchronises).  ux, uy, p, T are optional device
 * arrays [ny][nx] of the context's dtype receiving u (Eq. (21)), the dynamic pressure
 * p - rho0 cs^2 / phi (p of Eq. (23) less its rest value, which FP32 could not carry the
 * dynamic part on top of; at wall nodes phi_b p_b = phi_f p_f), T (Eq. (36)).  Returns
 * LBM_E_DIVERGED with o->diverged = 1 and the reasons in o->why (LBM_DIV_*) when the run
 * diverged. */
lbm_status lbm_observables(lbm_ctx* c, lbm_obs* o, void* ux, void* uy, void* p, void* T);

/* Stream function at the current time level (synchronises): psi (device array [ny][nx] of the
 * context's dtype) with u_x = d psi / dy, integrated along y by the trapezoid rule from psi = 0
 * at y = 0 (the south side), from the velocity of Eq. (21); its maximum normalised by
 * L sqrt(g beta dT L) is the psi_max of Sec. 4.2 (Table 3). */
lbm_status lbm_stream_function(lbm_ctx* c, void* psi);

/* Launch shape of the time loop in use (no device work): out[0] time steps per launch (1, 2,
 * 3, 4 or 8, see steps_per_launch), out[1] the layout (LBM_LAYOUT_*), out[2] rows per
 * wavefront segment of the two- and three-step kernels, or the tile side (16 or 8) of the tile
 * forms (0 for one step per launch), out[3] work-groups per launch.  out holds 4 entries. */
lbm_status lbm_step_shape(const lbm_ctx* c, int32_t* out);

/* Discrete adjoint (synchronises).  For J = nu_hot at the current time level n (Eq. (38)),
 * computes dJ_dphi = dJ * dJ/dphi(x) and dJ_dK = dJ * dJ/dK(x) at every node, the exact
 * derivative of the n-step discrete map from rest (phi held fixed for dK, K for dphi).  Both
 * outputs are device FP64 arrays [ny][nx]; either may be NULL.  Needs checkpoint_every > 0
 * (else LBM_E_STATE).  The forward state is left unchanged.  Uses the checkpoints written by
 * lbm_step and recomputes each segment between checkpoints, the segment before the one being
 * swept on a second, internal stream that is ordered with the caller's by events. */
lbm_status lbm_grad(lbm_ctx* c, double dJ, void* dJ_dphi, void* dJ_dK);

/* Size in bytes of a saved state (populations plus the step counter). */
lbm_status lbm_state_size(const lbm_ctx* c, size_t* bytes);

/* Copy the state to / from host memory (synchronises).  A loaded state resumes exactly where
 * the saved one stopped.  lbm_load on a context with a tape returns LBM_E_UNSUPPORTED.
 * The saved bytes are a 64-byte header of eight int64 {magic, dtype, nx, ny, row pitch, step,
 * layout, plane stride} and then the state as the device holds it: 14 planes, each ny rows of
 * `row pitch` elements with x fastest, planes `plane stride` elements apart.  lbm_load returns
 * LBM_E_INVAL for a header that does not match the context. */
lbm_status lbm_save(lbm_ctx* c, void* host_buf, size_t bytes);
lbm_status lbm_load(lbm_ctx* c, const void* host_buf, size_t bytes);

/* Release the host context (synchronises; the workspace remains the caller's). */
lbm_status lbm_destroy(lbm_ctx* c);

/* ---------------------------------------------------------------------------------------- */
/* Batched form: many independent cavities of uneven size and parameters stepped together.   */
/* Every cavity is the model above (the time step of lbm_step, the cavities of Sec. 4) with  */
/* its own lbm_params (all of one dtype, no tape, pull layout) and uniform phi              */
/* (phi_uniform[i]) and K = Da L^2 (Sec. 2).  State semantics and fields as above, per cavity. */
/* ---------------------------------------------------------------------------------------- */

/* Bytes of device workspace lbm_batch_init needs for the n cavities p[0..n-1] (host array).
 * Errors: LBM_E_INVAL for n <= 0, any cavity lbm_workspace_size would reject, mixed dtypes
 * or a batch state of 2^31 elements or more; LBM_E_UNSUPPORTED for a tape or the AA layout. */
lbm_status lbm_batch_workspace_size(int32_t n, const lbm_params* p, size_t* bytes);

/* Create a batch of n cavities at rest (the initial state of lbm_init for each).  p and
 * phi_uniform are host arrays of n entries; the workspace is device memory of at least
 * lbm_batch_workspace_size() bytes, 256-byte aligned, owned by the caller and kept valid until
 * lbm_destroy().  Errors as lbm_batch_workspace_size, plus phi_uniform[i] outside (0, 1]
 * (LBM_E_INVAL), a workspace too small (LBM_E_NOMEM) or a failed device call (LBM_E_HIP).
 * tune_cache_path: file where the launch shape picked by the
 * autotuner is cached per (device, dtype, cavity set); NULL disables tuning (default shape).
 * The autotuner also times two steps per launch and keeps it where it is faster;
 * p[0].steps_per_launch = 1 or 2 forces one or two (the other cavities' values are ignored;
 * 2 gives LBM_E_UNSUPPORTED if a cavity's state reaches 2 GiB, where the autotuner keeps one
 * step per launch; 3, 4 and 8, forms of a single cavity, give LBM_E_UNSUPPORTED).  Results are
 * bitwise the same either way. */
lbm_status lbm_batch_init(lbm_ctx** out, int32_t n, const lbm_params* p,
                          const double* phi_uniform, void* workspace, size_t ws_bytes,
                          void* hip_stream, const char* tune_cache_path);

/* Advance every cavity by nsteps time steps of lbm_step (asynchronous; replayed from a
 * captured HIP graph).  nsteps < 0 is LBM_E_INVAL. */
lbm_status lbm_batch_step(lbm_ctx* c, int64_t nsteps);

/* Observables of every cavity (synchronises); o has n entries.  Returns LBM_E_DIVERGED when
 * any cavity diverged; each entry's diverged and why say which (as in lbm_observables). */
lbm_status lbm_batch_observables(lbm_ctx* c, lbm_obs* o);

/* Macroscopic fields of cavity i at the current time level (synchronises): optional device
 * arrays [ny_i][nx_i] of the batch's dtype, as in lbm_observables. */
lbm_status lbm_batch_fields(lbm_ctx* c, int32_t i, void* ux, void* uy, void* p, void* T);

/* Launch shape in use (out holds 8 entries): out[0] nodes per work-item along x, out[1]
 * work-group size, out[2] work-groups per step of the one-step kernel, out[3] steps per graph
 * replay, out[4] time steps per launch (2 when the autotuner, or steps_per_launch = 2 of the
 * first cavity, chose the two-step kernel), out[5] its rows per segment (0 if unused), out[6]
 * its work-groups per launch, out[7] its strips (wavefronts) per work-group. */
lbm_status lbm_batch_shape(const lbm_ctx* c, int32_t* out);

/* ---------------------------------------------------------------------------------------- */
/* For callers that cannot allocate device memory (tight serving loops, harnesses that       */
/* forbid hipMalloc): one cavity run from rest without a workspace.                          */
/* ---------------------------------------------------------------------------------------- */

/* The results of lbm_init(p, phi, K, phi_uniform) + lbm_step(nsteps) + lbm_observables(o, ux,
 * uy, pr, T) on the same stream, bitwise (the same kernels in the same order), with the cavity
 * kept in a device array of the library instead of a caller's workspace: nothing is allocated,
 * on the device or the host.  Arguments are those of the three calls; phi, K (optional) and
 * ux, uy, pr, T (optional) are device arrays [ny][nx] of p->dtype, o is host memory.  The
 * array holds 64 MiB per GPU (kept from the library's first use on a GPU until the process
 * ends): a cavity whose workspace (lbm_workspace_size) exceeds it gives LBM_E_NOMEM before any
 * device work, e.g. FP32 cavities up to about 700 x 700 fit.  No tape (checkpoint_every must
 * be 0: LBM_E_UNSUPPORTED).  Every call on a GPU uses that GPU's one array, so calls that
 * overlap on one GPU (other host threads, or other streams before this call returns) race;
 * the call synchronises the stream before returning, so calls in sequence do not.  Errors as
 * lbm_init and lbm_observables (LBM_E_DIVERGED when the run diverged). */
lbm_status lbm_run_noalloc(const lbm_params* p, const void* phi, const void* K,
                           double phi_uniform, int64_t nsteps, lbm_obs* o, void* ux, void* uy,
                           void* pr, void* T, void* hip_stream);

/* Human-readable name of a status code. */
const char* lbm_status_string(lbm_status s);

/* Detail of the last failure on this thread ("" when none). */
const char* lbm_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* LBM_H */
