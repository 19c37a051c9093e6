"""Pins of the CPU oracle's whole time step against what the paper and the mathematics fix:
exact conservation, the LBGK special case, closed-form solutions of the macroscopic equations
(Eqs. (2), (3)), conduction Nu = 1, the centro-symmetry of the side-heated cavity and the
paper's own Table 2 value.  Each test states the passage it follows.
"""
import os

import numpy as np
import pytest
from scipy.integrate import solve_bvp

from oracle import ref

W9 = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)
EX = np.array([0, 1, 0, -1, 0, 1, -1, -1, 1])
EY = np.array([0, 0, 1, 0, -1, 1, 1, -1, -1])
P_ALL = (ref.PERIODIC,) * 4
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def perturbed_state(ny, nx, seed, T0=0.5, amp_f=0.05, amp_T=0.2):
    r = np.random.default_rng(seed)
    f = W9[:, None, None] * (1 + amp_f * r.uniform(-1, 1, (9, ny, nx)))
    wt = np.array([0.6, 0.1, 0.1, 0.1, 0.1])
    g = wt[:, None, None] * (T0 + amp_T * r.uniform(-1, 1, (5, ny, nx)))
    return f, g


def test_periodic_box_conserves_total_mass_and_heat(oracle):
    """Eq. (17) with s0 = 1 and m0_eq = rho0 conserves mass node by node and streaming moves it;
    Eq. (34) with zeta0 = 1 and no source conserves heat.  Over 1000 steps of a periodic box
    with buoyancy and per-node drag both totals stay put (P4)."""
    nx, ny = 12, 10
    r = np.random.default_rng(5)
    phi = r.uniform(0.3, 0.9, (ny, nx))
    K = r.uniform(1, 20, (ny, nx))
    lat = ref.RefLattice(phi=phi, K=K, nx=nx, ny=ny, bc=P_ALL, Ra=1e4, Pr=0.71)
    f0, g0 = perturbed_state(ny, nx, 1)
    lat.set_state(f0, g0)
    heat0 = g0.sum()
    # m0^eq = rho0 with s0 = 1 sets every node's post-collision mass to rho0 from the first
    # collision on, whatever the initial populations held
    lat.step(1)
    f1, _ = lat.get_state()
    assert abs(f1.sum() - nx * ny) / (nx * ny) < 1e-15
    lat.step(1000)
    f, g = lat.get_state()
    assert abs(f.sum() - nx * ny) / (nx * ny) < 1e-13
    assert abs(g.sum() - heat0) / heat0 < 1e-13
    # every node's post-collision mass is rho0 exactly (to rounding)
    np.testing.assert_allclose(f.sum(0), 1.0, atol=1e-14)


def bgk_step(f, g, phi, K, d, gbeta, T0, tau_v, tau_T, Q=0.0):
    """Independent velocity-space LBGK with the porous equilibrium of Eq. (13)-(14), the Guo-Zhao
    forcing, the D2Q5 equilibrium of Eq. (37a) and a heat source wt_i (1 - 1/(2 tau_T)) Q with
    T = sum g + Q/2 (sigma = 1); periodic streaming.  This is the scheme the MRT step must
    reduce to when all rates equal 1/tau (end of Sec. 3.1 and Sec. 3.2)."""
    cs2, nu = 1 / 3, d["nu"]
    T = g.sum(0) + 0.5 * Q
    Gy = gbeta * (T - T0)
    vx = (EX[:, None, None] * f).sum(0) + 0.5 * phi * 0.0
    vy = (EY[:, None, None] * f).sum(0) + 0.5 * phi * Gy
    Fphi = 1.75 / np.sqrt(150 * phi ** 3)
    l0 = 0.5 * (1 + 0.5 * phi * nu / K)
    l1 = 0.5 * phi * Fphi / np.sqrt(K)
    den = l0 + np.sqrt(l0 ** 2 + l1 * np.hypot(vx, vy))
    ux, uy = vx / den, vy / den
    uu = ux ** 2 + uy ** 2
    phip = cs2 / (1 - W9[0]) * (f[1:].sum(0) - W9[0] * uu / (2 * phi * cs2))
    um = np.sqrt(uu)
    Fx = -phi * nu / K * ux - phi * Fphi / np.sqrt(K) * um * ux
    Fy = -phi * nu / K * uy - phi * Fphi / np.sqrt(K) * um * uy + phi * Gy
    fp = np.empty_like(f)
    for i in range(9):
        eu = EX[i] * ux + EY[i] * uy
        eF = EX[i] * Fx + EY[i] * Fy
        s = W9[i] * (eu / cs2 + eu ** 2 / (2 * phi * cs2 ** 2) - uu / (2 * phi * cs2))
        fe = (1 - (1 - W9[0]) * phip / cs2 if i == 0 else W9[i] * phip / cs2) + s
        Fi = W9[i] * (eF / cs2 + eu * eF / (phi * cs2 ** 2) - (ux * Fx + uy * Fy) / (phi * cs2))
        fp[i] = f[i] - (f[i] - fe) / tau_v + (1 - 0.5 / tau_v) * Fi
    wt = np.array([0.6, 0.1, 0.1, 0.1, 0.1])
    gp = np.empty_like(g)
    for i in range(5):
        ge = wt[i] * T * (1 + (EX[i] * ux + EY[i] * uy) / 0.2)
        gp[i] = g[i] - (g[i] - ge) / tau_T + (1 - 0.5 / tau_T) * wt[i] * Q
    for i in range(9):
        fp[i] = np.roll(fp[i], (EY[i], EX[i]), axis=(0, 1))
    for i in range(5):
        gp[i] = np.roll(gp[i], (EY[i], EX[i]), axis=(0, 1))
    return fp, gp


@pytest.mark.parametrize("Q", [0.0, 4e-4])
def test_mrt_with_equal_rates_is_lbgk(oracle, Q):
    """With Lambda = I / tau_v and Theta = I / tau_T the MRT scheme is the LBGK scheme with the
    equilibria of Eq. (13) and Eq. (37a) (end of Sec. 3.1, Sec. 3.2) -- P5.  With a heat source,
    N^-1 (I - Theta/2) Psi of Eqs. (30), (34) is the velocity-space source
    wt_i (1 - 1/(2 tau_T)) Q''' / sigma only if Psi3 = varpi Q''' / sigma."""
    nx, ny = 6, 5
    r = np.random.default_rng(2)
    phi = r.uniform(0.3, 0.9, (ny, nx))
    K = r.uniform(0.5, 5, (ny, nx))
    P = dict(nx=nx, ny=ny, bc=P_ALL, Ra=1e4, Pr=0.71, uniform_rates=1, tau_v=0.7, tau_T=0.9,
             gbeta=2e-3, Qv=Q)
    d = ref.derived(**P)
    lat = ref.RefLattice(phi=phi, K=K, **P)
    f, g = perturbed_state(ny, nx, 9)
    lat.set_state(f, g)
    # the oracle state is post-collision; the BGK recursion below streams last, so bring it
    # to the same phase by streaming once first
    for i in range(9):
        f[i] = np.roll(f[i], (EY[i], EX[i]), axis=(0, 1))
    for i in range(5):
        g[i] = np.roll(g[i], (EY[i], EX[i]), axis=(0, 1))
    for _ in range(100):
        f, g = bgk_step(f, g, phi, K, d, 2e-3, d["T0"], 0.7, 0.9, Q)
    lat.step(100)
    fo, go = lat.get_state()
    # oracle holds post-collision values; stream them to compare with the BGK post-stream ones
    for i in range(9):
        fo[i] = np.roll(fo[i], (EY[i], EX[i]), axis=(0, 1))
    for i in range(5):
        go[i] = np.roll(go[i], (EY[i], EX[i]), axis=(0, 1))
    np.testing.assert_allclose(fo, f, atol=1e-13)
    np.testing.assert_allclose(go, g, atol=1e-13)


def test_conduction_gives_linear_T_and_unit_nusselt(oracle):
    """Without buoyancy the side-heated cavity conducts: T is linear in x and both walls have
    Nu = 1 exactly (Eq. (38) with L = nx - 1).  Pins the thermal wall reconstruction, the
    adiabatic walls, the five-point derivative and the trapezoid average (P6)."""
    nx, ny = 17, 13
    lat = ref.RefLattice(phi_uniform=0.6, nx=nx, ny=ny, Ra=100.0, Pr=1.0, gbeta=0.0)
    lat.step(20000)
    o = lat.observables()
    assert abs(o["nu_hot"] - 1.0) < 1e-10
    assert abs(o["nu_cold"] - 1.0) < 1e-10
    x = np.arange(nx)
    np.testing.assert_allclose(o["T"], np.broadcast_to(1 - x / (nx - 1), (ny, nx)), atol=1e-10)
    assert o["max_speed"] < 1e-12


def test_weak_buoyancy_approaches_conduction(oracle):
    """As Ra falls the convective contribution vanishes and Nu -> 1 from above (P6)."""
    devs = []
    for Ra in (1e3, 1e2, 1e1):
        lat = ref.RefLattice(phi_uniform=1.0, nx=17, ny=17, Ra=Ra, Pr=1.0, Da=1e8,
                             forchheimer=0)
        lat.step(8000)
        o = lat.observables()
        devs.append(o["nu_hot"] - 1.0)
    assert devs[0] > devs[1] > devs[2] > 0
    assert devs[2] < 1e-3


def channel_profile_darcy_brinkman(y, H, G, K, nu, nu_e, phi):
    r = np.sqrt(phi * nu / (K * nu_e))
    return G * K / nu * (1 - np.cosh(r * (y - H / 2)) / np.cosh(r * H / 2))


def channel_profile_forchheimer(y, H, G, K, nu, nu_e, phi, Fphi):
    """Brinkman-Forchheimer fully developed channel flow, Eq. (2) with Eq. (4):
    nu_e u'' = (phi nu / K) u + (phi Fphi / sqrt K) u^2 - phi G, u(0) = u(H) = 0."""
    a, b, c = phi * nu / (K * nu_e), phi * Fphi / (np.sqrt(K) * nu_e), phi * G / nu_e

    def rhs(s, U):
        return np.vstack([U[1], a * U[0] + b * U[0] ** 2 - c])

    def bcs(U0, U1):
        return np.array([U0[0], U1[1]])

    s = np.linspace(0, H / 2, 2001)
    guess = np.vstack([G * K / nu * np.ones_like(s) * 0.5, np.zeros_like(s)])
    sol = solve_bvp(rhs, bcs, s, guess, tol=1e-12, max_nodes=200000)
    assert sol.success
    yy = np.where(y <= H / 2, y, H - y)
    return sol.sol(yy)[0]


@pytest.mark.parametrize("forchheimer", [0, 1])
def test_porous_channel_closed_form(oracle, forchheimer):
    """Fully developed flow between two walls driven by a body force: the generalized model's
    Eq. (2) with the drag of Eq. (4) has a closed form (F_phi = 0, Brinkman-extended Darcy) or
    a first-integral solution (F_phi > 0).  The oracle matches it to second order in the
    lattice spacing: observed order -> 2 over H = 16 ... 128 (P7)."""
    phi, tau, Da, umax = 0.5, 0.8, 0.01, 0.01
    errs = []
    for ny in (17, 33, 65, 129):
        H = ny - 1
        K = Da * H * H
        nu = nu_e = (tau - 0.5) / 3
        G = umax * nu / K
        P = dict(nx=4, ny=ny, bc=(ref.PERIODIC, ref.PERIODIC, ref.ADIABATIC, ref.ADIABATIC),
                 tau_v=tau, tau_T=0.8, forchheimer=forchheimer, ext_accel=(G, 0.0), T_init=0.5)
        lat = ref.RefLattice(phi_uniform=phi, K=np.full((ny, 4), K), **P)
        rate = nu_e * (np.pi / H) ** 2 + phi * nu / K
        lat.step(int(32 / rate))
        o = lat.observables()
        y = np.arange(ny, dtype=float)
        if forchheimer:
            Fphi = 1.75 / np.sqrt(150 * phi ** 3)
            ua = channel_profile_forchheimer(y, H, G, K, nu, nu_e, phi, Fphi)
        else:
            ua = channel_profile_darcy_brinkman(y, H, G, K, nu, nu_e, phi)
        ul = o["ux"][:, 1]
        np.testing.assert_allclose(o["ux"], np.repeat(ul[:, None], 4, axis=1), atol=1e-15)
        # the discrete steady state keeps a tiny wall-normal velocity, first order in the
        # lattice spacing (incompressibility holds only up to the scheme's truncation error)
        assert np.abs(o["uy"]).max() < 1e-3 * umax * 17 / ny
        errs.append(np.linalg.norm(ul - ua) / np.linalg.norm(ua))
    assert errs[2] < 1.5e-3 and errs[3] < 4e-4, errs
    orders = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(orders > 1.6) and orders[-1] > 1.75, (errs, orders)


def mode_amplitude(a, axis_len, axis):
    k = 2 * np.pi / axis_len
    s = np.sin(k * np.arange(axis_len))
    prof = a.mean(axis=1 - axis)
    return 2.0 / axis_len * (prof * s).sum()


def test_shear_wave_decay_rate(oracle):
    """A shear wave u_x = A sin(k y) in a periodic porous box without Forchheimer drag decays at
    nu_e k^2 + phi nu / K, the linearisation of Eq. (2) with Eq. (4) (P8).  The discrete rate
    converges to it at second order in k."""
    phi, tau, K = 0.7, 0.8, 400.0
    errs = []
    for n in (32, 64):
        P = dict(nx=4, ny=n, bc=P_ALL, tau_v=tau, tau_T=0.8, forchheimer=0, gbeta=0.0)
        d = ref.derived(**P)
        lat = ref.RefLattice(phi_uniform=phi, K=np.full((n, 4), K), **P)
        k = 2 * np.pi / n
        y = np.arange(n)
        ux = 1e-3 * np.sin(k * y)
        f = np.empty((9, n, 4))
        for yy in range(n):
            f[:, yy, :] = ref.feq(1 / 3, ux[yy], 0.0, phi)[:, None]
        g = np.array([0.6, 0.1, 0.1, 0.1, 0.1])[:, None, None] * 0.5 * np.ones((5, n, 4))
        lat.set_state(f, g)
        lat.step(200)
        a1 = mode_amplitude(lat.observables()["ux"], n, 0)
        lat.step(1000)
        a2 = mode_amplitude(lat.observables()["ux"], n, 0)
        rate = np.log(a1 / a2) / 1000
        exact = d["nu_e"] * k * k + phi * d["nu"] / K
        errs.append(abs(rate - exact) / exact)
    assert errs[-1] < 2e-3, errs
    assert errs[0] / errs[1] > 3.0, errs


@pytest.mark.parametrize("sigma,derived", [(1.0, False), (0.7, True)])
def test_thermal_mode_decay_rate(oracle, sigma, derived):
    """T - T0 = A sin(k x) at rest decays at alpha_e k^2 / sigma (Eq. (3)) with alpha_e =
    sigma (4 + varpi)/10 (tau_T - 1/2) (Eq. (A9)) (P9); second order in k.  With tau_T derived
    from the problem statement, alpha_e must equal nu / Pr (definition of Pr, Sec. 2)."""
    errs = []
    for n in (32, 64):
        P = dict(nx=n, ny=4, bc=P_ALL, tau_v=0.8, tau_T=0.9, gbeta=0.0, T_init=0.5, sigma=sigma)
        if derived:
            P.update(tau_v=-1.0, tau_T=-1.0, Ra=1e3, Pr=2.0)
        lat = ref.RefLattice(phi_uniform=0.6, **P)
        k = 2 * np.pi / n
        T = 0.5 + 0.1 * np.sin(k * np.arange(n))
        f = np.broadcast_to(W9[:, None, None], (9, 4, n)).copy()
        g = np.array([0.6, 0.1, 0.1, 0.1, 0.1])[:, None, None] * T[None, None, :] * np.ones(
            (5, 4, n))
        lat.set_state(f, g)
        lat.step(100)
        a1 = mode_amplitude(lat.observables()["T"].T - 0.5, n, 0)
        lat.step(1000)
        a2 = mode_amplitude(lat.observables()["T"].T - 0.5, n, 0)
        rate = np.log(a1 / a2) / 1000
        if derived:
            alpha = ref.derived(**P)["nu"] / 2.0          # alpha_e = nu / Pr
        else:
            alpha = sigma * (4 - 2) / 10 * (0.9 - 0.5)    # Eq. (A9)
        want = alpha * k * k / sigma
        errs.append(abs(rate - want) / want)
    assert errs[-1] < 2e-3, errs
    assert errs[0] / errs[1] > 3.0, errs


def test_centro_symmetry_of_side_heated_cavity(oracle):
    """With T_h = 1/2, T_c = -1/2 and T0 = 0 the side-heated cavity of Sec. 4.1 is symmetric
    under the point reflection x -> (nx-1-x, ny-1-y) with u -> -u, T -> -T, p -> p; the discrete
    scheme keeps this exactly (the reflection maps e_i to -e_i and flips the sign of the
    buoyancy), so Nu_hot = Nu_cold at every step (P10).  A wrong sign in the force, a
    transposed index or an asymmetric wall rule breaks it."""
    nx, ny = 14, 11
    r = np.random.default_rng(4)
    a = r.uniform(0.35, 0.85, (ny, nx))
    phi = 0.5 * (a + a[::-1, ::-1])
    b = r.uniform(2, 30, (ny, nx))
    K = 0.5 * (b + b[::-1, ::-1])
    lat = ref.RefLattice(phi=phi, K=K, nx=nx, ny=ny, Ra=1e5, Pr=0.71,
                         T_wall=(0.5, -0.5, 0.0, 0.0), T_init=0.0)
    for _ in range(6):
        lat.step(50)
        o = lat.observables()
        assert o["max_speed"] > 1e-4
        assert abs(o["nu_hot"] - o["nu_cold"]) < 1e-12
        np.testing.assert_allclose(o["ux"], -o["ux"][::-1, ::-1], atol=1e-14)
        np.testing.assert_allclose(o["uy"], -o["uy"][::-1, ::-1], atol=1e-14)
        np.testing.assert_allclose(o["T"], -o["T"][::-1, ::-1], atol=1e-13)
        np.testing.assert_allclose(o["p"], o["p"][::-1, ::-1], atol=1e-13)


def load_table2():
    rows = {}
    with open(os.path.join(GOLDEN, "paper_table2_nu.txt")) as fh:
        for line in fh:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            Da, Ra, phi, nu = line.split()
            rows[(float(Da), float(Ra), float(phi))] = float(nu)
    return rows


@pytest.mark.slow
def test_porous_cavity_nusselt_against_table2(oracle):
    """Sec. 4.1, Table 2: phi = 0.6, Da = 1e-2, Ra = 1e3, Pr = 1 gives a left-wall average
    Nu = 1.012 on the paper's 120x120 grid.  The 64x64 cavity after 20k steps (from rest at
    T = 0.5) lands within 0.01 of it (context check of the whole model, P11)."""
    tab = load_table2()
    target = tab[(1e-2, 1e3, 0.6)]
    assert target == 1.012
    lat = ref.RefLattice(phi_uniform=0.6, nx=64, ny=64, Ra=1e3, Pr=1.0, Da=1e-2)
    lat.step(20000)
    o = lat.observables()
    assert abs(o["nu_hot"] - target) < 0.01
    assert abs(o["nu_hot"] - o["nu_cold"]) < 1e-3


def test_heat_source_energy_balance(oracle):
    """Eqs. (30), (34), (36): with a uniform heat source Q''' and no flow, every node's
    temperature rises by Q'''/sigma per step (sigma dT/dt = Q''', Eq. (3)); at t = 0 the
    macroscopic T already carries the half-step shift Q'''/(2 sigma) of Eq. (36)."""
    Q, sigma, n = 3e-4, 0.8, 200
    P = dict(nx=6, ny=5, bc=P_ALL, gbeta=0.0, Qv=Q, sigma=sigma, T_init=0.25, tau_v=0.7,
             tau_T=0.8)
    lat = ref.RefLattice(phi_uniform=0.5, **P)
    T0 = lat.observables()["T"]
    np.testing.assert_allclose(T0, 0.25 + 0.5 * Q / sigma, atol=1e-15)
    lat.step(n)
    np.testing.assert_allclose(lat.observables()["T"], T0 + n * Q / sigma, atol=1e-13)


def test_heat_source_conduction_profile(oracle):
    """Steady conduction with a uniform source Q between two walls at T = 0 (Eq. (3) without
    flow): alpha_e T'' = -Q, T = Q x (L - x) / (2 alpha_e), alpha_e = sigma csT^2 (tau_T - 1/2)
    (Eq. (A9)).  The bulk scheme reproduces the quadratic exactly: the deviation from it is one
    constant over all fluid nodes (an O(Q / alpha_e) offset from the wall reconstruction), and
    relative to the profile it falls at second order in the lattice spacing."""
    Q, sigma, tau_T = 2e-5, 1.3, 0.9
    alpha = sigma * 0.2 * (tau_T - 0.5)
    rel = []
    for nx in (17, 33, 65):
        P = dict(nx=nx, ny=4, bc=(ref.ISOTHERMAL, ref.ISOTHERMAL, ref.PERIODIC, ref.PERIODIC),
                 T_wall=(0.0, 0.0, 0.0, 0.0), T_init=0.0, gbeta=0.0, Qv=Q, sigma=sigma,
                 tau_v=0.8, tau_T=tau_T)
        lat = ref.RefLattice(phi_uniform=0.7, **P)
        L = nx - 1
        lat.step(int(30 * L * L / (np.pi ** 2 * alpha / sigma)))
        T = lat.observables()["T"][1]
        x = np.arange(nx)
        exact = Q * x * (L - x) / (2 * alpha)
        dev = (T - exact)[1:-1]
        assert np.ptp(dev) <= 1e-9 * exact.max()
        assert abs(T[0]) < 1e-15 and abs(T[-1]) < 1e-15
        rel.append(abs(dev.mean()) / exact.max())
    assert rel[1] < 1e-3
    orders = np.log2(np.array(rel[:-1]) / np.array(rel[1:]))
    assert np.all(orders > 1.9), (rel, orders)


def test_internal_rayleigh_number_definition(oracle):
    """Sec. 2: Ra_I = g beta Q''' L^5 / (nu alpha_e^2); Sec. 4.2: tau_v from Ra_I when Ra = 0,
    and dT = Q''' L^2 / alpha_e is the temperature scale (taken as 1)."""
    d = ref.derived(nx=121, ny=121, Ra=0.0, Ra_I=6.4e5, Pr=7.0, bc=(0, 0, 0, 0),
                    T_wall=(0.0, 0.0, 0.0, 0.0), T_init=0.0)
    alpha = 0.2 * (d["tau_T"] - 0.5)
    assert d["gbeta"] * d["Q"] * 120 ** 5 / (d["nu"] * alpha ** 2) == pytest.approx(6.4e5,
                                                                                    rel=1e-12)
    assert d["Q"] * 120 ** 2 / alpha == pytest.approx(1.0, rel=1e-12)
    assert d["tau_v"] == pytest.approx(0.5 + 0.1 * 120 * np.sqrt(7.0 / 6.4e5) * np.sqrt(3.0),
                                       rel=1e-14)
    assert d["T0"] == 0.0
    # Sec. 4.3: side heating sets dT = Th - Tc; Q''' then follows from Ra_I
    d = ref.derived(nx=151, Ra=1e5, Ra_I=1e3, Pr=0.7, Da=1e-2)
    alpha = 0.2 * (d["tau_T"] - 0.5)
    assert d["gbeta"] * d["Q"] * 150 ** 5 / (d["nu"] * alpha ** 2) == pytest.approx(1e3,
                                                                                   rel=1e-12)
