"""Pins of the CPU oracle's single-node formulas against facts the paper and algebra fix.

Each test names the passage of arXiv:1308.2071 it follows.  None of them re-types an oracle
formula and compares it with itself: they check identities that link two different printed
formulas (e.g. Eq. (13) and Eq. (16)), closed forms, or a textbook special case.
"""
import numpy as np
import pytest

from oracle import ref

W9 = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)
EX = np.array([0, 1, 0, -1, 0, 1, -1, -1, 1])
EY = np.array([0, 0, 1, 0, -1, 1, 1, -1, -1])


def rng_cases(n=25, seed=7):
    r = np.random.default_rng(seed)
    for _ in range(n):
        yield dict(phip=r.uniform(0.1, 0.6), ux=r.uniform(-0.1, 0.1), uy=r.uniform(-0.1, 0.1),
                   phi=r.uniform(0.2, 1.0), Fx=r.uniform(-1e-3, 1e-3), Fy=r.uniform(-1e-3, 1e-3),
                   T=r.uniform(-1, 2))


def test_transforms_orthogonal_and_inverse(oracle):
    """Eqs. (11), (28): rows of M and N are mutually orthogonal with the stated norms, and the
    oracle's inverses invert them (P1)."""
    M, Mi, N, Ni = ref.matrices()
    np.testing.assert_allclose(M @ M.T, np.diag([9, 36, 36, 6, 12, 6, 12, 4, 4]), atol=0)
    np.testing.assert_allclose(N @ N.T, np.diag([5, 2, 2, 20, 4]), atol=0)
    np.testing.assert_allclose(Mi @ M, np.eye(9), atol=1e-15)
    np.testing.assert_allclose(M @ Mi, np.eye(9), atol=1e-15)
    np.testing.assert_allclose(Ni @ N, np.eye(5), atol=1e-15)
    # rows of M are the moments of Eq. (10): density, momentum and stress rows from e_i
    np.testing.assert_array_equal(M[3], EX)
    np.testing.assert_array_equal(M[5], EY)
    np.testing.assert_array_equal(M[7], EX ** 2 - EY ** 2)
    np.testing.assert_array_equal(M[8], EX * EY)


def test_meq_is_M_times_feq(oracle):
    """Eq. (15)-(16) equal M applied to Eq. (13)-(14) (the paper derives one from the other)."""
    M, _, _, _ = ref.matrices()
    for c in rng_cases():
        f = ref.feq(c["phip"], c["ux"], c["uy"], c["phi"])
        m = ref.meq(c["phip"], c["ux"], c["uy"], c["phi"])
        np.testing.assert_allclose(M @ f, m, atol=2e-15)


def test_neq_is_N_times_geq(oracle):
    """Eq. (29) equals N applied to the BGK-equivalent equilibrium of Eq. (37a)."""
    _, _, N, _ = ref.matrices()
    for varpi in (-2.0, -1.0, 0.5):
        for c in rng_cases(10):
            g = ref.geq(c["T"], c["ux"], c["uy"], sigma=1.3, varpi=varpi)
            n = ref.neq(c["T"], c["ux"], c["uy"], sigma=1.3, varpi=varpi)
            np.testing.assert_allclose(N @ g, n, atol=3e-15)


def guo_zhao_forcing(ux, uy, Fx, Fy, phi, rho0=1.0):
    """Velocity-space porous forcing of Guo and Zhao (the paper's ref. [19]) without the
    (1 - 1/(2 tau)) factor: w_i rho0 [e.F/cs2 + (e.u)(e.F)/(phi cs4) - u.F/(phi cs2)]."""
    cs2 = 1 / 3
    eF = EX * Fx + EY * Fy
    eu = EX * ux + EY * uy
    uF = ux * Fx + uy * Fy
    return W9 * rho0 * (eF / cs2 + eu * eF / (phi * cs2 ** 2) - uF / (phi * cs2))


def test_moment_forcing_is_M_times_guo_zhao(oracle):
    """Eq. (19) is the moment-space image of the Guo-Zhao velocity-space forcing."""
    M, _, _, _ = ref.matrices()
    for c in rng_cases():
        S = ref.forcing(c["ux"], c["uy"], c["Fx"], c["Fy"], c["phi"])
        S_v = M @ guo_zhao_forcing(c["ux"], c["uy"], c["Fx"], c["Fy"], c["phi"])
        np.testing.assert_allclose(S, S_v, atol=1e-17)


def test_feq_moments(oracle):
    """Eq. (13): sum f_eq = rho0, sum e f_eq = rho0 u, and sum e_a e_b f_eq = phi p delta +
    rho0 u_a u_b / phi (the porous incompressible equilibrium's defining moments)."""
    for c in rng_cases():
        f = ref.feq(c["phip"], c["ux"], c["uy"], c["phi"])
        assert abs(f.sum() - 1.0) < 1e-15
        assert abs((EX * f).sum() - c["ux"]) < 1e-16
        assert abs((EY * f).sum() - c["uy"]) < 1e-16
        Pxx = (EX * EX * f).sum()
        Pxy = (EX * EY * f).sum()
        assert abs(Pxx - (c["phip"] + c["ux"] ** 2 / c["phi"])) < 1e-15
        assert abs(Pxy - c["ux"] * c["uy"] / c["phi"]) < 1e-16


def test_pressure_and_velocity_recovered_from_feq(oracle):
    """Eqs. (21)-(23) return u and phi*p from f_eq(p, u) when there is no drag and no force
    (K = infinity gives l0 = 1/2, l1 = 0, so u = v)."""
    for c in rng_cases():
        f = ref.feq(c["phip"], c["ux"], c["uy"], c["phi"])
        g = ref.geq(0.5, 0, 0)  # T = T0 = 0.5: no buoyancy
        m = ref.macros(f, g, c["phi"], np.inf)
        assert abs(m["ux"] - c["ux"]) < 1e-16
        assert abs(m["uy"] - c["uy"]) < 1e-16
        assert abs(m["phip"] - c["phip"]) < 2e-15
        assert abs(m["T"] - 0.5) < 1e-15


@pytest.mark.parametrize("forchheimer", [1, 0])
def test_velocity_solves_the_generalized_quadratic(oracle, forchheimer):
    """Eq. (21) solves v = 2 l0 u + l1 |u| u with l0, l1 after Eq. (22) (the defining relation of
    the generalized model's semi-implicit drag); with F_phi = 0 it reduces to u = v/(2 l0)."""
    r = np.random.default_rng(3)
    d = ref.derived(Ra=1e4, Pr=0.71, nx=65)
    for _ in range(20):
        phi, K = r.uniform(0.2, 0.95), r.uniform(1e-2, 50)
        f = W9 * (1 + r.uniform(-0.3, 0.3, 9))
        g = ref.geq(0.5, 0, 0)
        m = ref.macros(f, g, phi, K, Ra=1e4, Pr=0.71, nx=65, forchheimer=forchheimer)
        vx, vy = (EX * f).sum(), (EY * f).sum()
        Fphi = 1.75 / np.sqrt(150 * phi ** 3) if forchheimer else 0.0
        l0 = 0.5 * (1 + phi * 0.5 * d["nu"] / K)
        l1 = phi * 0.5 * Fphi / np.sqrt(K)
        um = np.hypot(m["ux"], m["uy"])
        np.testing.assert_allclose([2 * l0 * m["ux"] + l1 * um * m["ux"],
                                    2 * l0 * m["uy"] + l1 * um * m["uy"]], [vx, vy],
                                   rtol=1e-13, atol=1e-17)
        if not forchheimer:
            np.testing.assert_allclose([m["ux"], m["uy"]], [vx / (2 * l0), vy / (2 * l0)],
                                       rtol=1e-14, atol=1e-17)


def test_collision_conserves_mass_heat_and_gives_momentum(oracle):
    """Eq. (17) with s0 = s3 = s5 = 1 and m0_eq = rho0: sum f+ = rho0 at every node; Eq. (34)
    with zeta0 = 1: sum g+ = T; and the post-collision momentum is rho0 u + rho0 F / 2, i.e.
    the full body force acts over one step (P4)."""
    r = np.random.default_rng(11)
    P = dict(Ra=1e5, Pr=1.0, nx=129, ext_accel=(1e-5, -2e-5))
    for _ in range(20):
        phi, K = r.uniform(0.2, 0.95), r.uniform(0.5, 50)
        f = W9 * (1 + r.uniform(-0.2, 0.2, 9))
        g = ref.geq(r.uniform(0, 1), 0, 0) * (1 + r.uniform(-0.2, 0.2, 5))
        fp, gp = ref.collide_fluid_node(f, g, phi, K, **P)
        m = ref.macros(f, g, phi, K, **P)
        assert abs(fp.sum() - 1.0) < 1e-15
        assert abs(gp.sum() - g.sum()) < 1e-15
        np.testing.assert_allclose((EX * fp).sum(), m["ux"] + 0.5 * m["Fx"], atol=1e-17)
        np.testing.assert_allclose((EY * fp).sum(), m["uy"] + 0.5 * m["Fy"], atol=1e-17)


def test_equilibrium_is_a_fixed_point_without_force(oracle):
    """A node already at f_eq(p, u), g_eq(T, u), with no body force, stays there."""
    P = dict(Ra=1e5, Pr=1.0, nx=129, gbeta=0.0, Da=0.0, forchheimer=0)
    for c in rng_cases(10):
        f = ref.feq(c["phip"], c["ux"], c["uy"], c["phi"])
        g = ref.geq(c["T"], c["ux"], c["uy"])
        fp, gp = ref.collide_fluid_node(f, g, c["phi"], np.inf, **P)
        np.testing.assert_allclose(fp, f, atol=1e-16)
        np.testing.assert_allclose(gp, g, atol=2e-16)


def test_derived_parameters_by_hand(oracle):
    """Eq. (37b), Eq. (24), Eq. (A9) and the Ma definition of Sec. 4, evaluated by hand for the
    64x64, Ra = 1e3 cavity: tau_v = 1/2 + sqrt(3) 0.1 * 63 * sqrt(1/1000)."""
    d = ref.derived(nx=64, ny=64, Ra=1e3, Pr=1.0, Da=1e-2)
    tv = 0.5 + 0.1 * 63 * np.sqrt(3.0) * np.sqrt(1e-3)
    assert d["tau_v"] == pytest.approx(tv, rel=1e-15)
    assert d["tau_v"] == pytest.approx(0.845065, abs=1e-6)
    assert d["nu_e"] == pytest.approx((tv - 0.5) / 3, rel=1e-15)
    # alpha_e = sigma (4 + varpi)/10 (tau_T - 1/2) = nu / Pr
    assert 0.2 * (d["tau_T"] - 0.5) == pytest.approx(d["nu"] / 1.0, rel=1e-15)
    assert d["tau_T"] == pytest.approx(1.075109, abs=1e-6)
    assert d["K_uniform"] == pytest.approx(39.69, rel=1e-15)
    # Ma = U / cs, U = sqrt(g beta dT L), dT = 1
    assert np.sqrt(d["gbeta"] * 1.0 * 63) / np.sqrt(1 / 3) == pytest.approx(0.1, rel=1e-15)
    # Ra = g beta dT L^3 / (nu alpha_e) with alpha_e = nu / Pr is then 1e3
    alpha = 0.2 * (d["tau_T"] - 0.5)
    assert d["gbeta"] * 63 ** 3 / (d["nu"] * alpha) == pytest.approx(1e3, rel=1e-13)
