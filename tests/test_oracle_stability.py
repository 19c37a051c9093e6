"""Linear stability of the step and the oracle's divergence diagnostic.

The paper fixes the flow relaxation rates at s_e = s_eps = 1.1 and s_q = 1.2 for every case
(Sec. 4), with s_v = 1/tau_v from Eq. (37b).  About the rest state the step is linear in the
populations; a von Neumann analysis of that linear map (written below from Eqs. (11), (16),
(17), (19), (21), (23) and (4), independently of the oracle) shows the bulk step becoming
unstable for tau_v above about 4.6455: the mode alternating in sign from node to node along one
axis (wave number pi) grows.  Cavities 0 (tau_v 4.83) and 9 (tau_v 5.32) of the seeded batched
workload lie beyond that limit; every other cavity of the draw lies within it.  These tests pin
(i) the oracle's growth of that mode to the analysis, (ii) the unstable set of the draw, and
(iii) the oracle's divergence flag on such runs and on states built to trip each criterion.
"""
import os

import numpy as np
import pytest

from oracle import ref
from paper_1308_2071_amd import workloads

EX = np.array([0, 1, 0, -1, 0, 1, -1, -1, 1])
EY = np.array([0, 0, 1, 0, -1, 1, 1, -1, -1])
# rows of Eq. (11): rho, e, eps, j_x, q_x, j_y, q_y, p_xx, p_xy
M = np.array([[1, 1, 1, 1, 1, 1, 1, 1, 1],
              [-4, -1, -1, -1, -1, 2, 2, 2, 2],
              [4, -2, -2, -2, -2, 1, 1, 1, 1],
              [0, 1, 0, -1, 0, 1, -1, -1, 1],
              [0, -2, 0, 2, 0, 1, -1, -1, 1],
              [0, 0, 1, 0, -1, 1, 1, -1, -1],
              [0, 0, -2, 0, 2, 1, 1, -1, -1],
              [0, 1, -1, 1, -1, 0, 0, 0, 0],
              [0, 0, 0, 0, 0, 1, -1, 1, -1]], dtype=float)
GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "batch64_stability.txt")
THRESHOLD = 4.6455  # tau_v where the wave-number-pi mode turns unstable (rates of Sec. 4)


@pytest.fixture(autouse=True)
def one_oracle_thread():
    """The small lattices here run on one oracle thread (OpenMP would only add overhead)."""
    threads = ref.get_threads()
    ref.set_threads(1)
    yield
    ref.set_threads(threads)


def linear_collision(tau_v, c_lin=0.0, rates=(1.1, 1.1, 1.2)):
    """Post-collision deviations as a linear map of post-streaming deviations about rest
    (rho0 = 1, no buoyancy): m = M f, m+ = m - s (m - m_eq) + (1 - s/2) S, f+ = M^-1 m+.
    Linear parts: phi p = cs^2/(1 - w0) sum_{i>=1} f_i (Eq. (23)), u = v / (2 l0) with
    l0 = 1/2 + c_lin/4 (Eq. (21) as |v| -> 0), m_eq = (0, 6 phi p, -9 phi p, u_x, -u_x, u_y, -u_y,
    0, 0) (Eq. (16)), S = (0, 0, 0, F_x, -F_x, F_y, -F_y, 0, 0) with F = -c_lin u (Eqs. (19),
    (4)); c_lin = phi nu / K."""
    s_e, s_eps, s_q = rates
    s = np.array([1, s_e, s_eps, 1, s_q, 1, s_q, 1 / tau_v, 1 / tau_v])
    Minv = np.linalg.inv(M)
    l0 = 0.5 + 0.25 * c_lin
    C = np.zeros((9, 9))
    for j in range(9):
        f = np.zeros(9)
        f[j] = 1.0
        m = M @ f
        phip = (1 / 3) / (1 - 4 / 9) * f[1:].sum()
        ux, uy = (EX @ f) / (2 * l0), (EY @ f) / (2 * l0)
        meq = np.array([0, 6 * phip, -9 * phip, ux, -ux, uy, -uy, 0, 0])
        S = np.array([0, 0, 0, -c_lin * ux, c_lin * ux, -c_lin * uy, c_lin * uy, 0, 0])
        C[:, j] = Minv @ (m - s * (m - meq) + (1 - s / 2) * S)
    return C


def amplification(tau_v, kx, ky, **kw):
    """Largest |eigenvalue| of streaming after collision for the Fourier mode exp(i k.x):
    f_i(x) <- f_i+(x - e_i) multiplies population i by exp(-i k.e_i) (Eq. (18))."""
    C = linear_collision(tau_v, **kw)
    kx, ky = np.broadcast_arrays(np.atleast_1d(kx), np.atleast_1d(ky))
    sh = np.exp(-1j * (kx[:, None] * EX[None, :] + ky[:, None] * EY[None, :]))
    A = sh[:, :, None] * C[None, :, :]
    return np.abs(np.linalg.eigvals(A)).max(axis=1)


def max_amplification(tau_v, n=48, **kw):
    k = np.linspace(0, np.pi, n)
    kx, ky = np.meshgrid(k, k)
    return float(amplification(tau_v, kx.ravel(), ky.ravel(), **kw).max())


def nyquist_run(tau_v, amp, spans):
    """Amplitude of a perturbation alternating in sign along x after each of `spans` steps, in
    the oracle on a periodic 8 x 4 box without buoyancy or drag."""
    lat = ref.RefLattice(phi_uniform=1.0, nx=8, ny=4, bc=(ref.PERIODIC,) * 4, Ra=1e3,
                         Pr=1.0, Da=-1.0, tau_v=tau_v, tau_T=1.0, gbeta=0.0, T_init=0.5)
    f, g = lat.get_state()
    r = np.random.default_rng(3)
    pert = r.standard_normal(9)[:, None, None] * ((-1.0) ** np.arange(8))[None, None, :]
    lat.set_state(f + amp * pert, g, 0)
    out = [np.abs(amp * pert).max()]
    for n in spans:
        lat.step(n)
        out.append(np.abs(lat.get_state()[0] - f).max())
    return out


def nyquist_growth(tau_v, amp=1e-9):
    """Per-step growth of that perturbation over steps 3000..4000 (the least damped eigenmode
    of the wave-number-pi subspace dominates by then)."""
    a = nyquist_run(tau_v, amp, (3000, 1000))
    return (a[2] / a[1]) ** (1.0 / 1000)


def test_linear_analysis_is_neutral_at_small_tau():
    """Below the limit every Fourier mode is damped or neutral (the neutral ones: the pressure
    level, k = 0)."""
    for tau in (0.51, 0.8, 1.5, 3.0, 4.5):
        assert max_amplification(tau) <= 1 + 1e-12, tau


@pytest.mark.parametrize("tau_v", [4.8339, 5.3208])
def test_oracle_growth_of_the_unstable_mode_matches_the_analysis(oracle, tau_v):
    lam = float(amplification(tau_v, np.pi, 0.0)[0])
    assert lam > 1.004
    g = nyquist_growth(tau_v)
    assert abs(g - lam) < 2e-7, (g, lam)


def test_oracle_does_not_grow_that_mode_below_the_limit(oracle):
    """Cavity 33's tau_v (4.08): the wave-number-pi subspace keeps a neutral mode (|lambda| = 1,
    like the pressure level at k = 0) and nothing grows, in the analysis and in the oracle."""
    lam = float(amplification(4.0842, np.pi, 0.0)[0])
    assert abs(lam - 1) < 1e-12
    g = nyquist_growth(4.0842, amp=1e-6)
    assert abs(g - 1) < 1e-9, g


def test_stability_threshold():
    """The wave-number-pi mode turns unstable between tau_v 4.645 and 4.646."""
    assert amplification(THRESHOLD - 5e-4, np.pi, 0.0)[0] <= 1 + 1e-12
    assert amplification(THRESHOLD + 5e-4, np.pi, 0.0)[0] > 1 + 1e-6


def batch64_taus():
    out = []
    for c in workloads.batch64():
        d = ref.derived(**c["params"])
        c_lin = c["phi"] * d["nu"] / d["K_uniform"]
        out.append((d["tau_v"], c_lin))
    return out


def test_unstable_cavities_of_the_batched_draw(oracle):
    """Of the 64 seeded cavities exactly 0 and 9 have a growing mode (drag included)."""
    unstable = [i for i, (tau, cl) in enumerate(batch64_taus())
                if max_amplification(tau, n=24, c_lin=cl) > 1 + 1e-9
                or amplification(tau, np.pi, 0.0, c_lin=cl)[0] > 1 + 1e-9]
    assert unstable == [0, 9]


def read_stability():
    rows = {}
    with open(GOLDEN) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            v = line.split()
            rows[int(v[0])] = dict(side=int(v[1]), tau_v=float(v[6]), first_flag=int(v[7]),
                                   nu_hot=float(v[8]), nu_cold=float(v[9]),
                                   max_speed=float(v[10]), T_min=float(v[11]),
                                   T_max=float(v[12]))
    return rows


@pytest.mark.skipif(not os.path.exists(GOLDEN), reason="stability record not written")
def test_stability_record_flags_exactly_the_unstable_cavities():
    """The oracle's 10,000-step runs of all 64 cavities (stored record) flag exactly the two
    cavities the analysis calls unstable; every other cavity ends finite with T inside the
    walls' range."""
    rows = read_stability()
    assert sorted(rows) == list(range(64))
    flagged = sorted(i for i, r in rows.items() if r["first_flag"] >= 0)
    assert flagged == [0, 9]
    for i, r in rows.items():
        if i in flagged:
            continue
        assert np.isfinite(r["nu_hot"]) and r["max_speed"] < 0.2
        assert -1e-6 <= r["T_min"] and r["T_max"] <= 1 + 1e-6


def small_cavity(**kw):
    p = dict(workloads.cavity(16), Ra=1e4, Pr=0.71, Da=1e-2)
    p.update(kw)
    return ref.RefLattice(phi_uniform=0.6, **p)


def test_healthy_run_is_not_flagged(oracle):
    lat = small_cavity()
    lat.step(300)
    o = lat.observables()
    assert not o["diverged"]
    assert 0 <= o["T_min"] and o["T_max"] <= 1
    assert o["phip_dev_max"] < 1e-2


def test_flag_catches_an_overflowing_velocity(oracle):
    """|v|^2 overflowing makes the denominator of Eq. (21) infinite and u = v/inf = 0; with T
    and p finite, only the |v| check sees it."""
    lat = small_cavity()
    f, g = lat.get_state()
    f[1, 8, 8] = 1e200  # moves east: arrives at (9, 8) with j_x ~ 1e200
    f[3, 8, 10] = -1e200 + 0.25  # the opposite direction, so that mass and pressure stay finite
    lat.set_state(f, g, 0)
    o = lat.observables()
    assert np.isfinite(o["T_max"]) and o["max_speed"] <= 0.1
    assert o["diverged"]


def test_flag_catches_temperature_outside_the_bounds(oracle):
    """T_walls in [0, 1], T_init 0.5, dT 1: T must stay within [-1, 2]."""
    wt = np.array([0.6, 0.1, 0.1, 0.1, 0.1])
    for T_node, flagged in ((1.9, False), (2.1, True), (-0.9, False), (-1.1, True)):
        lat = small_cavity()
        f, g = lat.get_state()
        # after streaming, node (7, 7) gathers g_i from (7 - ex_i, 7 - ey_i)
        for i, (ex, ey) in enumerate(((0, 0), (1, 0), (0, 1), (-1, 0), (0, -1))):
            g[i, 7 - ey, 7 - ex] = wt[i] * T_node
        lat.set_state(f, g, 0)
        o = lat.observables()
        assert abs(o["T_max" if T_node > 0 else "T_min"] - T_node) < 1e-12
        assert o["diverged"] == flagged, T_node


def test_heat_source_widens_the_temperature_bounds(oracle):
    """With a source Q''' and isothermal walls T may rise by Q Lmax^2 / (2 alpha_e) above the
    walls' range (conduction alpha_e T'' = -Q from one isothermal side)."""
    lat = small_cavity(Qv=1e-3)
    d = ref.derived(**lat.params)
    alpha = d["csT2"] * (d["tau_T"] - 0.5)
    rise = 1e-3 * 15 ** 2 / (2 * alpha)
    wt = np.array([0.6, 0.1, 0.1, 0.1, 0.1])
    for T_node, flagged in ((2 + rise - 0.05, False), (2 + rise + 0.05, True)):
        f, g = lat.get_state()
        for i, (ex, ey) in enumerate(((0, 0), (1, 0), (0, 1), (-1, 0), (0, -1))):
            g[i, 7 - ey, 7 - ex] = wt[i] * (T_node - 0.5e-3)  # Eq. (36): T = sum g + Q/2
        lat.set_state(f, g, 0)
        o = lat.observables()
        assert o["diverged"] == flagged, (T_node, rise)


def test_pressure_level_is_reported_not_judged(oracle):
    """The level of phi p is a gauge of the step (``test_oracle_gauge.py``) and drifts slowly in
    long runs, even in FP64: a node whose phi p is shifted by 0.4 (more than the rest value
    rho0 cs^2) is reported in phip_dev_max but not flagged."""
    w = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)
    lat = small_cavity()
    f, g = lat.get_state()
    # Eq. (13): a phi p shift c changes f_0 by -(1 - w0) c / cs^2 and f_i by w_i c / cs^2
    for i in range(9):
        f[i, 7 - EY[i], 7 - EX[i]] += -(1 - w[0]) * 0.4 * 3 if i == 0 else w[i] * 0.4 * 3
    lat.set_state(f, g, 0)
    o = lat.observables()
    assert abs(o["phip_dev_max"] - 0.4) < 1e-12
    assert not o["diverged"]


def test_pressure_level_drifts_in_a_long_fp64_run(oracle):
    """The drift the previous test allows for: a 150^2 clear-fluid cavity (FP64 oracle) moves
    its phi p level by more than 1e-4 between steps 10,000 and 20,000 and stays unflagged."""
    lat = ref.RefLattice(phi_uniform=1.0, **workloads.cavity(150, Ra=1e5, Pr=0.7, Da=-1.0))
    ref.set_threads(os.cpu_count() or 1)
    lat.step(10000)
    a = lat.observables()
    lat.step(10000)
    b = lat.observables()
    assert b["phip_dev_max"] - a["phip_dev_max"] > 1e-4
    assert not b["diverged"]


@pytest.mark.slow
def test_unstable_cavity_of_the_draw_is_flagged_by_step_10000(oracle):
    """Cavity 0 of the batched draw (512^2, Ra 2.92e3, Pr 7, Da 0.0118, phi 0.767, tau_v 4.83):
    the FP64 oracle's divergence flag is set by step 10,000.  (Before the |v| and bounds checks
    it was not: at step 10,000 |v|^2 had overflowed, u read 0 and T about 1e217.)"""
    c = workloads.batch64()[0]
    ref.set_threads(os.cpu_count() or 1)
    lat = ref.RefLattice(phi_uniform=c["phi"], **c["params"])
    lat.step(10000)
    o = lat.observables()
    assert o["diverged"]
