"""The pressure level is a gauge of the scheme (the reading behind the FP32 pressure checks).

A uniform shift c of the product phi p at every node, made through the populations as Eq. (13)
makes it (f_0 by -(1 - w0) c / cs^2, f_i by w_i c / cs^2 for i >= 1, cs^2 = 1/3), leaves the
step's velocity and temperature unchanged and keeps phi p shifted by exactly c, at every node and
every later step: the shift moves M f by (0, 6c, -9c, 0, ...), which is exactly how Eq. (16)
moves m_eq, so m - m_eq, the collision, Eq. (21) and Eq. (36) do not see it; Eq. (23) returns
phi p + c; and the wall rule phi_b p_b = phi_f p_f carries the shift to the walls.  With a
per-node porosity, p itself then shifts by c / phi(x), not by a constant.
"""
import numpy as np
import pytest

from oracle import ref
from paper_1308_2071_amd import workloads

W9 = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)


def shift(c):
    d = W9 * 3.0 * c
    d[0] = -(1 - W9[0]) * 3.0 * c
    return d[:, None, None]


@pytest.fixture(autouse=True)
def one_oracle_thread():
    threads = ref.get_threads()
    ref.set_threads(1)
    yield
    ref.set_threads(threads)


def run_pair(c, pre_steps, steps, **kw):
    nx, ny = 14, 11
    phi, K = workloads.random_medium(ny, nx, seed=21)
    params = dict(workloads.cavity(nx, ny, Ra=3e4, Pr=0.71), **kw)
    a = ref.RefLattice(phi=phi, K=K, **params)
    b = ref.RefLattice(phi=phi, K=K, **params)
    a.step(pre_steps)
    f, g = a.get_state()
    b.set_state(f + shift(c), g, pre_steps)
    a.step(steps)
    b.step(steps)
    return phi, a.observables(), b.observables()


@pytest.mark.parametrize("pre_steps", [0, 150])
@pytest.mark.parametrize("c", [0.05, -0.02])
def test_uniform_phi_p_shift_is_a_gauge(oracle, pre_steps, c):
    """From rest (pre_steps = 0) and from a developed state, 300 steps later."""
    phi, oa, ob = run_pair(c, pre_steps, 300)
    for k in ("ux", "uy", "T"):
        assert np.abs(ob[k] - oa[k]).max() <= 1e-14, k
    assert abs(ob["nu_hot"] - oa["nu_hot"]) <= 1e-12
    # phi p moves by c at every node, so p by c / phi(x)
    np.testing.assert_allclose(phi * ob["p"] - phi * oa["p"], c, rtol=0, atol=1e-14)
    dp = ob["p"] - oa["p"]
    assert np.ptp(dp) > 0.1 * abs(c)   # not a constant shift of p with per-node phi


def test_gauge_holds_with_a_heat_source(oracle):
    phi, oa, ob = run_pair(0.03, 100, 200, Qv=2e-4)
    for k in ("ux", "uy", "T"):
        assert np.abs(ob[k] - oa[k]).max() <= 1e-14, k
    np.testing.assert_allclose(phi * (ob["p"] - oa["p"]), 0.03, rtol=0, atol=1e-14)
