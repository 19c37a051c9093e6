"""The seeded input recipes (the paper's cavity set-up, Sec. 4.1, with the synthetic porous
media): distributions, the Kozeny-Carman scaling of Eq. (5), and determinism.  No GPU."""
import numpy as np

from paper_1308_2071_amd import workloads

HOT_COLD_ADIABATIC = dict(bc=(0, 0, 1, 1), T_wall=(1.0, 0.0, 0.0, 0.0), T_init=0.5)


def check_cavity(p, n):
    assert p["nx"] == p["ny"] == n
    for k, v in HOT_COLD_ADIABATIC.items():
        assert tuple(p[k]) == tuple(v) if isinstance(v, tuple) else p[k] == v


def test_uniform_cavities():
    a, b = workloads.porous64(), workloads.porous256()
    check_cavity(a["params"], 64)
    check_cavity(b["params"], 256)
    assert (a["phi"], a["params"]["Da"], a["params"]["Ra"], a["params"]["Pr"], a["steps"]) == \
        (0.6, 1e-2, 1e3, 1.0, 20000)
    assert (b["phi"], b["params"]["Da"], b["params"]["Ra"], b["params"]["Pr"], b["steps"]) == \
        (0.4, 1e-2, 1e5, 1.0, 50000)


def test_roofline_medium():
    n = 256                                     # the same recipe as 4096^2, smaller
    w = workloads.roofline4096(n)
    check_cavity(w["params"], n)
    phi, K = w["phi"], w["K"]
    assert phi.min() >= 0.3 and phi.max() < 0.9 and abs(phi.mean() - 0.6) < 0.01
    # Eq. (5): K = phi^3 d_p^2 / (150 (1 - phi)^2), one d_p for the field, mean Da = 1e-3
    dp2 = K * 150.0 * (1.0 - phi) ** 2 / phi ** 3
    assert np.allclose(dp2, dp2.flat[0], rtol=1e-12)
    assert abs(K.mean() / (1e-3 * (n - 1) ** 2) - 1.0) < 1e-12
    assert (w["params"]["Ra"], w["params"]["Pr"], w["steps"]) == (1e6, 0.71, 2000)
    w2 = workloads.roofline4096(n)
    assert np.array_equal(w2["phi"], phi) and np.array_equal(w2["K"], K)


def test_batch_of_64_uneven_cavities():
    cav = workloads.batch64()
    assert len(cav) == 64
    sides = set()
    for c in cav:
        p = c["params"]
        sides.add(p["nx"])
        assert p["nx"] in (64, 96, 128, 192, 256, 384, 512)
        check_cavity(p, p["nx"])
        assert 1e3 <= p["Ra"] <= 1e6 and 1e-4 <= p["Da"] <= 1e-1
        assert 0.2 <= c["phi"] <= 0.9 and p["Pr"] in (0.71, 1.0, 7.0)
    assert len(sides) == 7                      # every side length drawn
    assert [c["params"] for c in workloads.batch64()] == [c["params"] for c in cav]


def test_adjoint_medium_and_probes():
    w = workloads.adjoint256()
    n = 256
    check_cavity(w["params"], n)
    phi, K = w["phi"], w["K"]
    assert phi.min() >= 0.2 and phi.max() <= 0.9
    assert abs(phi.mean() - 0.5) < 0.01 and abs(phi.std() - 0.1) < 0.01
    # smoothed: neighbouring nodes are strongly correlated (unlike the i.i.d. roofline field)
    assert np.corrcoef(phi[:, :-1].ravel(), phi[:, 1:].ravel())[0, 1] > 0.9
    assert abs(K.mean() / (1e-2 * (n - 1) ** 2) - 1.0) < 1e-12
    assert (w["steps"], w["checkpoint"]) == (2000, 100)
    probes = w["probes"]
    assert len(probes) == 16 and len(set(probes)) == 16
    assert all(1 <= x <= 8 for _, x in probes[:8])          # the hot-wall layer
    assert all(1 <= y <= n - 2 and 1 <= x <= n - 2 for y, x in probes)
