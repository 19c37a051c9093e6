"""The AA-pattern layout: one population buffer stepped in place by two alternating forms of the
step.  Its results must equal the two-buffer pull layout bitwise (same per-node arithmetic), at
even and odd step counts (the two forms the state can be in), through graph replay, save/load
and the stream function, in every precision; one case is also held against the FP64 oracle.
"""
import numpy as np
import pytest
import torch

from oracle import ref
from paper_1308_2071_amd import Cavity, workloads

pytestmark = pytest.mark.gpu

FIELDS = ("ux", "uy", "p", "T")
ISO, ADIA, PER = 0, 1, 2
BCS = {
    "side_heated": dict(bc=(ISO, ISO, ADIA, ADIA), T_wall=(1.0, 0.0, 0.0, 0.0)),
    "all_iso": dict(bc=(ISO, ISO, ISO, ISO), T_wall=(1.0, 0.0, 0.7, 0.1)),
    "channel_x": dict(bc=(PER, PER, ISO, ADIA), T_wall=(0.0, 0.0, 1.0, 0.0),
                      ext_accel=(1e-5, 0.0), tau_v=0.8, tau_T=0.9, gbeta=1e-3),
    "channel_y": dict(bc=(ISO, ISO, PER, PER), T_wall=(1.0, 0.0, 0.0, 0.0),
                      ext_accel=(0.0, 2e-5), tau_T=0.9, gbeta=1e-3),
    "periodic": dict(bc=(PER, PER, PER, PER), ext_accel=(3e-5, -1e-5), T_init=0.5, tau_v=0.7,
                     tau_T=0.9, gbeta=1e-3),
}


def pair(params, dtype, phi=None, K=None, phi_u=0.6):
    tdt = torch.float64 if dtype == "fp64" else torch.float32
    kw = dict(phi=None if phi is None else torch.tensor(phi, dtype=tdt),
              K=None if K is None else torch.tensor(K, dtype=tdt), phi_uniform=phi_u)
    a = Cavity(dict(params, dtype=dtype, layout="pull"), **kw)
    b = Cavity(dict(params, dtype=dtype, layout="aa"), **kw)
    return a, b


def assert_same(a, b, what):
    oa, ob = a.observables(), b.observables()
    for k in FIELDS:
        assert torch.equal(oa[k], ob[k]), f"{what}: {k}"
    assert oa["nu_hot"] == ob["nu_hot"] and oa["nu_cold"] == ob["nu_cold"], what
    assert oa["step"] == ob["step"]


@pytest.mark.parametrize("dtype", ["fp32", "fp64", "fp32_f64"])
@pytest.mark.parametrize("shape", [(5, 5), (7, 6), (33, 20), (300, 9)])
@pytest.mark.parametrize("bc", list(BCS))
def test_aa_equals_pull_bitwise(bc, shape, dtype):
    nx, ny = shape
    params = dict(nx=nx, ny=ny, Ra=1e5, Pr=0.71, **BCS[bc])
    phi, K = workloads.random_medium(ny, nx, seed=5 * nx + ny)
    a, b = pair(params, dtype, phi=phi, K=K)
    done = 0
    for n in (1, 2, 3, 7, 20):          # odd and even step counts
        a.step(n - done)
        b.step(n - done)
        done = n
        assert_same(a, b, f"{bc} {shape} {dtype} after {n}")
    a.close()
    b.close()


@pytest.mark.parametrize("dtype", ["fp32", "fp64"])
def test_aa_graph_replay_and_uniform_medium(dtype):
    """Long runs replay a captured graph of 48 alternating launches; 131 steps = two graphs
    plus an odd remainder.  Uniform medium: no medium planes."""
    params = dict(nx=70, ny=44, Ra=1e5, Pr=1.0, Da=2e-2)
    a, b = pair(params, dtype, phi_u=0.45)
    a.step(131)
    b.step(131)
    assert_same(a, b, "131 steps")
    a.step(128)
    b.step(128)
    assert_same(a, b, "259 steps")
    a.close()
    b.close()


def test_aa_against_oracle_fp64():
    params = dict(nx=40, ny=33, Ra=1e5, Pr=0.71, Ra_I=1e5)
    phi, K = workloads.random_medium(33, 40, seed=11)
    cav = Cavity(dict(params, dtype="fp64", layout="aa"), phi=torch.tensor(phi),
                 K=torch.tensor(K))
    lat = ref.RefLattice(phi=phi, K=K, **params)
    for n in (1, 36):
        cav.step(n)
        lat.step(n)
        g = cav.observables()
        r = lat.observables(dynamic_pressure=True)
        for k in FIELDS:
            err = np.abs(g[k].cpu().numpy() - r[k]).max()
            assert err <= 1e-12, (n, k, err)
        assert abs(g["nu_hot"] - r["nu_hot"]) <= 1e-10
    cav.close()
    lat.close()


def test_aa_save_load_resume_and_stream_function():
    params = dict(nx=48, ny=41, Ra=1e5, Pr=0.71, Da=1e-2, dtype="fp32", layout="aa")
    a = Cavity(params, phi_uniform=0.6)
    b = Cavity(params, phi_uniform=0.6)
    a.step(137)                      # odd: the state is in its streamed form
    snap = a.save()
    a.step(63)
    b.load(snap)
    b.step(63)
    assert np.array_equal(a.save(), b.save())
    assert_same(a, b, "resumed")
    c = Cavity(dict(params, layout="pull"), phi_uniform=0.6)
    c.step(200)
    assert torch.equal(a.stream_function(), c.stream_function())
    for cav in (a, b, c):
        cav.close()
