"""Two time steps per launch (temporal blocking, the default for the pull layout without a
tape) against one step per launch: bitwise equal fields and Nusselt numbers for every boundary
setting, grid shapes from the smallest allowed to ragged multi-strip ones, all precisions, odd
and even step counts (an odd count ends with one single step) and graph-replayed runs.  The
oracle parity tests run on the fused path as well, since it is the default.
"""
import pytest
import torch

from paper_1308_2071_amd import Cavity, lbm_step_shape, workloads

pytestmark = pytest.mark.gpu

FIELDS = ("ux", "uy", "p", "T")
ISO, ADIA, PER = 0, 1, 2
BCS = {
    "side_heated": dict(bc=(ISO, ISO, ADIA, ADIA), T_wall=(1.0, 0.0, 0.0, 0.0)),
    "mixed": dict(bc=(ADIA, ISO, ISO, ADIA), T_wall=(0.0, 0.2, 1.0, 0.0)),
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
    one = Cavity(dict(params, dtype=dtype, steps_per_launch=1), **kw)
    two = Cavity(dict(params, dtype=dtype, steps_per_launch=2), **kw)
    return one, two


def assert_same(a, b, what):
    oa, ob = a.observables(), b.observables()
    for k in FIELDS:
        assert torch.equal(oa[k], ob[k]), f"{what}: {k}"
    assert oa["nu_hot"] == ob["nu_hot"] and oa["nu_cold"] == ob["nu_cold"], what
    assert oa["step"] == ob["step"]
    assert torch.equal(a.stream_function(), b.stream_function()), what


@pytest.mark.parametrize("dtype", ["fp32", "fp64", "fp32_f64"])
@pytest.mark.parametrize("shape", [(5, 5), (7, 6), (64, 33), (125, 70), (300, 9)])
@pytest.mark.parametrize("bc", list(BCS))
def test_two_steps_per_launch_equal_single_steps(bc, shape, dtype):
    nx, ny = shape
    params = dict(nx=nx, ny=ny, Ra=1e5, Pr=0.71, **BCS[bc])
    phi, K = workloads.random_medium(ny, nx, seed=3 * nx + ny)
    a, b = pair(params, dtype, phi=phi, K=K)
    done = 0
    for n in (2, 3, 8, 21):
        a.step(n - done)
        b.step(n - done)
        done = n
        assert_same(a, b, f"{bc} {shape} {dtype} after {n}")
    a.close()
    b.close()


@pytest.mark.parametrize("dtype", ["fp32", "fp64"])
def test_fused_graph_replay_uniform_medium_and_heat_source(dtype):
    params = dict(nx=200, ny=150, Ra=1e5, Ra_I=1e5, Pr=0.7, Da=1e-2)
    a, b = pair(params, dtype, phi_u=0.4)
    a.step(257)            # graphs of 48 steps (24 fused launches) and an odd remainder
    b.step(257)
    assert_same(a, b, "257 steps")
    a.close()
    b.close()


@pytest.mark.parametrize("dtype", ["fp32", "fp64"])
@pytest.mark.parametrize("C", [3, 4, 7])
@pytest.mark.parametrize("shape", [(40, 30), (70, 33), (130, 21)])
def test_two_steps_between_checkpoints_keep_the_tape_exact(shape, C, dtype):
    """With a tape, two-step launches run only between checkpoints (an odd interval leaves one
    single step per segment): fields, Nusselt numbers and the gradients of J = Nu_hot equal those
    of one step per launch bitwise."""
    nx, ny = shape
    n = 23
    params = dict(nx=nx, ny=ny, Ra=1e5, Pr=0.71, dtype=dtype, checkpoint_every=C,
                  bc=(0, 0, 1, 1), T_wall=(1.0, 0.0, 0.0, 0.0))
    phi, K = workloads.random_medium(ny, nx, seed=3 * nx + ny + C)
    tdt = torch.float64 if dtype == "fp64" else torch.float32
    kw = dict(phi=torch.tensor(phi, dtype=tdt), K=torch.tensor(K, dtype=tdt), nsteps_max=n)
    a = Cavity(dict(params, steps_per_launch=1), **kw)
    b = Cavity(dict(params, steps_per_launch=2), **kw)
    assert lbm_step_shape(b.ctx)[0] == 2
    a.step(n)
    b.step(n)
    oa, ob = a.observables(), b.observables()
    for k in ("ux", "uy", "p", "T"):
        assert torch.equal(oa[k], ob[k]), k
    assert oa["nu_hot"] == ob["nu_hot"]
    for x, y in zip(a.grad(), b.grad()):
        assert torch.isfinite(x).all()
        assert torch.equal(x, y)
    a.close()
    b.close()


def test_a_tape_keeps_the_default_steps_per_launch():
    """The default form of the time loop (two steps per launch on this grid) is the same with and
    without a tape."""
    params = dict(nx=1024, ny=1024, dtype="fp32", Ra=1e5, Pr=0.71)
    phi, K = workloads.random_medium(1024, 1024, seed=5)
    kw = dict(phi=torch.tensor(phi, dtype=torch.float32), K=torch.tensor(K, dtype=torch.float32))
    plain = Cavity(params, **kw)
    taped = Cavity(dict(params, checkpoint_every=2), nsteps_max=4, **kw)
    assert lbm_step_shape(plain.ctx)[0] == 2
    assert lbm_step_shape(taped.ctx)[0] == 2
    plain.close()
    taped.close()
