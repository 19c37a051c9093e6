"""Three time steps per launch (FP32 storage and arithmetic: step n+1 in registers, step n+2 in
a ring of rows in LDS) against one step per launch: bitwise equal fields and Nusselt numbers for
every boundary setting, grid shapes from the smallest allowed to ragged multi-strip ones (strips
of 60 columns; segments whose last one takes the rows left over), step counts that are not
multiples of three (the remainder runs as single steps), graph-replayed runs and a tape.
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


def pair(params, phi=None, K=None, phi_u=0.6, **extra):
    kw = dict(phi=None if phi is None else torch.tensor(phi, dtype=torch.float32),
              K=None if K is None else torch.tensor(K, dtype=torch.float32), phi_uniform=phi_u,
              **extra)
    one = Cavity(dict(params, dtype="fp32", steps_per_launch=1), **kw)
    three = Cavity(dict(params, dtype="fp32", steps_per_launch=3), **kw)
    assert lbm_step_shape(three.ctx)[0] == 3
    return one, three


def assert_same(a, b, what):
    oa, ob = a.observables(), b.observables()
    for k in FIELDS:
        assert torch.equal(oa[k], ob[k]), f"{what}: {k}"
    assert oa["nu_hot"] == ob["nu_hot"] and oa["nu_cold"] == ob["nu_cold"], what
    assert oa["step"] == ob["step"]


@pytest.mark.parametrize("shape", [(5, 5), (7, 6), (6, 9), (64, 33), (125, 70), (300, 9),
                                   (61, 12), (121, 13)])
@pytest.mark.parametrize("bc", list(BCS))
def test_three_steps_per_launch_equal_single_steps(bc, shape):
    nx, ny = shape
    params = dict(nx=nx, ny=ny, Ra=1e5, Pr=0.71, **BCS[bc])
    phi, K = workloads.random_medium(ny, nx, seed=5 * nx + ny)
    a, b = pair(params, phi=phi, K=K)
    done = 0
    for n in (3, 4, 9, 23):
        a.step(n - done)
        b.step(n - done)
        done = n
        assert_same(a, b, f"{bc} {shape} after {n}")
    a.close()
    b.close()


@pytest.mark.parametrize("bc,shape", [("periodic", (2, 2)), ("periodic", (3, 2)),
                                      ("periodic", (2, 3)), ("periodic", (4, 7)),
                                      ("channel_x", (2, 5)), ("channel_x", (3, 6)),
                                      ("channel_y", (5, 2)), ("channel_y", (6, 3))])
def test_three_steps_on_the_narrowest_periodic_axes(bc, shape):
    """A periodic axis of two or three nodes: the halo columns (lanes beyond the grid) and the
    halo rows of the intermediate steps wrap onto the same few nodes."""
    nx, ny = shape
    params = dict(nx=nx, ny=ny, Ra=1e5, Pr=0.71, **BCS[bc])
    phi, K = workloads.random_medium(ny, nx, seed=7 * nx + ny)
    a, b = pair(params, phi=phi, K=K)
    done = 0
    for n in (3, 7, 30):
        a.step(n - done)
        b.step(n - done)
        done = n
        assert_same(a, b, f"{bc} {shape} after {n}")
    a.close()
    b.close()


def test_three_steps_graph_replay_uniform_medium_and_heat_source():
    params = dict(nx=200, ny=150, Ra=1e5, Ra_I=1e5, Pr=0.7, Da=1e-2)
    a, b = pair(params, phi_u=0.4)
    a.step(257)            # graphs of 48 steps (16 launches) and a remainder
    b.step(257)
    assert_same(a, b, "257 steps")
    a.close()
    b.close()


@pytest.mark.parametrize("C", [3, 4, 7])
def test_three_steps_between_checkpoints_keep_the_tape_exact(C):
    nx, ny, n = 70, 33, 23
    params = dict(nx=nx, ny=ny, Ra=1e5, Pr=0.71, checkpoint_every=C)
    phi, K = workloads.random_medium(ny, nx, seed=C)
    a, b = pair(params, phi=phi, K=K, nsteps_max=n)
    a.step(n)
    b.step(n)
    assert_same(a, b, f"C={C}")
    for x, y in zip(a.grad(), b.grad()):
        assert torch.equal(x, y)
    a.close()
    b.close()


def test_roofline4096_three_steps_equal_single_steps():
    w = workloads.roofline4096()
    phi = torch.from_numpy(w["phi"].astype("float32"))
    K = torch.from_numpy(w["K"].astype("float32"))
    a = Cavity(dict(w["params"], dtype="fp32", steps_per_launch=1), phi=phi, K=K)
    b = Cavity(dict(w["params"], dtype="fp32", steps_per_launch=3), phi=phi, K=K)
    for n in (99, 1):
        a.step(n)
        b.step(n)
        assert_same(a, b, f"after {n} more")
    a.close()
    b.close()


@pytest.mark.parametrize("n,dtype,spl", [(4096, "fp32", 3), (3072, "fp32", 3), (2048, "fp32", 3),
                                         (1536, "fp32", 2), (1024, "fp32", 2),
                                         (4096, "fp64", 2), (4096, "fp32_f64", 2)])
def test_default_form_by_grid(n, dtype, spl):
    """The default time loop takes three steps per launch in FP32 where segments of 8 rows give
    three rounds of the resident set (2048^2 and up on this device), else two on these grids;
    FP64 arithmetic never takes three."""
    tdt = torch.float64 if dtype == "fp64" else torch.float32
    c = Cavity(dict(nx=n, ny=n, Ra=1e6, Pr=0.71, dtype=dtype), phi=torch.full((n, n), 0.6, dtype=tdt),
               K=torch.full((n, n), 1.0, dtype=tdt))
    shape = lbm_step_shape(c.ctx)
    c.close()
    assert shape[0] == spl, shape
