"""Several time steps per launch on small grids (each tile of 16 x 16 nodes advanced four steps in
LDS with a halo of four nodes, or each tile of 8 x 8 nodes eight steps with a halo of eight)
against one step per launch: bitwise equal fields and Nusselt numbers for
every boundary setting, grid shapes from the smallest allowed to ragged ones whose last tile is
one node thick at a wall, all precisions, per-node and uniform media, step counts that are not
multiples of the steps per launch (the remainder runs as single steps) and graph-replayed runs.  With a tape the
tiles run between checkpoints, and the gradients equal those of a one-step-per-launch forward
bitwise.
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


def assert_same(a, b, what):
    oa, ob = a.observables(), b.observables()
    for k in FIELDS:
        assert torch.equal(oa[k], ob[k]), f"{what}: {k}"
    assert oa["nu_hot"] == ob["nu_hot"] and oa["nu_cold"] == ob["nu_cold"], what
    assert oa["step"] == ob["step"]
    assert torch.equal(a.stream_function(), b.stream_function()), what


SIDE = {4: 16, 8: 8}   # tile side of each form


def pair(params, dtype, phi=None, K=None, phi_u=0.6, spl=4):
    tdt = torch.float64 if dtype == "fp64" else torch.float32
    kw = dict(phi=None if phi is None else torch.tensor(phi, dtype=tdt),
              K=None if K is None else torch.tensor(K, dtype=tdt), phi_uniform=phi_u)
    one = Cavity(dict(params, dtype=dtype, steps_per_launch=1), **kw)
    tiled = Cavity(dict(params, dtype=dtype, steps_per_launch=spl), **kw)
    shape = lbm_step_shape(tiled.ctx)
    assert shape[0] == spl and shape[2] == SIDE[spl], shape
    return one, tiled


@pytest.mark.parametrize("spl", [4, 8])
@pytest.mark.parametrize("dtype", ["fp32", "fp64", "fp32_f64"])
@pytest.mark.parametrize("shape", [(5, 5), (7, 6), (17, 33), (64, 33), (49, 81), (300, 9)])
@pytest.mark.parametrize("bc", list(BCS))
def test_steps_in_lds_equal_single_steps(bc, shape, dtype, spl):
    nx, ny = shape
    params = dict(nx=nx, ny=ny, Ra=1e5, Pr=0.71, **BCS[bc])
    phi, K = workloads.random_medium(ny, nx, seed=7 * nx + ny)
    a, b = pair(params, dtype, phi=phi, K=K, spl=spl)
    done = 0
    for n in (4, 7, 16, 23):
        a.step(n - done)
        b.step(n - done)
        done = n
        assert_same(a, b, f"{bc} {shape} {dtype} after {n}")
    a.close()
    b.close()


@pytest.mark.parametrize("spl", [4, 8])
@pytest.mark.parametrize("dtype", ["fp32", "fp64", "fp32_f64"])
def test_tile_graph_replay_uniform_medium_and_heat_source(dtype, spl):
    params = dict(nx=200, ny=150, Ra=1e5, Ra_I=1e5, Pr=0.7, Da=1e-2)
    a, b = pair(params, dtype, phi_u=0.4, spl=spl)
    a.step(259)            # graphs of 48 steps (48 / spl launches); of the 19 left, 3 single
    b.step(259)
    assert_same(a, b, "259 steps")
    a.close()
    b.close()


def test_default_uses_tiles_on_the_256_workload():
    w = workloads.porous256()
    c = Cavity(dict(w["params"], dtype="fp32"), phi_uniform=w["phi"])
    assert lbm_step_shape(c.ctx)[0] == 4
    c.close()


def test_default_uses_eight_step_tiles_on_the_64_workload():
    w = workloads.porous64()
    c = Cavity(dict(w["params"], dtype="fp64"), phi_uniform=w["phi"])
    shape = lbm_step_shape(c.ctx)
    assert shape[0] == 8 and shape[2] == 8, shape
    c.close()


@pytest.mark.parametrize("spl", [4, 8])
@pytest.mark.parametrize("C", [3, 4, 6, 9])
def test_tiles_between_checkpoints_keep_the_tape_exact(C, spl):
    """With a tape, four steps per launch run only between checkpoints; the checkpoints, the
    final state and the gradient equal those of one step per launch bitwise."""
    nx, ny, n = 40, 30, 37
    params = dict(nx=nx, ny=ny, Ra=1e4, Pr=1.0, dtype="fp64", checkpoint_every=C)
    phi, K = workloads.random_medium(ny, nx, seed=11 + C)
    kw = dict(phi=torch.tensor(phi), K=torch.tensor(K), nsteps_max=n)
    a = Cavity(dict(params, steps_per_launch=1), **kw)
    b = Cavity(dict(params, steps_per_launch=spl), **kw)
    assert lbm_step_shape(b.ctx)[0] == spl
    a.step(n)
    b.step(n)
    assert_same(a, b, f"C={C}")
    ga, gb = a.grad(), b.grad()
    for x, y in zip(ga, gb):
        assert torch.equal(x, y), f"C={C}"
    a.close()
    b.close()


ADJ_BCS = ("side_heated", "mixed", "all_iso", "channel_y")


@pytest.mark.parametrize("spl", [4, 8])
@pytest.mark.parametrize("dtype", ["fp32", "fp64", "fp32_f64"])
@pytest.mark.parametrize("shape", [(5, 5), (7, 6), (21, 19), (37, 21), (19, 37), (64, 33)])
@pytest.mark.parametrize("bc", ADJ_BCS)
def test_gradients_equal_with_and_without_forward_tiles(bc, shape, dtype, spl):
    """Gradients of J = Nu_hot after a forward pass in LDS tiles (between checkpoints) against
    one step per launch: the tape's states, and so the gradients, are bitwise equal.  Segments of
    7 steps leave remainders that go one step at a time; the shapes include ragged last tiles."""
    nx, ny = shape
    n, C = 23, 7
    params = dict(nx=nx, ny=ny, Ra=1e5, Pr=0.71, checkpoint_every=C, **BCS[bc])
    phi, K = workloads.random_medium(ny, nx, seed=5 * nx + ny)
    tdt = torch.float64 if dtype == "fp64" else torch.float32
    kw = dict(phi=torch.tensor(phi, dtype=tdt), K=torch.tensor(K, dtype=tdt), nsteps_max=n)
    a = Cavity(dict(params, dtype=dtype, steps_per_launch=1), **kw)
    b = Cavity(dict(params, dtype=dtype, steps_per_launch=spl), **kw)
    a.step(n)
    b.step(n)
    assert_same(a, b, f"{bc} {shape} {dtype}")
    ga, gb = a.grad(), b.grad()
    for x, y in zip(ga, gb):
        assert torch.isfinite(x).all()
        assert torch.equal(x, y), f"{bc} {shape} {dtype}"
    a.close()
    b.close()


@pytest.mark.parametrize("dtype", ["fp32", "fp64"])
def test_gradients_with_forward_tiles_uniform_medium_and_heat_source(dtype):
    params = dict(nx=45, ny=38, Ra=1e5, Ra_I=1e5, Pr=0.7, Da=1e-2, checkpoint_every=10)
    a = Cavity(dict(params, dtype=dtype, steps_per_launch=1), phi_uniform=0.4, nsteps_max=30)
    b = Cavity(dict(params, dtype=dtype, steps_per_launch=4), phi_uniform=0.4, nsteps_max=30)
    a.step(30)
    b.step(30)
    for x, y in zip(a.grad(), b.grad()):
        assert torch.isfinite(x).all() and x.abs().max() > 0
        assert torch.equal(x, y), dtype
    a.close()
    b.close()
