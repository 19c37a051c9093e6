"""Parity of the HIP time step with the FP64 CPU oracle, element by element on the same seeded
inputs: u_x, u_y, p, T at every node and the two wall Nusselt numbers (Eq. (38)).

Tolerances: FP64 max-abs 1e-12 after short runs on tiny grids and 1e-10 after the 20k steps of
the 64 x 64 cavity; FP32 1e-4 of each field's range (range = max - min of the oracle's field)
and Nu within 1e-3; FP32 storage with FP64 arithmetic ("fp32_f64") 1e-5 and 1e-4.  p is the
pressure of Eq. (23) less its rest value rho0 cs^2 / phi, as the library reports it (the
oracle's p is converted in FP64).  FP32 compares p up to a constant: the density is fixed at
rho0, only pressure differences enter the momentum equation and nothing pins the level of phi p,
which rounding moves (a uniform phi p shift is exact gauge of the step, pinned by
``test_oracle_gauge.py``; with per-node phi it moves p by c / phi(x)).  In the first steps a
field's range can be far below its
magnitude; there the range is floored at 1e-2 of the field's magnitude, so the bar never drops
below ~15 FP32 ulps of the value.  For FP32-storage runs the oracle receives the FP32-rounded
phi and K, so only the arithmetic and the storage differ.
"""
import numpy as np
import pytest
import torch

from oracle import ref
from paper_1308_2071_amd import Cavity, workloads
from pressure_gauge import phip_gauged

pytestmark = pytest.mark.gpu

FIELDS = ("ux", "uy", "p", "T")
FP32_STORAGE = ("fp32", "fp32_f64")
# FP32 storage: field tolerance as a fraction of the range, and Nu; FP64 arithmetic on FP32
# storage ("fp32_f64") rounds each stored value once per step and is held to a 10x tighter bar
RTOL = {"fp32": (1e-4, 1e-3), "fp32_f64": (1e-5, 1e-4)}


def run_pair(params, steps, phi=None, K=None, phi_u=0.6, dtype="fp64", chunks=None):
    """Run the same cavity on the GPU and in the oracle; yields (gpu_obs, ref_obs) at each
    chunk boundary."""
    if dtype in FP32_STORAGE:
        phi = None if phi is None else phi.astype(np.float32).astype(np.float64)
        K = None if K is None else K.astype(np.float32).astype(np.float64)
        phi_u = float(np.float32(phi_u))
    tdt = torch.float64
    cav = Cavity(dict(params, dtype=dtype),
                 phi=None if phi is None else torch.tensor(phi, dtype=tdt),
                 K=None if K is None else torch.tensor(K, dtype=tdt), phi_uniform=phi_u)
    lat = ref.RefLattice(phi=phi, K=K, phi_uniform=phi_u, **params)
    chunks = chunks or [steps]
    for n in chunks:
        cav.step(n)
        lat.step(n)
        g = cav.observables()
        r = lat.observables(dynamic_pressure=True)
        r["phi"] = phi if phi is not None else phi_u
        yield {k: (g[k].double().cpu().numpy() if k in FIELDS else g[k]) for k in g}, r
    cav.close()


def assert_match(g, r, dtype, atol64=1e-12, what="", floor=1e-2):
    for k in FIELDS:
        a, b = g[k], r[k]
        if dtype == "fp64":
            err = np.abs(a - b).max()
            assert err <= atol64, f"{what} {k}: max-abs {err:.3e} > {atol64:.1e}"
        else:
            rng = max(b.max() - b.min(), floor * np.abs(b).max(), 1e-12)
            d = a - b
            if k == "p":
                # the level of phi p is free: FP32 is compared up to a uniform phi p shift
                d = phip_gauged(d, r["phi"])
            err = np.abs(d).max() / rng
            assert err <= RTOL[dtype][0], f"{what} {k}: {err:.3e} of range"
    tol = atol64 * 100 if dtype == "fp64" else RTOL[dtype][1]
    assert abs(g["nu_hot"] - r["nu_hot"]) <= tol, (what, g["nu_hot"], r["nu_hot"])
    assert abs(g["nu_cold"] - r["nu_cold"]) <= tol, (what, g["nu_cold"], r["nu_cold"])
    assert not g["diverged"]


ISO, ADIA, PER = 0, 1, 2
BC_CASES = {
    "side_heated": dict(bc=(ISO, ISO, ADIA, ADIA), T_wall=(1.0, 0.0, 0.0, 0.0)),
    "mixed": dict(bc=(ADIA, ISO, ISO, ADIA), T_wall=(0.0, 0.2, 1.0, 0.0)),
    "all_iso": dict(bc=(ISO, ISO, ISO, ISO), T_wall=(1.0, 0.0, 0.7, 0.1)),
    "all_adia": dict(bc=(ADIA, ADIA, ADIA, ADIA), T_wall=(0.0, 0.0, 0.0, 0.0), T_init=0.3),
    "channel_x": dict(bc=(PER, PER, ISO, ADIA), T_wall=(0.0, 0.0, 1.0, 0.0),
                      ext_accel=(1e-5, 0.0)),
    "channel_y": dict(bc=(ISO, ISO, PER, PER), T_wall=(1.0, 0.0, 0.0, 0.0),
                      ext_accel=(0.0, 2e-5)),
    "periodic": dict(bc=(PER, PER, PER, PER), ext_accel=(3e-5, -1e-5), T_init=0.5),
}


@pytest.mark.parametrize("dtype", ["fp64", "fp32", "fp32_f64"])
@pytest.mark.parametrize("shape", [(5, 5), (7, 6), (16, 16), (300, 70)])
@pytest.mark.parametrize("bcname", list(BC_CASES))
def test_tiny_grids_step_by_step(shape, bcname, dtype):
    nx, ny = shape
    params = dict(nx=nx, ny=ny, Ra=1e5, Pr=0.71, **BC_CASES[bcname])
    if bcname in ("channel_x", "periodic"):
        params["tau_v"] = 0.8 if bcname == "channel_x" else 0.7
    if bcname.startswith("channel") or bcname == "periodic":
        params["tau_T"] = 0.9
        params["gbeta"] = 1e-3
    phi, K = workloads.random_medium(ny, nx, seed=nx * 1000 + ny)
    for i, (g, r) in enumerate(run_pair(params, 0, phi=phi, K=K, dtype=dtype,
                                        chunks=[1, 1, 3, 20, 75])):
        assert_match(g, r, dtype, what=f"{bcname} {shape} chunk {i}")


@pytest.mark.parametrize("dtype", ["fp64", "fp32", "fp32_f64"])
@pytest.mark.parametrize("forch", [0, 1])
def test_uniform_medium_and_forchheimer_flag(dtype, forch):
    params = dict(nx=33, ny=29, Ra=1e4, Pr=1.0, Da=3e-3, forchheimer=forch)
    for g, r in run_pair(params, 0, phi_u=0.45, dtype=dtype, chunks=[1, 49, 150]):
        assert_match(g, r, dtype, what=f"uniform forch={forch}")


def test_infinite_permeability():
    params = dict(nx=24, ny=24, Ra=1e4, Pr=0.71, Da=-1.0)   # K = infinity: no drag
    for g, r in run_pair(params, 0, phi_u=0.9999, dtype="fp64", chunks=[10, 90]):
        assert_match(g, r, "fp64", what="K=inf")


def test_porous64_full_run_fp64():
    """The 64 x 64 porous cavity (phi = 0.6, Da = 1e-2, Ra = 1e3, Pr = 1), all 20k steps."""
    w = workloads.porous64()
    for g, r in run_pair(w["params"], 0, phi_u=w["phi"], dtype="fp64",
                         chunks=[1000, 19000]):
        assert_match(g, r, "fp64", atol64=1e-10, what="porous64")
    assert abs(r["nu_hot"] - 1.012) < 0.01  # Table 2, phi = 0.6, Ra = 1e3 (context)


def test_graph_replay_equals_eager_launches():
    """lbm_step replays a captured HIP graph for long runs; the result must be bitwise the
    same as the same number of single launches."""
    params = dict(nx=70, ny=40, Ra=1e5, Pr=0.71)
    phi, K = workloads.random_medium(40, 70, seed=3)
    a = Cavity(dict(params, dtype="fp32"), phi=torch.tensor(phi), K=torch.tensor(K))
    b = Cavity(dict(params, dtype="fp32"), phi=torch.tensor(phi), K=torch.tensor(K))
    a.step(300)           # graph chunks + remainder
    for _ in range(300):  # one launch per call
        b.step(1)
    sa, sb = a.save(), b.save()
    assert np.array_equal(sa, sb)


def test_save_load_resume_is_bitwise():
    params = dict(nx=50, ny=45, Ra=1e5, Pr=1.0, dtype="fp64")
    a = Cavity(params, phi_uniform=0.5)
    b = Cavity(params, phi_uniform=0.5)
    a.step(137)
    snap = a.save()
    a.step(63)
    b.load(snap)
    b.step(63)
    assert b.observables(False)["step"] == 200
    assert np.array_equal(a.save(), b.save())


@pytest.mark.parametrize("spl", [1, 2])
def test_zero_steps_is_a_no_op_and_negative_steps_are_rejected(spl):
    params = dict(nx=33, ny=20, Ra=1e5, Pr=0.71, dtype="fp32", steps_per_launch=spl)
    cav = Cavity(params, phi_uniform=0.6)
    cav.step(5)
    before = cav.observables()
    snap = cav.save()
    cav.step(0)
    after = cav.observables()
    assert after["step"] == 5 and np.array_equal(cav.save(), snap)
    for k in FIELDS:
        assert torch.equal(before[k], after[k]), k
    with pytest.raises(RuntimeError, match="LBM_E_INVAL"):
        cav.step(-1)
    assert cav.observables(False)["step"] == 5
    cav.close()


def test_divergence_is_reported():
    """A non-finite value in the state (here planted through lbm_load, the way a corrupted
    checkpoint would arrive) spreads within a few steps; the library reports LBM_E_DIVERGED
    with the flag set instead of returning garbage silently."""
    params = dict(nx=16, ny=16, Ra=1e5, Pr=1.0, dtype="fp32")
    cav = Cavity(params, phi_uniform=0.5)
    cav.step(10)
    assert not cav.observables(False)["diverged"]
    snap = cav.save()
    pitch = int(snap[:64].view(np.int64)[4])
    off = 64 + (5 * pitch + 5) * 4          # plane f0, node (5, 5), after the 64-byte header
    snap[off:off + 4] = np.frombuffer(np.float32(np.nan).tobytes(), dtype=np.uint8)
    cav.load(snap)
    cav.step(3)
    o = cav.observables(fields=False)
    assert o["diverged"] and o["status"] == -4


def test_overflowing_velocity_is_reported():
    """|v|^2 overflowing (FP64) makes Eq. (21)'s denominator infinite and u = 0 while T and p
    stay finite; the |v| check reports it (LBM_DIV_NONFINITE).  The state is planted through
    lbm_load: f'_1 at (8, 8) and f'_3 at (10, 8) of +-1e200 both stream into (9, 8)."""
    params = dict(nx=16, ny=16, Ra=1e4, Pr=0.71, Da=1e-2, dtype="fp64")
    cav = Cavity(params, phi_uniform=0.6)
    snap = cav.save()
    hdr = snap[:64].view(np.int64)          # {magic, dtype, nx, ny, pitch, step, layout, stride}
    pitch, plane = int(hdr[4]), int(hdr[7])
    st = snap[64:].view(np.float64)
    st[1 * plane + 8 * pitch + 8] = 1e200
    st[3 * plane + 8 * pitch + 10] = -1e200
    cav.load(snap)
    o = cav.observables(fields=False)
    assert o["status"] == -4 and o["diverged"]
    assert o["why"] & 1 and o["max_speed"] < 0.1 and np.isfinite(o["T_max"])
    cav.close()


def test_unstable_cavity_is_reported_in_fp64():
    """Cavity 0 of the batched draw (512^2, tau_v 4.83, beyond the step's linear stability
    limit of about 4.6455): the FP64 library reports LBM_E_DIVERGED by step 10,000, as the FP64
    oracle does (before the |v| and bounds checks both returned OK on u = 0 and T ~ 1e217)."""
    c = workloads.batch64()[0]
    cav = Cavity(dict(c["params"], dtype="fp64"), phi_uniform=c["phi"])
    cav.step(10000)
    o = cav.observables(fields=False)
    assert o["diverged"] and o["status"] == -4, o
    cav.close()


HEAT_CASES = {
    # Sec. 4.3: side heating plus internal heating
    "side_and_internal": dict(nx=40, ny=33, Ra=1e5, Ra_I=1e5, Pr=0.7, Da=1e-2),
    # Sec. 4.2: all walls cold, internal heating only, Brinkman-extended Darcy (phi = 1, F = 0)
    "internal_only": dict(nx=37, ny=30, Ra=0.0, Ra_I=6.4e5, Pr=7.0, Da=1e-2, forchheimer=0,
                          bc=(ISO, ISO, ISO, ISO), T_wall=(0.0, 0.0, 0.0, 0.0), T_init=0.0),
    # a source given directly, adiabatic sides
    "direct_source": dict(nx=30, ny=26, Ra=1e4, Pr=1.0, Qv=2e-5, sigma=1.3,
                          bc=(ISO, ADIA, ADIA, ISO), T_wall=(1.0, 0.0, 0.0, 0.2)),
}


@pytest.mark.parametrize("dtype", ["fp64", "fp32", "fp32_f64"])
@pytest.mark.parametrize("name", list(HEAT_CASES))
def test_heat_source_step_by_step(name, dtype):
    """Eqs. (30), (33), (34), (36): the heat-source term against the oracle."""
    params = HEAT_CASES[name]
    ny, nx = params["ny"], params["nx"]
    if name == "internal_only":
        runs = run_pair(params, 0, phi_u=1.0, dtype=dtype, chunks=[1, 9, 90, 300])
    else:
        phi, K = workloads.random_medium(ny, nx, seed=nx + 7 * ny)
        runs = run_pair(params, 0, phi=phi, K=K, dtype=dtype, chunks=[1, 9, 90, 300])
    for i, (g, r) in enumerate(runs):
        assert_match(g, r, dtype, what=f"{name} chunk {i}")


def test_stream_function_integrates_the_oracle_velocity():
    """psi with u_x = d psi / dy, trapezoid along y from psi = 0 on the south side, against the
    same integral of the oracle's u_x (and u_y = -d psi / dx to second order in the interior)."""
    params = dict(nx=48, ny=41, Ra=1e5, Pr=0.71, Da=1e-2)
    cav = Cavity(dict(params, dtype="fp64"), phi_uniform=0.6)
    lat = ref.RefLattice(phi_uniform=0.6, **params)
    cav.step(400)
    lat.step(400)
    psi = cav.stream_function().cpu().numpy()
    ux = lat.observables()["ux"]
    want = np.zeros_like(ux)
    want[1:] = np.cumsum(0.5 * (ux[1:] + ux[:-1]), axis=0)
    assert np.abs(psi - want).max() <= 1e-12
    assert np.abs(psi).max() > 1e-3
