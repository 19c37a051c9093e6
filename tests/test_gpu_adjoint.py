"""Parity of the HIP discrete adjoint (lbm_grad) with the oracle adjoint: the exact gradient of
J = Nu_hot after N steps (Eq. (38)) with respect to the per-node porosity phi and permeability
K, obtained by reverse-mode differentiation of the plain FP64 CPU step (``oracle/torch_ref``),
compared at every node.

Tolerances: FP64 max-abs <= 1e-9 of max |dJ/d.| over the field (dJ/dK is ~1e-4 of dJ/dphi in
these cavities, so its rounding floor relative to its own maximum sits near 1e-10); FP32 <= 1e-3
of it (both gradients of the same discrete map; FP32 carries the forward's rounding into the
backward); FP32 storage with FP64 arithmetic <= 1e-4.
"""
import numpy as np
import pytest
import torch

from oracle import torch_ref
from paper_1308_2071_amd import Cavity, NuHot, workloads

pytestmark = pytest.mark.gpu

ISO, ADIA, PER = 0, 1, 2


def gpu_grad(params, phi, K, steps, C, dtype, uniform=False, phi_u=0.6):
    p = dict(params, dtype=dtype, checkpoint_every=C)
    if uniform:
        cav = Cavity(p, phi_uniform=phi_u, nsteps_max=steps)
    else:
        cav = Cavity(p, phi=torch.tensor(phi), K=torch.tensor(K), nsteps_max=steps)
    cav.step(steps)
    J = cav.observables(fields=False)["nu_hot"]
    gphi, gK = cav.grad(1.0)
    cav.close()
    return J, gphi.cpu().numpy(), gK.cpu().numpy()


def check(gpu, ref, tol, what):
    scale = np.abs(ref).max()
    assert scale > 0, what
    err = np.abs(gpu - ref).max() / scale
    assert err <= tol, f"{what}: {err:.3e} of max |grad| > {tol:.0e}"


CASES = {
    "side_heated": (dict(bc=(ISO, ISO, ADIA, ADIA), T_wall=(1.0, 0.0, 0.0, 0.0)), (12, 12)),
    "mixed": (dict(bc=(ISO, ADIA, ADIA, ISO), T_wall=(1.0, 0.0, 0.0, 0.3)), (11, 9)),
    "all_iso": (dict(bc=(ISO, ISO, ISO, ISO), T_wall=(1.0, 0.0, 0.6, 0.2)), (10, 13)),
    "channel": (dict(bc=(ISO, ISO, PER, PER), T_wall=(1.0, 0.0, 0.0, 0.0),
                     ext_accel=(0.0, 1e-4)), (9, 8)),
    "ragged": (dict(bc=(ISO, ISO, ADIA, ADIA), T_wall=(1.0, 0.0, 0.0, 0.0)), (300, 7)),
    # 65 columns and 9 rows: the backward kernel's last tile along each walled axis would be one
    # node wide, so it starts one node earlier to keep the wall nodes with their neighbours
    "shifted_tiles": (dict(bc=(ISO, ADIA, ISO, ADIA), T_wall=(1.0, 0.0, 0.5, 0.0)), (65, 9)),
}


@pytest.mark.parametrize("dtype", ["fp64", "fp32", "fp32_f64"])
@pytest.mark.parametrize("name", list(CASES))
def test_adjoint_matches_oracle(name, dtype):
    extra, (nx, ny) = CASES[name]
    steps, C = (40, 7) if nx < 100 else (12, 5)
    params = dict(nx=nx, ny=ny, Ra=1e5, Pr=0.71, **extra)
    phi, K = workloads.random_medium(ny, nx, seed=31 + nx + ny, K_lo=2.0, K_hi=20.0)
    if dtype != "fp64":
        phi = phi.astype(np.float32).astype(np.float64)
        K = K.astype(np.float32).astype(np.float64)
    J, gphi, gK = gpu_grad(params, phi, K, steps, C, dtype)
    Jr, rphi, rK = torch_ref.grad_nu_hot(phi, K, steps, **params)
    tol = {"fp64": 1e-9, "fp32": 1e-3, "fp32_f64": 1e-4}[dtype]
    Jtol = {"fp64": 1e-11, "fp32": 1e-4, "fp32_f64": 1e-5}[dtype]
    assert abs(J - Jr) <= Jtol * max(1.0, abs(Jr))
    check(gphi, rphi, tol, f"{name} dJ/dphi")
    check(gK, rK, tol, f"{name} dJ/dK")


@pytest.mark.parametrize("forch", [0, 1])
def test_adjoint_uniform_medium(forch):
    """No medium planes: the gradient is still per node (each node's phi and K)."""
    nx, ny, steps = 11, 10, 30
    params = dict(nx=nx, ny=ny, Ra=1e5, Pr=1.0, Da=2e-2, forchheimer=forch)
    J, gphi, gK = gpu_grad(params, None, None, steps, 8, "fp64", uniform=True, phi_u=0.45)
    K = 2e-2 * (nx - 1) ** 2
    Jr, rphi, rK = torch_ref.grad_nu_hot(np.full((ny, nx), 0.45), np.full((ny, nx), K), steps,
                                         **params)
    check(gphi, rphi, 1e-10, "uniform dJ/dphi")
    check(gK, rK, 1e-10, "uniform dJ/dK")


def test_grad_without_tape_is_a_state_error():
    cav = Cavity(dict(nx=8, ny=8, dtype="fp64"), phi_uniform=0.5)
    cav.step(3)
    with pytest.raises(RuntimeError, match="LBM_E_STATE"):
        cav.grad()


def test_tape_length_is_enforced():
    cav = Cavity(dict(nx=8, ny=8, dtype="fp32", checkpoint_every=4), phi_uniform=0.5,
                 nsteps_max=8)
    cav.step(8)
    with pytest.raises(RuntimeError, match="LBM_E_STATE"):
        cav.step(1)


def test_grad_leaves_forward_state_unchanged():
    params = dict(nx=14, ny=12, Ra=1e5, Pr=0.71, dtype="fp64", checkpoint_every=5)
    phi, K = workloads.random_medium(12, 14, seed=2)
    cav = Cavity(params, phi=torch.tensor(phi), K=torch.tensor(K), nsteps_max=40)
    cav.step(23)
    before = cav.observables()
    g1 = cav.grad()
    after = cav.observables()
    for k in ("ux", "uy", "p", "T"):
        assert torch.equal(before[k], after[k])
    g2 = cav.grad()        # repeatable
    assert torch.equal(g1[0], g2[0]) and torch.equal(g1[1], g2[1])


def test_nuhot_autograd_function_gradcheck():
    """NuHot's backward is the HIP adjoint; torch.autograd.gradcheck compares it with finite
    differences of its own forward (FP64, tiny grid)."""
    nx, ny = 8, 7
    params = dict(nx=nx, ny=ny, Ra=1e5, Pr=0.71, dtype="fp64")
    phi, K = workloads.random_medium(ny, nx, seed=5)
    tphi = torch.tensor(phi, device="cuda", requires_grad=True)
    tK = torch.tensor(K, device="cuda", requires_grad=True)
    f = lambda a, b: NuHot.apply(a, b, params, 15, 4)
    assert torch.autograd.gradcheck(f, (tphi, tK), eps=1e-6, atol=1e-8, rtol=1e-5)


def test_nuhot_chains_through_kozeny_carman():
    """The total derivative with respect to porosity when K = K(phi) (Eq. (5)) comes from torch's
    chain rule through the Kozeny-Carman map, on top of lbm_grad's partial derivatives."""
    nx, ny, steps = 10, 9, 20
    params = dict(nx=nx, ny=ny, Ra=1e5, Pr=1.0, dtype="fp64")
    eps = torch.tensor(workloads.smoothed_porosity(10, 4)[:ny, :nx], device="cuda",
                       requires_grad=True)
    dp2 = 150 * 1e-2 * (nx - 1) ** 2 / float((eps ** 3 / (1 - eps) ** 2).mean())

    def J(e):
        K = e ** 3 * dp2 / (150 * (1 - e) ** 2)
        return NuHot.apply(e, K, params, steps, 6)

    J(eps).backward()
    g = eps.grad.cpu().numpy()
    e0 = eps.detach().cpu().numpy()
    Kr = e0 ** 3 * dp2 / (150 * (1 - e0) ** 2)
    _, rphi, rK = torch_ref.grad_nu_hot(e0, Kr, steps, nx=nx, ny=ny, Ra=1e5, Pr=1.0)
    dK = 3 * e0 ** 2 * dp2 / (150 * (1 - e0) ** 2) + 2 * e0 ** 3 * dp2 / (150 * (1 - e0) ** 3)
    check(g, rphi + rK * dK, 1e-10, "total dJ/deps")


def test_adjoint_with_heat_source():
    """The adjoint of the step with the heat source of Eqs. (30), (34), (36) (Sec. 4.3 setting)."""
    nx, ny, steps = 13, 11, 30
    params = dict(nx=nx, ny=ny, Ra=1e5, Ra_I=1e5, Pr=0.7)
    phi, K = workloads.random_medium(ny, nx, seed=44, K_lo=2.0, K_hi=20.0)
    J, gphi, gK = gpu_grad(params, phi, K, steps, 7, "fp64")
    Jr, rphi, rK = torch_ref.grad_nu_hot(phi, K, steps, **params)
    assert abs(J - Jr) <= 1e-11 * max(1.0, abs(Jr))
    check(gphi, rphi, 1e-9, "heat source dJ/dphi")
    check(gK, rK, 1e-9, "heat source dJ/dK")
