"""Pins of the oracle adjoint (``oracle/torch_ref.py``): its forward pass against the plain C
oracle, and its gradient of the hot-wall average Nusselt number (Eq. (38)) with respect to the
per-node porosity and permeability against central finite differences of the C oracle, at every
node of a small cavity (P13).  The finite differences use Richardson extrapolation, so their
truncation error is fourth order in the step.
"""
import numpy as np
import pytest
import torch

from oracle import ref, torch_ref

NX, NY, STEPS = 12, 12, 50
PARAMS = dict(nx=NX, ny=NY, Ra=1e5, Pr=0.71, bc=(0, 0, 1, 1), T_wall=(1.0, 0.0, 0.0, 0.0))


def fields(seed=13):
    r = np.random.default_rng(seed)
    phi = r.uniform(0.3, 0.9, (NY, NX))
    K = r.uniform(2.0, 20.0, (NY, NX))
    return phi, K


def test_torch_forward_equals_c_oracle(oracle):
    phi, K = fields()
    P = dict(PARAMS, bc=(0, 1, 1, 0), T_wall=(1.0, 0.0, 0.0, 0.25))
    lat = ref.RefLattice(phi=phi, K=K, **P)
    lat.step(STEPS)
    o = lat.observables()
    tl = torch_ref.TorchLattice(**P)
    f, g = tl.rest_state()
    tphi, tK = torch.tensor(phi), torch.tensor(K)
    for _ in range(STEPS):
        f, g = tl.step(f, g, tphi, tK)
    ot = tl.observables(f, g, tphi, tK)
    for k in ("ux", "uy", "p", "T"):
        np.testing.assert_allclose(ot[k].numpy(), o[k], atol=1e-14)
    assert abs(float(ot["nu_hot"]) - o["nu_hot"]) < 1e-13
    assert abs(float(ot["nu_cold"]) - o["nu_cold"]) < 1e-13
    fo, go = lat.get_state()
    np.testing.assert_allclose(f.numpy(), fo, atol=1e-14)
    np.testing.assert_allclose(g.numpy(), go, atol=1e-14)


def nu_hot_c(phi, K):
    lat = ref.RefLattice(phi=phi, K=K, **PARAMS)
    lat.step(STEPS)
    return lat.observables()["nu_hot"]


def fd_gradient(field, other, which, h):
    """Richardson-extrapolated central differences of the C oracle at every node."""
    g = np.zeros_like(field)
    for y in range(NY):
        for x in range(NX):
            vals = []
            for hh in (h, h / 2):
                fp, fm = field.copy(), field.copy()
                fp[y, x] += hh
                fm[y, x] -= hh
                if which == "phi":
                    jp, jm = nu_hot_c(fp, other), nu_hot_c(fm, other)
                else:
                    jp, jm = nu_hot_c(other, fp), nu_hot_c(other, fm)
                vals.append((jp - jm) / (2 * hh))
            g[y, x] = (4 * vals[1] - vals[0]) / 3
    return g


@pytest.mark.slow
def test_adjoint_gradient_equals_finite_differences(oracle):
    phi, K = fields()
    J, gphi, gK = torch_ref.grad_nu_hot(phi, K, STEPS, **PARAMS)
    assert abs(J - nu_hot_c(phi, K)) < 1e-13
    fphi = fd_gradient(phi, K, "phi", 1e-2)
    fK = fd_gradient(K, phi, "K", 1e-1)
    # gradients are nonzero throughout the cavity interior after 50 steps
    assert np.count_nonzero(np.abs(gphi) > 1e-12) > 0.8 * NX * NY
    np.testing.assert_allclose(gphi, fphi, rtol=0, atol=1e-8 * np.abs(fphi).max())
    # dJ/dK is ~3e-4 of dJ/dphi here; its differences sit closer to the rounding floor of J
    np.testing.assert_allclose(gK, fK, rtol=0, atol=2e-6 * np.abs(fK).max())


def test_adjoint_with_checkpoint_segments_is_unchanged(oracle):
    """Checkpoint-and-recompute over time segments changes nothing in the gradient."""
    phi, K = fields(21)
    _, g1, k1 = torch_ref.grad_nu_hot(phi, K, 30, **PARAMS)
    _, g2, k2 = torch_ref.grad_nu_hot(phi, K, 30, segment=7, **PARAMS)
    np.testing.assert_allclose(g1, g2, atol=1e-15)
    np.testing.assert_allclose(k1, k2, atol=1e-15)
