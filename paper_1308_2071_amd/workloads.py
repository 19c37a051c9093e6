"""Seeded synthetic inputs for the cavity workloads.  This module holds no arithmetic of the
lattice Boltzmann method: it only draws the problem statements (grids, dimensionless groups,
porosity fields) that both the HIP path and the CPU oracle receive.

The porous media are synthetic: the paper's cavities are homogeneous (Sec. 2); the per-node
porosity fields below apply its Ergun / Kozeny-Carman permeability, Eq. (5), K = phi^3 d_p^2 /
(150 (1 - phi)^2), pointwise, with d_p chosen so that the sample mean of K equals Da L^2.

Workloads (W = west, E = east, S = south, N = north walls):
  porous64      64 x 64, phi = 0.6, Da = 1e-2, Ra = 1e3, Pr = 1, 20k steps, FP64
  porous256     256 x 256, phi = 0.4, Da = 1e-2, Ra = 1e5, Pr = 1, 50k steps, FP32 and FP64
  roofline4096  4096 x 4096, phi ~ U[0.3, 0.9] per node, K Kozeny-Carman with mean Da = 1e-3,
                Ra = 1e6, Pr = 0.71, FP32, 2000 timed steps
  batch64       64 cavities, side in {64, 96, 128, 192, 256, 384, 512}, Ra log-uniform
                [1e3, 1e6], Da log-uniform [1e-4, 1e-1], phi ~ U[0.2, 0.9], Pr in {0.71, 1, 7},
                FP32, 10k steps each
  adjoint256    256 x 256, Ra = 1e5, Pr = 1, phi = clip(0.5 + 0.1 z, 0.2, 0.9) with z unit
                Gaussian noise smoothed by a Gaussian of 4 nodes and re-standardised, K
                Kozeny-Carman with mean Da = 1e-2, 2000 steps, checkpoint every 100
All cavities: hot west wall T = 1, cold east wall T = 0, adiabatic south and north walls,
start from rest at T = 0.5 (Sec. 4.1).
"""
from __future__ import annotations

import numpy as np

SEED_ROOFLINE = 13082071
SEED_BATCH = 13082072
SEED_ADJOINT = 13082073
SEED_PROBES = 13082074

ISO, ADIA, PER = 0, 1, 2
CAVITY = dict(bc=(ISO, ISO, ADIA, ADIA), T_wall=(1.0, 0.0, 0.0, 0.0), T_init=0.5)


def cavity(nx, ny=None, **kw) -> dict:
    d = dict(CAVITY, nx=int(nx), ny=int(ny if ny is not None else nx))
    d.update(kw)
    return d


def porous64() -> dict:
    return dict(params=cavity(64, Ra=1e3, Pr=1.0, Da=1e-2), phi=0.6, steps=20000)


def porous256() -> dict:
    return dict(params=cavity(256, Ra=1e5, Pr=1.0, Da=1e-2), phi=0.4, steps=50000)


def kozeny_carman_field(phi: np.ndarray, mean_Da: float, L: float) -> np.ndarray:
    """Eq. (5) permeability with d_p^2 fixed by mean(K) = mean_Da L^2."""
    shape = phi ** 3 / (150.0 * (1.0 - phi) ** 2)
    dp2 = mean_Da * L * L / shape.mean()
    return shape * dp2


def roofline4096(n: int = 4096, seed: int = SEED_ROOFLINE) -> dict:
    rng = np.random.default_rng(seed)
    phi = rng.uniform(0.3, 0.9, size=(n, n))
    K = kozeny_carman_field(phi, 1e-3, n - 1)
    return dict(params=cavity(n, Ra=1e6, Pr=0.71), phi=phi, K=K, steps=2000)


def batch64(n: int = 64, seed: int = SEED_BATCH) -> list:
    rng = np.random.default_rng(seed)
    sides = (64, 96, 128, 192, 256, 384, 512)
    out = []
    for _ in range(n):
        side = int(rng.choice(sides))
        Ra = 10.0 ** rng.uniform(3, 6)
        Da = 10.0 ** rng.uniform(-4, -1)
        phi = float(rng.uniform(0.2, 0.9))
        Pr = float(rng.choice((0.71, 1.0, 7.0)))
        out.append(dict(params=cavity(side, Ra=float(Ra), Pr=Pr, Da=float(Da)), phi=phi))
    return out


def smoothed_porosity(n: int, seed: int, mean=0.5, std=0.1, sigma=4.0, lo=0.2, hi=0.9):
    from scipy.ndimage import gaussian_filter
    rng = np.random.default_rng(seed)
    z = gaussian_filter(rng.standard_normal((n, n)), sigma=sigma, mode="reflect", truncate=4.0)
    z = (z - z.mean()) / z.std()
    return np.clip(mean + std * z, lo, hi)


def adjoint256(n: int = 256, seed: int = SEED_ADJOINT) -> dict:
    phi = smoothed_porosity(n, seed)
    K = kozeny_carman_field(phi, 1e-2, n - 1)
    rng = np.random.default_rng(SEED_PROBES)
    near = [(int(rng.integers(1, n - 1)), int(rng.integers(1, 9))) for _ in range(8)]
    anywhere = [(int(rng.integers(1, n - 1)), int(rng.integers(1, n - 1))) for _ in range(8)]
    return dict(params=cavity(n, Ra=1e5, Pr=1.0), phi=phi, K=K, steps=2000, checkpoint=100,
                probes=near + anywhere)  # probes are (y, x)


def random_medium(ny, nx, seed, phi_lo=0.3, phi_hi=0.9, K_lo=2.0, K_hi=40.0):
    rng = np.random.default_rng(seed)
    return rng.uniform(phi_lo, phi_hi, (ny, nx)), rng.uniform(K_lo, K_hi, (ny, nx))
