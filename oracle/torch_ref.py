"""Differentiable FP64 CPU oracle: the same time step as ``lbm_ref.c``, written with plain
PyTorch CPU tensor operations so that reverse-mode automatic differentiation yields the exact
gradient of the discrete map.

TEST INFRASTRUCTURE ONLY (tests, smoke check, CPU-baseline leg of the benchmark).  It is the
reference for the discrete adjoint: the derivative of the hot-wall average Nusselt number
(Eq. (38)) after N steps with respect to the per-node porosity phi and permeability K.  Its
forward pass is checked against ``lbm_ref.c`` and its gradient against central finite
differences of ``lbm_ref.c``.

The step order and the readings of the paper are those of ``lbm_ref.c``:
stream (Eqs. (18), (35)) -> non-equilibrium extrapolation at wall nodes -> macroscopic recovery
(Eqs. (36), (22), (21), (23), (4)) -> collision in moment space (Eqs. (17), (34)).

The two non-smooth points of the model, |v| in Eq. (21) and |u| in Eq. (4) at zero velocity,
are differentiated by their continuous limits: d|v|/dv is taken as 0 at v = 0, which gives
du/dv = I/(2 l0) there and d(|u| u)/du = 0 at u = 0.
"""
from __future__ import annotations

import numpy as np
import torch
from torch.utils.checkpoint import checkpoint

from . import ref

DT = torch.float64
EX = (0, 1, 0, -1, 0, 1, -1, -1, 1)
EY = (0, 0, 1, 0, -1, 1, 1, -1, -1)
W9 = (4 / 9, 1 / 9, 1 / 9, 1 / 9, 1 / 9, 1 / 36, 1 / 36, 1 / 36, 1 / 36)
# Eq. (11) and Eq. (28)
M = torch.tensor([
    [1, 1, 1, 1, 1, 1, 1, 1, 1],
    [-4, -1, -1, -1, -1, 2, 2, 2, 2],
    [4, -2, -2, -2, -2, 1, 1, 1, 1],
    [0, 1, 0, -1, 0, 1, -1, -1, 1],
    [0, -2, 0, 2, 0, 1, -1, -1, 1],
    [0, 0, 1, 0, -1, 1, 1, -1, -1],
    [0, 0, -2, 0, 2, 1, 1, -1, -1],
    [0, 1, -1, 1, -1, 0, 0, 0, 0],
    [0, 0, 0, 0, 0, 1, -1, 1, -1]], dtype=DT)
N = torch.tensor([
    [1, 1, 1, 1, 1],
    [0, 1, 0, -1, 0],
    [0, 0, 1, 0, -1],
    [-4, 1, 1, 1, 1],
    [0, 1, -1, 1, -1]], dtype=DT)
MINV = torch.linalg.inv(M)
NINV = torch.linalg.inv(N)


def _safe_norm(ax, ay):
    """sqrt(ax^2 + ay^2) whose derivative is taken as 0 where the vector vanishes."""
    s = ax * ax + ay * ay
    pos = s > 0
    r = torch.sqrt(torch.where(pos, s, torch.ones_like(s)))
    return torch.where(pos, r, torch.zeros_like(s))


class TorchLattice:
    """One cavity; the state is the post-collision population field (f[9,ny,nx], g[5,ny,nx])."""

    def __init__(self, **params):
        p = dict(ref.DEFAULTS)
        p.update(params)
        self.p = p
        self.d = ref.derived(**params)
        self.nx, self.ny = int(p["nx"]), int(p["ny"])
        nx, ny = self.nx, self.ny
        bc = p["bc"]
        self.perx = bc[0] == ref.PERIODIC
        self.pery = bc[2] == ref.PERIODIC
        xs = torch.arange(nx).view(1, nx).expand(ny, nx)
        ys = torch.arange(ny).view(ny, 1).expand(ny, nx)
        onW = (xs == 0) & (bc[0] != ref.PERIODIC)
        onE = (xs == nx - 1) & (bc[1] != ref.PERIODIC)
        onS = (ys == 0) & (bc[2] != ref.PERIODIC)
        onN = (ys == ny - 1) & (bc[3] != ref.PERIODIC)
        self.wall = onW | onE | onS | onN
        dx = onW.long() - onE.long()
        dy = onS.long() - onN.long()
        self.xf_index = ((ys + dy) * nx + (xs + dx)).reshape(-1)   # inward neighbour
        # wall temperature: isothermal side(s) fix it, otherwise the neighbour's T is used
        Tw = p["T_wall"]
        iso = [b == ref.ISOTHERMAL for b in bc]
        isoX = (onW & iso[0]) | (onE & iso[1])
        isoY = (onS & iso[2]) | (onN & iso[3])
        TX = torch.where(onW, torch.tensor(float(Tw[0]), dtype=DT),
                         torch.tensor(float(Tw[1]), dtype=DT))
        TY = torch.where(onS, torch.tensor(float(Tw[2]), dtype=DT),
                         torch.tensor(float(Tw[3]), dtype=DT))
        self.T_fixed = torch.where(isoX & isoY, 0.5 * (TX + TY),
                                   torch.where(isoX, TX, torch.where(isoY, TY,
                                                                     torch.zeros((), dtype=DT))))
        self.T_is_fixed = isoX | isoY
        # rates, Eq. (20) and Eq. (31) with the values of Sec. 4
        sv, sT = 1.0 / self.d["tau_v"], 1.0 / self.d["tau_T"]
        if p["uniform_rates"]:
            s = [sv] * 9
            z = [sT] * 5
        else:
            s = [1.0, p["s_e"], p["s_eps"], 1.0, p["s_q"], 1.0, p["s_q"], sv, sv]
            z = [1.0, sT, sT, p["zeta3"], p["zeta4"]]
        self.s = torch.tensor(s, dtype=DT).view(9, 1, 1)
        self.z = torch.tensor(z, dtype=DT).view(5, 1, 1)

    # ---- state ----
    def rest_state(self):
        p = self.p
        f = torch.tensor(W9, dtype=DT).view(9, 1, 1) * p["rho0"] * torch.ones(
            9, self.ny, self.nx, dtype=DT)
        varpi = p["varpi"]
        wt = torch.tensor([(1 - varpi) / 5] + [(4 + varpi) / 20] * 4, dtype=DT).view(5, 1, 1)
        g = wt * p["T_init"] * torch.ones(5, self.ny, self.nx, dtype=DT)
        return f, g

    # ---- pieces of one step ----
    def _stream(self, a, ex, ey, fill):
        """a_i(x) <- a_i(x - e_i); out-of-domain sources (only at wall nodes, which are rebuilt
        afterwards) are filled with a finite constant so that no NaN enters the derivative."""
        nx, ny = self.nx, self.ny
        out = []
        for i in range(a.shape[0]):
            plane = torch.roll(a[i], shifts=(ey[i], ex[i]), dims=(0, 1))
            if not self.perx and ex[i] != 0:
                col = 0 if ex[i] > 0 else nx - 1
                mask = torch.zeros(ny, nx, dtype=torch.bool)
                mask[:, col] = True
                plane = torch.where(mask, torch.full_like(plane, fill[i]), plane)
            if not self.pery and ey[i] != 0:
                row = 0 if ey[i] > 0 else ny - 1
                mask = torch.zeros(ny, nx, dtype=torch.bool)
                mask[row, :] = True
                plane = torch.where(mask, torch.full_like(plane, fill[i]), plane)
            out.append(plane)
        return torch.stack(out)

    def _fluid_macros(self, fh, gh, phi, K):
        p, d = self.p, self.d
        rho0 = p["rho0"]
        T = gh.sum(0) + 0.5 * d["Q"] / p["sigma"]                         # Eq. (36)
        Gx = torch.full_like(T, p["ext_accel"][0])
        Gy = p["ext_accel"][1] + d["gbeta"] * (T - d["T0"])
        ex = torch.tensor(EX, dtype=DT).view(9, 1, 1)
        ey = torch.tensor(EY, dtype=DT).view(9, 1, 1)
        vx = (ex * fh).sum(0) / rho0 + 0.5 * phi * Gx                      # Eq. (22)
        vy = (ey * fh).sum(0) / rho0 + 0.5 * phi * Gy
        Fphi = 1.75 / torch.sqrt(150.0 * phi ** 3) if p["forchheimer"] else torch.zeros_like(phi)
        l0 = 0.5 * (1.0 + phi * 0.5 * d["nu"] / K)
        l1 = phi * 0.5 * Fphi / torch.sqrt(K)
        vmag = _safe_norm(vx, vy)
        den = l0 + torch.sqrt(l0 * l0 + l1 * vmag)                          # Eq. (21)
        ux, uy = vx / den, vy / den
        uu = ux * ux + uy * uy
        cs2 = d["cs2"]
        s0 = W9[0] * (-uu / (2.0 * phi * cs2))                              # Eq. (14), i = 0
        phip = cs2 / (1.0 - W9[0]) * (fh[1:].sum(0) + rho0 * s0)            # Eq. (23) times phi
        umag = _safe_norm(ux, uy)
        Fx = -phi * d["nu"] / K * ux - phi * Fphi / torch.sqrt(K) * umag * ux + phi * Gx  # Eq. (4)
        Fy = -phi * d["nu"] / K * uy - phi * Fphi / torch.sqrt(K) * umag * uy + phi * Gy
        return T, ux, uy, phip, Fx, Fy

    def _feq(self, phip, ux, uy, phi):
        """Eq. (13) with Eq. (14)."""
        cs2, rho0 = self.d["cs2"], self.p["rho0"]
        uu = ux * ux + uy * uy
        out = []
        for i in range(9):
            eu = EX[i] * ux + EY[i] * uy
            si = W9[i] * (eu / cs2 + eu * eu / (2 * phi * cs2 * cs2) - uu / (2 * phi * cs2))
            if i == 0:
                out.append(rho0 - (1 - W9[0]) * phip / cs2 + rho0 * si)
            else:
                out.append(W9[i] * phip / cs2 + rho0 * si)
        return torch.stack(out)

    def _geq(self, T, ux, uy):
        """Eq. (37a)."""
        sigma, varpi = self.p["sigma"], self.p["varpi"]
        csT2 = (4 + varpi) / 10
        out = []
        for i in range(5):
            wt = (1 - varpi) / 5 if i == 0 else (4 + varpi) / 20
            out.append(wt * T * (1 + (EX[i] * ux + EY[i] * uy) / (sigma * csT2)))
        return torch.stack(out)

    def post_stream(self, f, g, phi, K):
        """Streaming + wall reconstruction + macroscopics: returns (fh, gh, macros)."""
        p, d = self.p, self.d
        varpi = p["varpi"]
        ffill = [W9[i] * p["rho0"] for i in range(9)]
        gfill = [((1 - varpi) / 5 if i == 0 else (4 + varpi) / 20) * p["T_init"] for i in range(5)]
        fh = self._stream(f, EX, EY, ffill)
        gh = self._stream(g, EX[:5], EY[:5], gfill)
        T, ux, uy, phip, Fx, Fy = self._fluid_macros(fh, gh, phi, K)
        n = self.nx * self.ny
        idx = self.xf_index

        def at_f(a):  # value at the inward neighbour, per node
            return a.reshape(-1)[idx].reshape(self.ny, self.nx)

        Tf, uxf, uyf, phipf, phif = at_f(T), at_f(ux), at_f(uy), at_f(phip), at_f(phi)
        fhf = fh.reshape(9, n)[:, idx].reshape(9, self.ny, self.nx)
        ghf = gh.reshape(5, n)[:, idx].reshape(5, self.ny, self.nx)
        zero = torch.zeros_like(T)
        Tb = torch.where(self.T_is_fixed, self.T_fixed, Tf)
        fb = self._feq(phipf, zero, zero, phi) + (fhf - self._feq(phipf, uxf, uyf, phif))
        gb = self._geq(Tb, zero, zero) + (ghf - self._geq(Tf, uxf, uyf))
        wall = self.wall
        fh = torch.where(wall, fb, fh)
        gh = torch.where(wall, gb, gh)
        T = torch.where(wall, Tb, T)
        ux = torch.where(wall, zero, ux)
        uy = torch.where(wall, zero, uy)
        phip = torch.where(wall, phipf, phip)
        Fx = torch.where(wall, phi * p["ext_accel"][0], Fx)
        Fy = torch.where(wall, phi * (p["ext_accel"][1] + d["gbeta"] * (Tb - d["T0"])), Fy)
        return fh, gh, (T, ux, uy, phip, Fx, Fy)

    def collide(self, fh, gh, mac, phi):
        p = self.p
        rho0, sigma, varpi = p["rho0"], p["sigma"], p["varpi"]
        T, ux, uy, phip, Fx, Fy = mac
        n = self.nx * self.ny
        m = (M @ fh.reshape(9, n)).reshape(9, self.ny, self.nx)
        uu = ux * ux + uy * uy
        meq = torch.stack([                                                # Eq. (16)
            torch.full_like(T, rho0),
            -4 * rho0 + 6 * phip + 3 * rho0 * uu / phi,
            4 * rho0 - 9 * phip - 3 * rho0 * uu / phi,
            rho0 * ux, -rho0 * ux, rho0 * uy, -rho0 * uy,
            rho0 * (ux * ux - uy * uy) / phi, rho0 * ux * uy / phi])
        uF = ux * Fx + uy * Fy
        S = torch.stack([                                                  # Eq. (19)
            torch.zeros_like(T), 6 * rho0 * uF / phi, -6 * rho0 * uF / phi,
            rho0 * Fx, -rho0 * Fx, rho0 * Fy, -rho0 * Fy,
            2 * rho0 * (ux * Fx - uy * Fy) / phi, rho0 * (ux * Fy + uy * Fx) / phi])
        mp = m - self.s * (m - meq) + (1 - 0.5 * self.s) * S                # Eq. (17)
        fp = (MINV @ mp.reshape(9, n)).reshape(9, self.ny, self.nx)
        nm = (N @ gh.reshape(5, n)).reshape(5, self.ny, self.nx)
        ne = torch.stack([T, ux * T / sigma, uy * T / sigma, varpi * T, torch.zeros_like(T)])  # Eq. (29)
        Q = self.d["Q"]
        psi = torch.tensor([Q / sigma, 0.0, 0.0, varpi * Q / sigma, 0.0], dtype=DT).view(5, 1, 1)
        np_ = nm - self.z * (nm - ne) + (1 - 0.5 * self.z) * psi           # Eqs. (30), (34)
        gp = (NINV @ np_.reshape(5, n)).reshape(5, self.ny, self.nx)
        return fp, gp

    def step(self, f, g, phi, K):
        fh, gh, mac = self.post_stream(f, g, phi, K)
        return self.collide(fh, gh, mac, phi)

    def nu(self, T):
        """Eq. (38): hot (west) and cold (east) wall averages with the five-point stencil."""
        d = self.d
        dh = (-25 * T[:, 0] + 48 * T[:, 1] - 36 * T[:, 2] + 16 * T[:, 3] - 3 * T[:, 4]) / 12
        dc = (25 * T[:, -1] - 48 * T[:, -2] + 36 * T[:, -3] - 16 * T[:, -4] + 3 * T[:, -5]) / 12
        w = torch.ones(self.ny, dtype=DT)
        w[0] = w[-1] = 0.5
        scale = -d["L"] / d["dT"] / (self.ny - 1)
        return scale * (w * dh).sum(), scale * (w * dc).sum()

    def observables(self, f, g, phi, K):
        _, _, mac = self.post_stream(f, g, phi, K)
        T, ux, uy, phip, _, _ = mac
        nh, nc = self.nu(T)
        return dict(ux=ux, uy=uy, p=phip / phi, T=T, nu_hot=nh, nu_cold=nc)

    # ---- whole runs ----
    def _segment(self, f, g, phi, K, nsteps):
        for _ in range(nsteps):
            f, g = self.step(f, g, phi, K)
        return f, g

    def nu_hot_after(self, phi, K, nsteps, segment=0):
        """J = Nu_hot after nsteps steps from rest; differentiable in phi and K.  With
        segment > 0 the run is split into checkpointed segments of that many steps."""
        f, g = self.rest_state()
        done = 0
        while done < nsteps:
            k = nsteps - done if segment <= 0 else min(segment, nsteps - done)
            if segment > 0 and torch.is_grad_enabled():
                # reentrant form: the non-reentrant one keeps every step's intermediates here
                f, g = checkpoint(self._segment, f, g, phi, K, k, use_reentrant=True)
            else:
                f, g = self._segment(f, g, phi, K, k)
            done += k
        return self.observables(f, g, phi, K)["nu_hot"]


def grad_nu_hot(phi: np.ndarray, K: np.ndarray, nsteps: int, segment: int = 0, **params):
    """Oracle adjoint: (J, dJ/dphi, dJ/dK) for J = Nu_hot after nsteps steps from rest."""
    lat = TorchLattice(**params)
    tphi = torch.tensor(np.asarray(phi, dtype=np.float64), requires_grad=True)
    tK = torch.tensor(np.asarray(K, dtype=np.float64), requires_grad=True)
    J = lat.nu_hot_after(tphi, tK, nsteps, segment=segment)
    J.backward()
    return float(J.detach()), tphi.grad.numpy().copy(), tK.grad.numpy().copy()
