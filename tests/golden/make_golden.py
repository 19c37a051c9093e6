"""Writes the stored expected values of the full-size parity tests.  Calls only the CPU oracle
(``oracle/``) on the seeded inputs of ``paper_1308_2071_amd.workloads``; nothing here comes from
the HIP path.

    python tests/golden/make_golden.py [porous256] [adjoint256]

porous256.npz   FP64 oracle after 50,000 steps of the 256 x 256 cavity (phi = 0.4, Da = 1e-2,
                Ra = 1e5, Pr = 1): u_x, u_y, p, T on every 4th node in x and y, each field's
                min and max over all nodes, Nu_hot and Nu_cold (Eq. (38)).
adjoint256.npz  J = Nu_hot after 2,000 steps of the smoothed-porosity 256 x 256 cavity:
                the oracle adjoint (reverse-mode derivative of the FP64 step) dJ/dphi, dJ/dK on
                every 2nd node, their maxima over all nodes, and central finite differences of
                the FP64 C oracle for dJ/deps at 16 probe nodes, where K = K(eps) by Eq. (5)
                with d_p held at its unperturbed value (Richardson-extrapolated, steps 1e-3
                and 5e-4).
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import ref, torch_ref  # noqa: E402
from paper_1308_2071_amd import workloads  # noqa: E402


def porous256():
    w = workloads.porous256()
    t0 = time.time()
    lat = ref.RefLattice(phi_uniform=w["phi"], **w["params"])
    lat.step(w["steps"])
    o = lat.observables()
    out = dict(steps=w["steps"], nu_hot=o["nu_hot"], nu_cold=o["nu_cold"])
    for k in ("ux", "uy", "p", "T"):
        out[k] = o[k][::4, ::4].copy()
        out[k + "_min"] = o[k].min()
        out[k + "_max"] = o[k].max()
    np.savez(os.path.join(HERE, "porous256.npz"), **out)
    print(f"porous256: Nu_hot {o['nu_hot']:.10f} Nu_cold {o['nu_cold']:.10f} "
          f"({time.time() - t0:.0f} s)", flush=True)


def kc(eps, dp2):
    return eps ** 3 * dp2 / (150.0 * (1.0 - eps) ** 2)


def adjoint256():
    w = workloads.adjoint256()
    eps, K, steps = w["phi"], w["K"], w["steps"]
    n = w["params"]["nx"]
    dp2 = (K / (eps ** 3 / (150.0 * (1.0 - eps) ** 2))).mean()
    t0 = time.time()
    # 20-step checkpoint segments keep the autograd tape near 6 GB at 256^2 (the segment length
    # does not change the gradient)
    J, gphi, gK = torch_ref.grad_nu_hot(eps, K, steps, segment=20, **w["params"])
    print(f"adjoint256: oracle adjoint J = {J:.12f} ({time.time() - t0:.0f} s)", flush=True)

    def J_at(e):
        lat = ref.RefLattice(phi=e, K=kc(e, dp2), **w["params"])
        lat.step(steps)
        return lat.observables()["nu_hot"]

    fd = []
    for (y, x) in w["probes"]:
        d = []
        for h in (1e-3, 5e-4):
            ep, em = eps.copy(), eps.copy()
            ep[y, x] += h
            em[y, x] -= h
            d.append((J_at(ep) - J_at(em)) / (2 * h))
        fd.append((4 * d[1] - d[0]) / 3)
        print(f"  probe {(y, x)}: fd {fd[-1]:.6e}", flush=True)
    deps = 3 * eps ** 2 * dp2 / (150 * (1 - eps) ** 2) + 2 * eps ** 3 * dp2 / (150 * (1 - eps) ** 3)
    np.savez(os.path.join(HERE, "adjoint256.npz"), J=J, steps=steps, n=n,
             gphi=gphi[::2, ::2].copy(), gK=gK[::2, ::2].copy(),
             gphi_absmax=np.abs(gphi).max(), gK_absmax=np.abs(gK).max(),
             probes=np.array(w["probes"]), fd_eps=np.array(fd),
             adj_eps=np.array([gphi[y, x] + gK[y, x] * deps[y, x] for (y, x) in w["probes"]]))
    print(f"adjoint256 done ({time.time() - t0:.0f} s)", flush=True)


if __name__ == "__main__":
    which = sys.argv[1:] or ["porous256", "adjoint256"]
    ref.set_threads(len(os.sched_getaffinity(0)))
    for name in which:
        globals()[name]()
