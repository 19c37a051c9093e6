"""The free level of the pressure, shared by the FP32 parity checks.

The step depends on phi p only through differences: a uniform shift c of phi p at every node
(Eq. (13): f_0 by -(1 - w0) c / cs^2, f_i by w_i c / cs^2) moves the equilibrium moments of
Eq. (16) by exactly what it moves M f, so m - m_eq, u and T are unchanged and phi p stays
shifted by c (pinned by ``test_oracle_gauge.py``).  Nothing in the scheme fixes that level, so
FP32 rounding moves it; the FP32 checks therefore compare p up to a uniform shift of phi p,
which at a node of porosity phi is c / phi.
"""
import numpy as np


def phip_gauged(dp, phi):
    """dp = p_gpu - p_oracle per node; phi a scalar or a field of the same shape.  Returns dp
    less c / phi, with c the mean of phi dp (the uniform phi p shift that fits best)."""
    phi = np.broadcast_to(np.asarray(phi, dtype=np.float64), dp.shape)
    c = float(np.mean(phi * dp))
    return dp - c / phi
