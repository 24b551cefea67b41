"""Dense per-mode solves (Section 2.1 discussion of Gaussian elimination;
Section 6: LU per mode, extra right-hand sides reuse the factors).

Negative modes use the parity of the modal operators under m -> -m
(g_{-m} = g_m, g^2_{-m} = g^2_m, g^3_{-m} = -g^3_m, odd powers of i m flip):
in the N expansion the t-t and theta-theta entries are even in m and the
cross entries odd, in the K expansion the reverse.  With unknowns
(J^1, J^2, M^1, M^2) and rows (H-equation t, theta, E-equation t, theta) this is
A_{-m} = D A_m D with D = diag(1, -1, -1, 1) per node, so
x_{-m} = D A_m^{-1} D b_{-m}.
"""
from __future__ import annotations

import numpy as np


def parity_diag(N):
    return np.tile(np.array([1.0, -1.0, -1.0, 1.0]), N)


def solve_modes(mats, w, rhs, m_lo, m_hi):
    """mats[m] (m = 0..M): L^2-weighted matrices; rhs [m_hi-m_lo+1, nrhs, 4N]
    in physical (unweighted) form.  Returns x of the same shape."""
    N = w.size
    sw = np.repeat(np.sqrt(w), 4)
    D = parity_diag(N)
    out = np.zeros_like(rhs)
    for i, m in enumerate(range(m_lo, m_hi + 1)):
        A = mats[abs(m)]
        b = rhs[i].T * sw[:, None]
        if m < 0:
            b = b * D[:, None]
        xt = np.linalg.solve(A, b)
        if m < 0:
            xt = xt * D[:, None]
        out[i] = (xt / sw[:, None]).T
    return out
