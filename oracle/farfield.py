"""Far-field pattern from the surface currents.

From the exterior representation (eq. exteriorfield) with the asymptotics of
the Green's function, E_0(x) ~ e^{i k0 |x|}/|x| E_inf(xhat) with

    E_inf(xhat) = (1/4pi) [ i k0 xhat x Mt - i omega mu0 xhat x (xhat x Jt) ],
    Jt = int_Gamma e^{-i k0 xhat.y} J(y) da(y),  Mt likewise,

(the printed far-field formula omits the M term; this is the statement that
follows from eq. exteriorfield).  J(y) = sum_m (J^1_m t + J^2_m e_theta) e^{i m theta};
the surface integral is a trapezoid rule in theta and the Gauss-Legendre
arclength weights along the generating curve.
"""
from __future__ import annotations

import numpy as np


def far_field(curve, w, x_modes, m_lo, k0, omega, mu0, dirs, n_theta=None):
    """x_modes: [n_modes, 4N] for one right-hand side (modes m_lo..).
    dirs: [D, 3] unit vectors.  Returns E_inf [D, 3] complex."""
    N = curve.n
    nm = x_modes.shape[0]
    ms = np.arange(m_lo, m_lo + nm)
    rmax = float(curve.r.max())
    if n_theta is None:
        n_theta = int(2 * (np.max(np.abs(ms)) + k0 * rmax) + 64)
    th = 2 * np.pi * np.arange(n_theta) / n_theta
    ph = np.exp(1j * np.outer(ms, th))  # [nm, T]
    X = x_modes.reshape(nm, N, 4)
    comps = np.einsum("mnc,mt->nct", X, ph)  # [N, 4, T]
    tr, tz = -curve.nz, curve.nr
    ct, st = np.cos(th), np.sin(th)
    def vec(a1, a2):
        # a1 t + a2 e_theta in Cartesian: t = tr e_r + tz e_z
        vx = a1 * tr[:, None] * ct - a2 * st
        vy = a1 * tr[:, None] * st + a2 * ct
        vz = a1 * tz[:, None]
        return np.stack([vx, vy, vz], axis=-1)  # [N, T, 3]
    J = vec(comps[:, 0], comps[:, 1])
    M = vec(comps[:, 2], comps[:, 3])
    y = np.stack([curve.r[:, None] * ct, curve.r[:, None] * st,
                  np.broadcast_to(curve.z[:, None], (N, n_theta))], axis=-1)
    da = (w * curve.r)[:, None] * (2 * np.pi / n_theta)
    out = np.zeros((len(dirs), 3), dtype=complex)
    for i, xh in enumerate(np.asarray(dirs, float)):
        e = np.exp(-1j * k0 * (y @ xh)) * da
        Jt = np.einsum("nt,ntc->c", e, J)
        Mt = np.einsum("nt,ntc->c", e, M)
        out[i] = (1j * k0 * np.cross(xh, Mt) - 1j * omega * mu0 * np.cross(xh, np.cross(xh, Jt))) / (4 * np.pi)
    return out
