"""Brute-force modal kernels by mpmath quadrature of the defining integrals
(eq. green11 and its target derivatives), for pinning the oracle."""
from __future__ import annotations

import mpmath as mp


def types_at(rt, zt, dr, dz, k0, k1, ms, dps=30):
    """[len(ms)][9] complex: g, d_r g, d_z g for k0, the same for the k0-k1
    difference, then the k0-k1 differences of d_rr, d_rz, d_zz, by adaptive
    quadrature over phi (differences taken in working precision)."""
    mp.mp.dps = dps
    rt, zt, dr, dz = (mp.mpf(v) for v in (rt, zt, dr, dz))
    rs = rt + dr
    zd = -dz
    k0 = mp.mpc(k0)
    k1 = mp.mpc(k1)
    d2 = dr * dr + dz * dz

    def integrands(phi):
        rho2 = d2 + 4 * rt * rs * mp.sin(phi / 2) ** 2
        rho = mp.sqrt(rho2)
        rd = rt - rs * mp.cos(phi)
        f = []
        for k in (k0, k1):
            E = mp.exp(1j * k * rho)
            F1 = (1j * k * rho - 1) * E / (rho * rho2)
            G = E * (3 - 3j * k * rho - k * k * rho2) / (rho2 * rho2 * rho)
            f.append((E / rho, F1, G))
        dg = f[0][0] - f[1][0]
        H = f[0][1] - f[1][1]
        G = f[0][2] - f[1][2]
        return [f[0][0], rd * f[0][1], zd * f[0][1], dg, rd * H, zd * H,
                rd * rd * G + H, rd * zd * G, zd * zd * G + H]

    sc = mp.sqrt(d2 / (rt * rs))
    pts = [mp.mpf(0)] + [sc * mp.mpf(3) ** j for j in range(0, 60) if sc * mp.mpf(3) ** j < mp.pi]
    pts += [mp.pi]
    res = []
    for m in ms:
        row = []
        for t in range(9):
            v = 2 * mp.quad(lambda p: integrands(p)[t] * mp.cos(m * p), pts) / (4 * mp.pi)
            row.append(complex(v))
        res.append(row)
    return res
