"""Brute-force modal kernels by mpmath quadrature of the defining integrals
(eq. green11 and its target derivatives), for pinning the oracle."""
from __future__ import annotations

import mpmath as mp


def types_at(rt, zt, dr, dz, k0, k1, ms, dps=30):
    """[len(ms)][9] complex: g, d_r g, d_z g for k0 and k1, then the k0-k1
    differences of d_rr, d_rz, d_zz, by adaptive quadrature over phi."""
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
        out = []
        hs = []
        for k in (k0, k1):
            E = mp.exp(1j * k * rho)
            F1 = (1j * k * rho - 1) * E / (rho * rho2)
            out += [E / rho, rd * F1, zd * F1]
            G = E * (3 - 3j * k * rho - k * k * rho2) / (rho2 * rho2 * rho)
            hs.append((G, F1))
        G = hs[0][0] - hs[1][0]
        H = hs[0][1] - hs[1][1]
        out += [rd * rd * G + H, rd * zd * G, zd * zd * G + H]
        return out

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
