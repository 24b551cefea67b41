"""Mie series for a homogeneous dielectric sphere: an independent pin.

Written from the textbook solution (Bohren & Huffman, ch. 4; e^{-i omega t}):
for E_inc = e exp(i k d.x) scattered by a sphere of radius a with relative
refractive index n_rel (mu1 = mu0),

  E_s ~ e^{i k r} / r  E_inf,   E_inf = (i/k) [S2 (e.e_par_i) e_par_s + S1 (e.e_perp) e_perp],
  e_perp = d x xhat / |d x xhat|, e_par_i = e_perp x d, e_par_s = e_perp x xhat,
  S1 = sum (2n+1)/(n(n+1)) (a_n pi_n + b_n tau_n),  S2 = sum (2n+1)/(n(n+1)) (a_n tau_n + b_n pi_n).
"""
from __future__ import annotations

import numpy as np
from scipy.special import spherical_jn, spherical_yn


def mie_coefficients(x, mrel, nmax):
    n = np.arange(1, nmax + 1)
    mx = mrel * x
    jx, djx = spherical_jn(n, x), spherical_jn(n, x, derivative=True)
    yx, dyx = spherical_yn(n, x), spherical_yn(n, x, derivative=True)
    jm, djm = spherical_jn(n, mx), spherical_jn(n, mx, derivative=True)
    psi_x, dpsi_x = x * jx, jx + x * djx
    psi_m, dpsi_m = mx * jm, jm + mx * djm
    xi_x = x * (jx + 1j * yx)
    dxi_x = (jx + 1j * yx) + x * (djx + 1j * dyx)
    a = (mrel * psi_m * dpsi_x - psi_x * dpsi_m) / (mrel * psi_m * dxi_x - xi_x * dpsi_m)
    b = (psi_m * dpsi_x - mrel * psi_x * dpsi_m) / (psi_m * dxi_x - mrel * xi_x * dpsi_m)
    return a, b


def amplitudes(a, b, mu):
    nmax = a.size
    pi = np.zeros(nmax + 1)
    tau = np.zeros(nmax + 1)
    pi[1] = 1.0
    tau[1] = mu
    for n in range(2, nmax + 1):
        pi[n] = ((2 * n - 1) / (n - 1)) * mu * pi[n - 1] - (n / (n - 1)) * pi[n - 2]
        tau[n] = n * mu * pi[n] - (n + 1) * pi[n - 1]
    n = np.arange(1, nmax + 1)
    c = (2 * n + 1) / (n * (n + 1))
    S1 = np.sum(c * (a * pi[1:] + b * tau[1:]))
    S2 = np.sum(c * (a * tau[1:] + b * pi[1:]))
    return S1, S2


def far_field(k, radius, n_rel, d, e, dirs, nmax=None):
    x = k * radius
    if nmax is None:
        nmax = int(x + 4 * x ** (1 / 3) + 20)
    a, b = mie_coefficients(x, n_rel, nmax)
    d = np.asarray(d, float)
    out = np.zeros((len(dirs), 3), dtype=complex)
    for i, xh in enumerate(np.asarray(dirs, float)):
        mu = float(np.dot(d, xh))
        S1, S2 = amplitudes(a, b, mu)
        ep = np.cross(d, xh)
        ep /= np.linalg.norm(ep)
        epi = np.cross(ep, d)
        eps_ = np.cross(ep, xh)
        out[i] = (1j / k) * (S2 * np.dot(e, epi) * eps_ + S1 * np.dot(e, ep) * ep)
    return out
