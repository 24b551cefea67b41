"""Mie series for a homogeneous sphere: an independent pin.

Written from the textbook solution (Bohren & Huffman, ch. 4; e^{-i omega t}):
for E_inc = e exp(i k d.x) in a medium of permeability mu scattered by a sphere
of radius a, permeability mu1 and relative refractive index m (= k1/k, complex
for an absorbing sphere), with Riccati-Bessel functions psi_n(x) = x j_n(x) and
xi_n(x) = x h_n^(1)(x),

  a_n = (mu m psi_n(mx) psi_n'(x) - mu1 psi_n(x) psi_n'(mx))
      / (mu m psi_n(mx) xi_n'(x) - mu1 xi_n(x) psi_n'(mx)),
  b_n = (mu1 psi_n(mx) psi_n'(x) - mu m psi_n(x) psi_n'(mx))
      / (mu1 psi_n(mx) xi_n'(x) - mu m xi_n(x) psi_n'(mx)),

  E_s ~ e^{i k r} / r  E_inf,   E_inf = (i/k) [S2 (e.e_par_i) e_par_s + S1 (e.e_perp) e_perp],
  e_perp = d x xhat / |d x xhat|, e_par_i = e_perp x d, e_par_s = e_perp x xhat,
  S1 = sum (2n+1)/(n(n+1)) (a_n pi_n + b_n tau_n),  S2 = sum (2n+1)/(n(n+1)) (a_n tau_n + b_n pi_n).

For mu1 = mu the coefficients reduce to the nonmagnetic ones.
"""
from __future__ import annotations

import numpy as np
from scipy.special import spherical_jn, spherical_yn


def mie_coefficients(x, mrel, nmax, mu=1.0, mu1=1.0):
    n = np.arange(1, nmax + 1)
    mx = mrel * x
    jx, djx = spherical_jn(n, x), spherical_jn(n, x, derivative=True)
    yx, dyx = spherical_yn(n, x), spherical_yn(n, x, derivative=True)
    jm, djm = spherical_jn(n, mx), spherical_jn(n, mx, derivative=True)
    psi_x, dpsi_x = x * jx, jx + x * djx
    psi_m, dpsi_m = mx * jm, jm + mx * djm
    xi_x = x * (jx + 1j * yx)
    dxi_x = (jx + 1j * yx) + x * (djx + 1j * dyx)
    a = (mu * mrel * psi_m * dpsi_x - mu1 * psi_x * dpsi_m) / (mu * mrel * psi_m * dxi_x - mu1 * xi_x * dpsi_m)
    b = (mu1 * psi_m * dpsi_x - mu * mrel * psi_x * dpsi_m) / (mu1 * psi_m * dxi_x - mu * mrel * xi_x * dpsi_m)
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


def far_field(k, radius, n_rel, d, e, dirs, nmax=None, mu=1.0, mu1=1.0):
    """E_inf at unit directions dirs [D, 3] (not parallel to d) for the
    incident polarization e (unit, perpendicular to d)."""
    x = k * radius
    if nmax is None:
        nmax = int(x * abs(n_rel) + 4 * x ** (1 / 3) + 20)
    a, b = mie_coefficients(x, n_rel, nmax, mu, mu1)
    d = np.asarray(d, float)
    out = np.zeros((len(dirs), 3), dtype=complex)
    for i, xh in enumerate(np.asarray(dirs, float)):
        cth = float(np.dot(d, xh))
        S1, S2 = amplitudes(a, b, cth)
        ep = np.cross(d, xh)
        ep /= np.linalg.norm(ep)
        epi = np.cross(ep, d)
        eps_ = np.cross(ep, xh)
        out[i] = (1j / k) * (S2 * np.dot(e, epi) * eps_ + S1 * np.dot(e, ep) * ep)
    return out


def cross_sections(k, radius, n_rel, nmax=None, mu=1.0, mu1=1.0):
    """Extinction and scattering cross sections (2 pi / k^2) sum (2n+1) Re(a_n + b_n)
    and (2 pi / k^2) sum (2n+1)(|a_n|^2 + |b_n|^2)."""
    x = k * radius
    if nmax is None:
        nmax = int(x * abs(n_rel) + 4 * x ** (1 / 3) + 20)
    a, b = mie_coefficients(x, n_rel, nmax, mu, mu1)
    n = np.arange(1, nmax + 1)
    ext = 2 * np.pi / k ** 2 * np.sum((2 * n + 1) * np.real(a + b))
    sca = 2 * np.pi / k ** 2 * np.sum((2 * n + 1) * (np.abs(a) ** 2 + np.abs(b) ** 2))
    return ext, sca
