"""Seeded, synthetic inputs: incident plane waves and their azimuthal modes.

The plane wave of Section 6 (eq:pw): E = (d x p) x d exp(i k0 d.x) and
H = sqrt(eps0/mu0) (d x p) exp(i k0 d.x) (H as printed for eps0 = mu0 = 1,
scaled so that curl E = i omega mu0 H for any eps0, mu0).  The right-hand side
of the Mueller system is handed to the solver as azimuthal Fourier modes
f_m = (1/2pi) int f(theta) e^{-i m theta} d theta of the tangential traces, in
(t, e_theta) components at every node of the generating curve (Section 3):

    row 4j+0: i omega mu0 (n x H_inc)_t      row 4j+2: i omega eps0 (n x E_inc)_t
    row 4j+1: i omega mu0 (n x H_inc)_theta  row 4j+3: i omega eps0 (n x E_inc)_theta

with (n x V)_t = V_theta and (n x V)_theta = -(r' V_r + z' V_z).  Modes are
computed with an FFT of the sampled traces; this is input preparation, not
part of the method.

The extinction test of Section 6 instead prescribes the field of a current
loop (eq. loop): inside the body the field radiated with the interior
wavenumber k1 by a circular loop lying outside it, outside the body zero.
Its tangential traces are the data of the indirect system (eq. dualmullrep),
whose rows take them in the order

    row 4j+0, 4j+1: i omega eps0 (n x H_inc)    row 4j+2, 4j+3: i omega mu0 (n x E_inc).
"""
from __future__ import annotations

import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np


def paper_default_direction():
    """d and p at the angles used throughout Section 6 (eq. incidentdirection)."""
    th1, ph1, th2, ph2 = np.pi / 3, 2 * np.pi / 3, np.pi / 2, np.pi / 3
    d = np.array([np.cos(th1) * np.sin(ph1), np.sin(th1) * np.sin(ph1), np.cos(ph1)])
    p = np.array([np.cos(th2) * np.sin(ph2), np.sin(th2) * np.sin(ph2), np.cos(ph2)])
    return d, p


def tilted_direction(deg: float):
    """d at `deg` from +z in the x-z plane, p perpendicular to d in that plane."""
    a = np.deg2rad(deg)
    return np.array([np.sin(a), 0.0, np.cos(a)]), np.array([np.cos(a), 0.0, -np.sin(a)])


def random_directions(seed: int, count: int):
    """Directions uniform on S^2 (normalized Gaussians) and polarizations p with
    |p x d| >= 0.1 so that (d x p) x d never degenerates."""
    rng = np.random.default_rng(seed)
    out = []
    while len(out) < count:
        d = rng.standard_normal(3)
        d /= np.linalg.norm(d)
        p = rng.standard_normal(3)
        p /= np.linalg.norm(p)
        if np.linalg.norm(np.cross(d, p)) < 0.1:
            continue
        out.append((d, p))
    return out


def plane_wave(d, p, k0, eps0=1.0, mu0=1.0):
    """Callables E(x), H(x) for x of shape [..., 3]."""
    d = np.asarray(d, float)
    p = np.asarray(p, float)
    q = np.cross(d, p)
    e = np.cross(q, d)
    h = np.sqrt(eps0 / mu0) * q

    def ph(x):
        return np.exp(1j * k0 * (x @ d))[..., None]
    return (lambda x: e * ph(x)), (lambda x: h * ph(x))


def current_loop(center, radius, k, omega, mu, n_quad=None):
    """Callables E(x), H(x) of the loop field of eq. loop: with the vector
    potential A(x) = int_loop G^k(x, y) dl(y), G^k = e^{i k R}/(4 pi R),

        E = curl A = int grad_x G x dl,
        H = curl curl A / (i omega mu) = int [(grad grad G) dl + k^2 G dl] / (i omega mu),

    for the loop y(s) = center + radius (cos s, sin s, 0) in the plane z = z0,
    integrated with the trapezoid rule in s (spectrally accurate away from the
    loop).  k may be complex (Im k >= 0)."""
    c = np.asarray(center, float)
    a = float(radius)
    k = complex(k)
    if n_quad is None:
        # the integrand's bandwidth along the loop is about |k| a
        n_quad = 64 + 4 * int(np.ceil(abs(k) * a))
    s = 2 * np.pi * np.arange(n_quad) / n_quad
    ys = c[None, :] + a * np.stack([np.cos(s), np.sin(s), np.zeros_like(s)], axis=1)
    dl = (2 * np.pi / n_quad) * a * np.stack([-np.sin(s), np.cos(s), np.zeros_like(s)], axis=1)

    def parts(x):
        x = np.asarray(x, float)
        R = x[..., None, :] - ys  # [..., Q, 3]
        r = np.linalg.norm(R, axis=-1)
        G = np.exp(1j * k * r) / (4 * np.pi * r)
        return R, r, G

    def E(x):
        R, r, G = parts(x)
        gradG = (G * (1j * k - 1.0 / r) / r)[..., None] * R
        return np.cross(gradG, dl).sum(axis=-2)

    def H(x):
        R, r, G = parts(x)
        Rdl = np.einsum("...qc,qc->...q", R, dl)
        f1 = G * (3.0 - 3j * k * r - (k * r) ** 2) / r ** 4  # coefficient of R_a R_b
        f2 = G * (1j * k * r - 1.0) / r ** 2                # coefficient of delta_ab
        hess_dl = (f1 * Rdl)[..., None] * R + f2[..., None] * dl
        return (hess_dl + k * k * G[..., None] * dl).sum(axis=-2) / (1j * omega * mu)

    return E, H


def rhs_from_fields(curve, fields, coefs, m_lo, m_hi, n_theta):
    """Modes [m_hi - m_lo + 1, len(fields), 4N] of the tangential traces of
    field pairs: fields[w] = (E, H) callables; rows 4j, 4j+1 carry coefs[0]
    (n x H) and rows 4j+2, 4j+3 coefs[1] (n x E)."""
    N = curve.n
    th = 2 * np.pi * np.arange(n_theta) / n_theta
    ct, st = np.cos(th), np.sin(th)
    x = np.stack([curve.r[:, None] * ct[None, :], curve.r[:, None] * st[None, :],
                  np.broadcast_to(curve.z[:, None], (N, n_theta))], axis=-1)
    rp = -curve.nz  # r' = -n_z
    zp = curve.nr   # z' = n_r
    out = np.zeros((m_hi - m_lo + 1, len(fields), 4 * N), dtype=complex)
    ms = np.arange(m_lo, m_hi + 1)
    for w, (Ef, Hf) in enumerate(fields):
        for fld, base, coef in ((Hf, 0, coefs[0]), (Ef, 2, coefs[1])):
            # in node chunks: a field given by a quadrature (the loop) holds a
            # [points, quadrature nodes, 3] array per call
            with ThreadPoolExecutor(max_workers=min(16, os.cpu_count() or 1)) as pool:
                V = np.concatenate(list(pool.map(fld, [x[i:i + 16] for i in range(0, N, 16)])), axis=0)
            Vr = V[..., 0] * ct + V[..., 1] * st
            Vt = -V[..., 0] * st + V[..., 1] * ct
            Vz = V[..., 2]
            tr_t = Vt
            tr_th = -(rp[:, None] * Vr + zp[:, None] * Vz)
            for comp, tr in ((0, tr_t), (1, tr_th)):
                F = np.fft.fft(tr, axis=1) / n_theta  # F[k] = (1/L) sum f e^{-i k theta}
                out[:, w, 4 * np.arange(N) + base + comp] = coef * F[:, ms % n_theta].T
    return out


def rhs_modes(curve, waves, k0, m_lo, m_hi, eps0=1.0, mu0=1.0, n_theta=None):
    """Right-hand-side modes [m_hi - m_lo + 1, len(waves), 4N] (complex128) of
    plane waves for the direct system (eq. mullerrep)."""
    omega = k0 / np.sqrt(eps0 * mu0)
    rmax = float(np.max(curve.r))
    mmax = max(abs(m_lo), abs(m_hi))
    if n_theta is None:
        n_theta = 1 << int(np.ceil(np.log2(2 * (mmax + k0 * rmax) + 64)))
    fields = [plane_wave(d, p, k0, eps0, mu0) for d, p in waves]
    return rhs_from_fields(curve, fields, (1j * omega * mu0, 1j * omega * eps0), m_lo, m_hi, n_theta)


def loop_rhs_modes(curve, center, radius, k1, omega, mu1, m_lo, m_hi, eps0=1.0, mu0=1.0, n_theta=None):
    """Right-hand-side modes [m_hi - m_lo + 1, 1, 4N] of the current-loop data
    for the indirect system (eq. dualmullrep): the exterior field is zero, so
    the traces of the incident field equal those of the loop field."""
    c = np.asarray(center, float)
    rmax = float(np.max(curve.r))
    mmax = max(abs(m_lo), abs(m_hi))
    if n_theta is None:
        # the traces on a ring of radius r carry modes up to about |k1| r plus
        # the offset of the loop's axis from the body's; 32 modes of margin
        n_theta = 1 << int(np.ceil(np.log2(2 * (mmax + abs(k1) * rmax + 8 * np.hypot(c[0], c[1])) + 64)))
    E, H = current_loop(c, radius, k1, omega, mu1)
    return rhs_from_fields(curve, [(E, H)], (1j * omega * eps0, 1j * omega * mu0), m_lo, m_hi, n_theta)
