"""Electric and magnetic fields off the surface from the surface currents.

Test infrastructure: a plain quadrature of the field representations of
Section 2, used only to check the GPU path.

For x in the exterior region (eq. exteriorfield)

    E = -(1/(i w eps0)) curl curl S^{k0} J + curl S^{k0} M,
    H =  (1/(i w mu0))  curl curl S^{k0} M + curl S^{k0} J,

for x in the interior with the currents of the direct system (eq. interiorfield)

    E =  (1/(i w eps1)) curl curl S^{k1} J - curl S^{k1} M,
    H = -(1/(i w mu1))  curl curl S^{k1} M - curl S^{k1} J,

and with those of the indirect system (eq. interior_dual)

    E = -(1/(i w eps0)) curl curl S^{k1} J + (mu1/mu0) curl S^{k1} M,
    H =  (1/(i w mu0))  curl curl S^{k1} M + (eps1/eps0) curl S^{k1} J,

where S^k V(x) = int_Gamma G^k(x, y) V(y) da(y), G^k = e^{i k R}/(4 pi R),
R = |x - y|.  With grad_x G = G (i k - 1/R) R_vec/R and the Hessian
d_a d_b G = G [(3 - 3 i k R - k^2 R^2) R_a R_b/R^4 + (i k R - 1) delta_ab/R^2]:

    curl S V       = int grad_x G x V da,
    curl curl S V  = int [(grad grad G) V + k^2 G V] da      (curl curl = grad div - Laplacian).

The currents are synthesized from their modes on a surface grid (trapezoid
rule in theta, the Gauss-Legendre arclength weights along the generating
curve), as for the far field.  The rule along the curve loses accuracy for
points whose distance to the surface is small against the panels; with
upsample = U each panel's currents, dr/du and dz/du are first interpolated
(Legendre interpolation in the panel coordinate u) to U sub-panels of 16
Gauss-Legendre nodes each.
"""
from __future__ import annotations

import numpy as np


def upsample_panels(curve, x_modes, U):
    """Nodes (r, z, r', z', arclength weight) and current modes [n_modes, 4 N U]
    at U sub-panels of 16 Gauss-Legendre nodes per panel, interpolated from the
    panel's 16 nodes: sub-panel q spans u in [-1 + 2q/U, -1 + 2(q+1)/U]."""
    from numpy.polynomial import legendre as npleg

    from .discretize import lagrange_matrix
    order = curve.order
    ug, wg = npleg.leggauss(order)
    uf = np.concatenate([-1.0 + (2 * q + ug + 1.0) / U for q in range(U)])
    wf = np.tile(wg, U) / U
    Lm = lagrange_matrix(ug, uf)  # [16 U, 16]
    npan = curve.n_panels
    nm = x_modes.shape[0]
    dru = -curve.nz * curve.dsdu  # dr/du = r' ds/du
    dzu = curve.nr * curve.dsdu
    panel = lambda a: (Lm @ a.reshape(npan, order).T).T.reshape(-1)
    r, z, ru, zu = panel(curve.r), panel(curve.z), panel(dru), panel(dzu)
    sp = np.hypot(ru, zu)
    w = np.tile(wf, npan) * sp
    X = x_modes.reshape(nm, npan, order, 4)
    Xf = np.einsum("fj,mpjc->mpfc", Lm, X).reshape(nm, -1)
    return r, z, ru / sp, zu / sp, w, Xf


def surface_grid(geom, x_modes, m_lo, n_theta):
    """Points y [N, T, 3], area weights da [N, T] and the currents J, M [N, T, 3]
    of one right-hand side, x_modes [n_modes, 4N] for modes m_lo..; geom =
    (r, z, r', z', arclength weights) of the N nodes."""
    gr, gz, tr, tz, w = geom
    N = gr.size
    nm = x_modes.shape[0]
    ms = np.arange(m_lo, m_lo + nm)
    th = 2 * np.pi * np.arange(n_theta) / n_theta
    ph = np.exp(1j * np.outer(ms, th))  # [nm, T]
    X = x_modes.reshape(nm, N, 4)
    comps = np.einsum("mnc,mt->nct", X, ph)  # [N, 4, T]
    ct, st = np.cos(th), np.sin(th)

    def vec(a1, a2):
        # a1 t + a2 e_theta with t = r' e_r + z' e_z
        vx = a1 * tr[:, None] * ct - a2 * st
        vy = a1 * tr[:, None] * st + a2 * ct
        vz = a1 * tz[:, None]
        return np.stack([vx, vy, vz], axis=-1)

    J = vec(comps[:, 0], comps[:, 1])
    M = vec(comps[:, 2], comps[:, 3])
    y = np.stack([gr[:, None] * ct, gr[:, None] * st,
                  np.broadcast_to(gz[:, None], (N, n_theta))], axis=-1)
    da = (w * gr)[:, None] * (2 * np.pi / n_theta) * np.ones((1, n_theta))
    return y, da, J, M


def potentials(x, y, da, V, k):
    """curl S^k V and curl curl S^k V at one point x [3] (sums over the grid)."""
    R = x[None, None, :] - y
    r = np.linalg.norm(R, axis=-1)
    G = np.exp(1j * k * r) / (4 * np.pi * r) * da
    gradG = (G * (1j * k - 1.0 / r) / r)[..., None] * R
    curl = np.cross(gradG, V).sum(axis=(0, 1))
    RV = np.einsum("ntc,ntc->nt", R, V)
    f1 = G * (3.0 - 3j * k * r - (k * r) ** 2) / r ** 4
    f2 = G * (1j * k * r - 1.0) / r ** 2
    cc = ((f1 * RV)[..., None] * R + (f2 + k * k * G)[..., None] * V).sum(axis=(0, 1))
    return curl, cc


def fields(curve, w, x_modes, m_lo, points, k0, k1, omega, eps0, mu0, eps1, mu1, region,
           formulation="direct", n_theta=None, upsample=1):
    """E, H [P, 3] at points [P, 3] lying in `region` ("exterior" or
    "interior") from the currents of one right-hand side."""
    nm = x_modes.shape[0]
    mmax = max(abs(m_lo), abs(m_lo + nm - 1))
    k = k0 if region == "exterior" else k1
    if n_theta is None:
        n_theta = int(4 * (mmax + abs(k) * float(curve.r.max())) + 128)
    if upsample > 1:
        *geom, xs = upsample_panels(curve, x_modes, upsample)
    else:
        geom, xs = (curve.r, curve.z, -curve.nz, curve.nr, w), x_modes
    y, da, J, M = surface_grid(geom, xs, m_lo, n_theta)
    iw = 1j * omega
    E = np.zeros((len(points), 3), dtype=complex)
    H = np.zeros_like(E)
    for i, x in enumerate(np.asarray(points, float)):
        cJ, ccJ = potentials(x, y, da, J, k)
        cM, ccM = potentials(x, y, da, M, k)
        if region == "exterior":
            E[i] = -ccJ / (iw * eps0) + cM
            H[i] = ccM / (iw * mu0) + cJ
        elif formulation == "direct":
            E[i] = ccJ / (iw * eps1) - cM
            H[i] = -ccM / (iw * mu1) - cJ
        elif formulation == "indirect":
            E[i] = -ccJ / (iw * eps0) + (mu1 / mu0) * cM
            H[i] = ccM / (iw * mu0) + (eps1 / eps0) * cJ
        else:
            raise ValueError(formulation)
    return E, H
