"""Panels, near-panel support points and interpolation (Section 5).

Nodes are panel-major: node j = ORDER * panel + k sits at the k-th Gauss-
Legendre point u_k of the panel's local coordinate u in [-1, 1].  For each
target node the near panels are its own panel and the panels sharing an
endpoint with it (wrapping around for a closed curve).  Integrals over a near
panel use the support nodes of the near-panel rules (eq. eq_nyslike):

    int_panel g(x_t, y) psi(y) ds ~= sum_q W_q (ds/du)(y_q) g(x_t, y_q) psi(y_q),
    psi(y_q) = sum_k l_k(y_q) psi(x_k)                       (eq. eq_nyslike2)

with l_k the Lagrange basis on the panel's Gauss-Legendre nodes (the transform
matrix U of eq_nyslike2 composed with the Legendre series).  The geometry at a
support node -- r, z and dr/du, dz/du -- is the degree-15 interpolant of the
nodal values, so that only nodal data are needed.  The offset of a support
node from its target, (r_s - r_t, z_s - z_t), is interpolated from the nodal
differences r_k - r_t rather than formed by subtracting interpolated
coordinates: self-panel support nodes lie as close as 1e-10 panel lengths to
the target, and the subtraction would leave only a few correct digits of the
distance that the log-singular kernels depend on.  On the target's own panel
the offset is written (y - u_t) Q(y), with Q the degree-14 interpolant, on the
other 15 nodes, of the divided differences (r_k - r_t)/(u_k - u_t): the same
polynomial, without the cancellation of summing O(1) terms into a tiny one.
Offsets are evaluated in x87 extended precision (numpy longdouble): near the
axis a support node can differ from its target mostly in r, and the small z
offset (which the z-derivative kernels are proportional to) would otherwise
keep only about 12 correct digits.  The interpolation nodes are the Gauss-
Legendre nodes rounded to double (refined in longdouble by Newton's method,
then rounded), so that y - u_t, as small as 1e-10, is exact.

Support slots per target: [0, NS) on its own panel, then NA on the left
neighbour, then NA on the right neighbour; missing neighbours (ends of an open
curve) leave their slots unused (weight 0).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
from numpy.polynomial import legendre as npleg


def bary_weights(x):
    n = x.size
    w = np.ones(n)
    for j in range(n):
        for k in range(n):
            if k != j:
                w[j] /= (x[j] - x[k])
    return w


def lagrange_matrix(xn, y):
    """l_k(y_q) for nodes xn (n) and points y (m): [m, n] (barycentric form)."""
    bw = bary_weights(xn)
    diff = y[:, None] - xn[None, :]
    exact = diff == 0.0
    diff[exact] = 1.0
    t = bw[None, :] / diff
    L = t / t.sum(axis=1, keepdims=True)
    rows = np.nonzero(exact.any(axis=1))[0]
    for r in rows:
        L[r] = exact[r].astype(float)
    return L


def gl_nodes_ext(order):
    """Gauss-Legendre nodes rounded to double, returned as longdouble (Newton on
    P_order in longdouble from numpy's nodes, which can be off by an ulp)."""
    x = npleg.leggauss(order)[0].astype(np.longdouble)
    for _ in range(4):
        p0, p1 = np.ones_like(x), x.copy()
        for k in range(2, order + 1):
            p0, p1 = p1, ((2 * k - 1) * x * p1 - (k - 1) * p0) / k
        dp = order * (x * p1 - p0) / (x * x - 1)
        x = x - p1 / dp
    return x.astype(np.float64).astype(np.longdouble)


def lagrange_matrix_ext(xn, y):
    """lagrange_matrix in longdouble (first barycentric form, y not a node)."""
    xn = np.asarray(xn, dtype=np.longdouble)
    y = np.asarray(y, dtype=np.longdouble)
    n = xn.size
    bw = np.ones(n, dtype=np.longdouble)
    for j in range(n):
        for k in range(n):
            if k != j:
                bw[j] /= (xn[j] - xn[k])
    diff = y[:, None] - xn[None, :]
    assert not np.any(diff == 0)
    ell = np.prod(diff, axis=1)
    return ell[:, None] * bw[None, :] / diff


@dataclass
class Support:
    r: np.ndarray      # [N, S]
    z: np.ndarray
    dr: np.ndarray     # r_s - r_t, z_s - z_t from interpolated nodal differences
    dz: np.ndarray
    tr: np.ndarray     # unit tangent components r', z'
    tz: np.ndarray
    wq: np.ndarray     # W_q * ds/du at the support node (0 = unused slot)
    panel: np.ndarray  # [N, S] panel index of the support node (-1 unused)
    lag: np.ndarray    # [N, S, ORDER] Lagrange values l_k(y_q)


def neighbours(n_panels, closed):
    left = np.arange(n_panels) - 1
    right = np.arange(n_panels) + 1
    if closed:
        left[0] = n_panels - 1
        right[-1] = 0
    else:
        left[0] = -1
        right[-1] = -1
    return left, right


def support_points(curve, self_rules, adj_rule):
    """Support-node geometry, weights and interpolation for every target."""
    order = curve.order
    ugx = gl_nodes_ext(order)
    ug = ugx.astype(np.float64)
    ys, ws = self_rules
    ya, wa = adj_rule
    NS, NA = ys.shape[1], ya.size
    S = NS + 2 * NA
    N = curve.n
    npan = curve.n_panels
    left, right = neighbours(npan, curve.closed)
    # nodal r, z, dr/du, dz/du per panel
    rp = curve.r.reshape(npan, order)
    zp = curve.z.reshape(npan, order)
    drp = (-curve.nz * curve.dsdu).reshape(npan, order)
    dzp = (curve.nr * curve.dsdu).reshape(npan, order)
    out = {k: np.zeros((N, S)) for k in ("r", "z", "dr", "dz", "tr", "tz", "wq")}
    panel = -np.ones((N, S), dtype=int)
    lag = np.zeros((N, S, order))

    def fill(t, slot0, p, y, w):
        Lm = lagrange_matrix(ug, y)
        r = Lm @ rp[p]
        z = Lm @ zp[p]
        dr = Lm @ drp[p]
        dz = Lm @ dzp[p]
        sp = np.hypot(dr, dz)
        sl = slice(slot0, slot0 + y.size)
        out["r"][t, sl] = r
        out["z"][t, sl] = z
        ld = lambda a: np.asarray(a, dtype=np.longdouble)
        rt, zt = ld(curve.r[t]), ld(curve.z[t])
        if p == t // order:  # own panel: divided differences
            kt = t % order
            keep = np.arange(order) != kt
            L15 = lagrange_matrix_ext(ugx[keep], y)
            du = ugx[keep] - ugx[kt]
            yu = ld(y) - ugx[kt]
            out["dr"][t, sl] = (yu * (L15 @ ((ld(rp[p][keep]) - rt) / du))).astype(np.float64)
            out["dz"][t, sl] = (yu * (L15 @ ((ld(zp[p][keep]) - zt) / du))).astype(np.float64)
        else:
            Lx = lagrange_matrix_ext(ugx, y)
            out["dr"][t, sl] = (Lx @ (ld(rp[p]) - rt)).astype(np.float64)
            out["dz"][t, sl] = (Lx @ (ld(zp[p]) - zt)).astype(np.float64)
        out["tr"][t, sl] = dr / sp
        out["tz"][t, sl] = dz / sp
        out["wq"][t, sl] = w * sp
        panel[t, sl] = p
        lag[t, sl] = Lm

    for t in range(N):
        p, k = divmod(t, order)
        fill(t, 0, p, ys[k], ws[k])
        if left[p] >= 0:
            fill(t, NS, left[p], ya, wa)
        if right[p] >= 0:
            fill(t, NS + NA, right[p], ya, wa)
    return Support(out["r"], out["z"], out["dr"], out["dz"], out["tr"], out["tz"], out["wq"],
                   panel, lag)


def near_mask(curve):
    """[N, N] True where the source node lies on a near panel of the target."""
    order = curve.order
    npan = curve.n_panels
    left, right = neighbours(npan, curve.closed)
    pt = np.arange(curve.n) // order
    ps = np.arange(curve.n) // order
    m = ps[None, :] == pt[:, None]
    lt = left[pt]
    rt = right[pt]
    m |= ps[None, :] == lt[:, None]
    m |= ps[None, :] == rt[:, None]
    return m
