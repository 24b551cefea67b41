"""Near-panel quadrature rules for the 16th-order Nystrom-like discretization.

Section 5 ("Generalized Gaussian Quadrature", equations eq_nyslike and
eq_nyslike2 and the remark after them) discretizes the weakly singular modal
operators with precomputed rules: target-dependent support nodes on the panel
that holds the target, and one target-independent rule on each adjacent panel.
The paper takes these tables from third-party code; they are inputs to the
method, so they live here, beside the other input generators, and are handed
to both the oracle and the GPU library as plain arrays.

Two rules are built with the generalized-Gaussian-quadrature construction of
Bremer, Gimbutas and Rokhlin (2010): oversample a family of functions with a
composite Gauss-Legendre rule, compress it to an orthonormal basis with an SVD,
pick nodes by pivoted QR, then remove nodes one at a time with Gauss-Newton
until the rule can shrink no further.

* ``self`` rules, one per Gauss-Legendre target node ``x_i`` of the panel:
  ``NSELF`` nodes on [-1, 1] that integrate ``p(y) log|x_i - y| + q(y)``
  (deg p, q < 16) exactly -- the exactness of the paper's self-panel rules.
  Nodes are chosen from a composite rule graded toward ``x_i`` by pivoted QR
  on the family; the weights solve the moment equations with exact moments.
  Candidates closer than ``SELF_DMIN`` to ``x_i`` are left out: unconstrained,
  the selection takes pairs of nodes within 1e-9 of targets near the panel
  ends, with weights of opposite sign around 0.1.  The derivative kernels grow
  like 1/|x - y| there and cancel in the combinations the operators use, so
  those pairs multiply the kernels' rounding by sum |w| / |y - x| ~ 1e8.  With
  the bound the factor is at most 2e4 and the rules stay as accurate.
* ``adjacent`` rule on [-1, 1], accurate for ``P_j(y)`` and
  ``P_j(y) log|y - x|`` (j < 16) for every singular point ``x`` that a target on
  a neighbouring panel can produce: outside the panel, at distance
  ``delta in [DELTA_MIN, DELTA_MAX]`` (panel half-lengths) from either endpoint,
  at any angle up to a right-angle corner.  Neighbouring panels may differ in
  length by at most a factor of 2 (dyadic refinement).

Run ``python -m workloads.rules`` to regenerate ``workloads/data/rules_p16.txt``.
"""
from __future__ import annotations

import os

import mpmath
import numpy as np
from numpy.polynomial import legendre as npleg

ORDER = 16
DELTA_MIN = 0.004  # < (1 - x_16) * 1/2: nearest neighbour node, 2:1 refined neighbour
DELTA_MAX = 4.5    # > (1 + x_16) * 2: farthest neighbour node, 2:1 coarser neighbour
DATA = os.path.join(os.path.dirname(__file__), "data", "rules_p16.txt")


# ----------------------------------------------------------------------------
# function families
# ----------------------------------------------------------------------------
def _leg_all(x, n):
    """P_0..P_{n-1} and their derivatives at x (arrays [n, len(x)])."""
    x = np.asarray(x, dtype=float)
    P = np.zeros((n, x.size))
    dP = np.zeros((n, x.size))
    P[0] = 1.0
    if n > 1:
        P[1] = x
        dP[1] = 1.0
    for j in range(1, n - 1):
        P[j + 1] = ((2 * j + 1) * x * P[j] - j * P[j - 1]) / (j + 1)
        dP[j + 1] = dP[j - 1] + (2 * j + 1) * P[j]
    return P, dP


def _adjacent_points():
    """Singular points x (complex) whose log|y - x| the adjacent rule must integrate."""
    deltas = np.geomspace(DELTA_MIN, DELTA_MAX, 48)
    alphas = np.linspace(0.0, np.pi / 2, 7)
    pts = []
    for d in deltas:
        for a in alphas:
            pts.append(1.0 + d * np.exp(1j * a))
            pts.append(-1.0 - d * np.exp(1j * a))
    return np.array(pts)


def _adjacent_family(y, pts):
    P, dP = _leg_all(y, ORDER)
    rows, drows = [P], [dP]
    for x in pts:
        dy = y - x.real
        q = dy * dy + x.imag * x.imag
        lg = 0.5 * np.log(q)
        rows.append(P * lg)
        drows.append(dP * lg + P * (dy / q))
    return np.vstack(rows), np.vstack(drows)


# ----------------------------------------------------------------------------
# composite oversampling rules
# ----------------------------------------------------------------------------
def _graded(a, b, levels, npts, both_ends):
    """Composite Gauss-Legendre rule on [a, b] graded dyadically toward a (and b)."""
    x0, w0 = npleg.leggauss(npts)
    cuts = [0.0]
    for lv in range(levels, 0, -1):
        cuts.append(2.0 ** (-lv))
    cuts.append(1.0)
    cuts = np.array(cuts)
    if both_ends:
        half = 0.5 * cuts
        cuts = np.concatenate([half, 1.0 - half[::-1][1:]])
    xs, ws = [], []
    for lo, hi in zip(cuts[:-1], cuts[1:]):
        xs.append(a + (b - a) * (lo + (hi - lo) * (x0 + 1) / 2))
        ws.append((b - a) * (hi - lo) / 2 * w0)
    return np.concatenate(xs), np.concatenate(ws)


# ----------------------------------------------------------------------------
# compression: SVD basis + pivoted QR nodes + Gauss-Newton node elimination
# ----------------------------------------------------------------------------
def _qr_select(B, r):
    """Greedy column-pivoted QR on B (r x K): indices of r columns."""
    A = B.copy()
    K = A.shape[1]
    piv = []
    norms = np.sum(A * A, axis=0)
    for _ in range(r):
        j = int(np.argmax(norms))
        piv.append(j)
        v = A[:, j] / np.sqrt(norms[j])
        A -= np.outer(v, v @ A)
        norms = np.sum(A * A, axis=0)
        norms[piv] = -1.0
    return np.array(sorted(piv))


class _Basis:
    """A well-conditioned set of r family members spanning the whole family.

    An SVD of the oversampled family gives its numerical rank r; column-pivoted
    QR on the (weighted) family matrix then picks r members whose span holds the
    rest.  Those members are evaluated directly (never through a combination
    with large coefficients), and their moments come from the oversampled rule
    unless exact ones are supplied.
    """

    def __init__(self, family, xo, wo, tol, exact_moments=None):
        self.family = family
        F, _ = family(xo)
        A = F * np.sqrt(wo)[None, :]
        U, s, Vt = np.linalg.svd(A, full_matrices=False)
        r = int(np.sum(s > tol * s[0]))
        self.r = r
        self.Vt = Vt[:r]
        rows = _qr_select((A / np.linalg.norm(A, axis=1)[:, None]).T.copy(), r)
        self.rows = rows
        self.scale = 1.0 / np.linalg.norm(A[rows], axis=1)
        mom = F[rows] @ wo if exact_moments is None else exact_moments[rows]
        self.moments = mom * self.scale

    def eval(self, x):
        F, dF = self.family(x)
        return F[self.rows] * self.scale[:, None], dF[self.rows] * self.scale[:, None]


def _gauss_newton(basis, x, w, to_v, from_v, dxdv, tol, iters=80):
    """Gauss-Newton (minimal-norm steps) on the moment equations.

    Nodes move in a variable v with x = from_v(v) so that they can never leave
    the interval and the Jacobian stays well scaled near a singular endpoint.
    """
    v = to_v(x)
    for _ in range(iters):
        x = from_v(v)
        B, dB = basis.eval(x)
        res = B @ w - basis.moments
        rn = np.linalg.norm(res)
        if np.max(np.abs(res)) < 0.25 * tol:
            return x, w, True
        J = np.hstack([B, dB * (w * dxdv(x))[None, :]])
        cs = np.linalg.norm(J, axis=0)
        cs[cs == 0] = 1.0
        step = np.linalg.lstsq(J / cs[None, :], res, rcond=None)[0] / cs
        n = w.size
        t = 1.0
        for _ in range(40):
            vn = v - t * step[n:]
            wn = w - t * step[:n]
            xn = from_v(vn)
            if np.all(np.isfinite(xn)):
                Bn, _ = basis.eval(xn)
                if np.linalg.norm(Bn @ wn - basis.moments) < rn:
                    break
            t *= 0.5
        else:
            break
        v, w = vn, wn
    x = from_v(v)
    B, _ = basis.eval(x)
    return x, w, np.max(np.abs(B @ w - basis.moments)) < tol


def _compress(basis, xo, wo, param, target, tol):
    to_v, from_v, dxdv = param
    idx = _qr_select(basis.Vt, basis.r)
    x = xo[idx]
    B, _ = basis.eval(x)
    w = np.linalg.solve(B, basis.moments)
    while x.size > target:
        B, _ = basis.eval(x)
        signif = np.abs(w) * np.sqrt(np.sum(B * B, axis=0))
        order = np.argsort(signif)
        done = False
        for cand in order[:12]:
            keep = np.ones(x.size, bool)
            keep[cand] = False
            xn, wn, ok = _gauss_newton(basis, x[keep].copy(), w[keep].copy(),
                                       to_v, from_v, dxdv, tol)
            if ok:
                x, w, done = xn, wn, True
                break
        if not done:
            break
    srt = np.argsort(x)
    return x[srt], w[srt]


_TANH_PARAM = (np.arctanh, np.tanh, lambda x: 1.0 - x * x)


NSELF = 2 * ORDER
SELF_DMIN = 1e-5  # smallest |y - x| of a self-rule node (panel coordinate)


def _self_family(y, x):
    P, dP = _leg_all(y, ORDER)
    d = y - x
    lg = np.log(np.abs(d))
    return np.vstack([P, P * lg]), np.vstack([dP, dP * lg + P / d])


def _self_moments(x):
    """Exact int_{-1}^{1} P_j(y) dy and int_{-1}^{1} P_j(y) log|y - x| dy."""
    mpmath.mp.dps = 32
    mom = np.zeros(2 * ORDER)
    mom[0] = 2.0
    xm = mpmath.mpf(x)
    for j in range(ORDER):
        f = lambda y, j=j: mpmath.legendre(j, y) * mpmath.log(abs(y - xm))
        mom[ORDER + j] = float(mpmath.quad(f, [-1, xm]) + mpmath.quad(f, [xm, 1]))
    return mom


def build_self_rules():
    """[ORDER, NSELF] nodes and weights on [-1, 1], one rule per GL target node."""
    xg, _ = npleg.leggauss(ORDER)
    xa, wa = _graded(0.0, 1.0, 20, 20, both_ends=False)
    nodes = np.zeros((ORDER, NSELF))
    weights = np.zeros((ORDER, NSELF))
    for i, x in enumerate(xg):
        xo = np.concatenate([x - (x + 1) * xa, x + (1 - x) * xa])
        wo = np.concatenate([(x + 1) * wa, (1 - x) * wa])
        keep = np.abs(xo - x) >= SELF_DMIN
        xo, wo = xo[keep], wo[keep]
        F, _ = _self_family(xo, x)
        A = F * np.sqrt(wo)[None, :]
        A /= np.linalg.norm(A, axis=1)[:, None]
        Vt = np.linalg.svd(A, full_matrices=False)[2][:NSELF]
        idx = _qr_select(Vt, NSELF)
        y = xo[idx]
        B, _ = _self_family(y, x)
        mom = _self_moments(x)
        w = np.linalg.solve(B, mom)
        # refine the weights: residual of the moment equations in extended
        # precision, so that the rule is exact to the moments' own rounding
        yl, xl = y.astype(np.longdouble), np.longdouble(x)
        P = np.zeros((ORDER, y.size), dtype=np.longdouble)
        P[0] = 1
        P[1] = yl
        for j in range(1, ORDER - 1):
            P[j + 1] = ((2 * j + 1) * yl * P[j] - j * P[j - 1]) / (j + 1)
        Bl = np.vstack([P, P * np.log(np.abs(yl - xl))])
        for _ in range(2):
            res = mom.astype(np.longdouble) - Bl @ w.astype(np.longdouble)
            w = w + np.linalg.solve(B, res.astype(np.float64))
        srt = np.argsort(y)
        nodes[i], weights[i] = y[srt], w[srt]
    # the node set is symmetric under y -> -y; keep, for each mirror pair of
    # targets, the rule with the smaller sum |w| and reflect it onto the other
    for i in range(ORDER // 2):
        j = ORDER - 1 - i
        if np.abs(weights[j]).sum() < np.abs(weights[i]).sum():
            nodes[i], weights[i] = -nodes[j][::-1], weights[j][::-1]
        nodes[j], weights[j] = -nodes[i][::-1], weights[i][::-1]
    return nodes, weights


def build_adjacent_rule(target=None):
    pts = _adjacent_points()
    fam = lambda y: _adjacent_family(y, pts)
    xo, wo = _graded(-1.0, 1.0, 14, 20, both_ends=True)
    basis = _Basis(fam, xo, wo, 1e-15)
    if target is None:
        target = basis.r
    return _compress(basis, xo, wo, _TANH_PARAM, target, 1e-13)


def write_rules(path=DATA):
    ys, ws = build_self_rules()
    ya, wa = build_adjacent_rule()
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w") as f:
        f.write("# near-panel quadrature rules, order 16 (generated by workloads/rules.py)\n")
        f.write(f"self {ORDER} {ys.shape[1]}\n")
        for i in range(ORDER):
            for y, w in zip(ys[i], ws[i]):
                f.write(f"{y:.17e} {w:.17e}\n")
        f.write(f"adjacent {ya.size}\n")
        for y, w in zip(ya, wa):
            f.write(f"{y:.17e} {w:.17e}\n")


def load_rules(path=DATA):
    """(self nodes [16, ns], self weights [16, ns]), (adjacent nodes [na], weights [na])."""
    with open(path) as f:
        lines = [ln for ln in f if not ln.startswith("#")]
    hdr = lines[0].split()
    nt, ns = int(hdr[1]), int(hdr[2])
    arr = np.array([[float(v) for v in ln.split()] for ln in lines[1:1 + nt * ns]])
    ys = arr[:, 0].reshape(nt, ns)
    ws = arr[:, 1].reshape(nt, ns)
    na = int(lines[1 + nt * ns].split()[1])
    arr = np.array([[float(v) for v in ln.split()] for ln in lines[2 + nt * ns:2 + nt * ns + na]])
    return (ys, ws), (arr[:, 0].copy(), arr[:, 1].copy())


if __name__ == "__main__":
    write_rules()
    (ys, ws), (ya, wa) = load_rules()
    print("self nodes", ys.shape, "adjacent nodes", ya.size)
