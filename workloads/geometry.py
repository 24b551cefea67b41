"""Seeded, synthetic inputs: discretized generating curves.

A generating curve gamma(t) = (r(t), z(t)) is cut into panels; each panel is
the image of the local coordinate u in [-1, 1] and carries ORDER Gauss-Legendre
nodes in u (Section 5, panel discretization; remark in Section 6 on sampling in
a parameter other than arclength).  Per node we keep r, z, the outward unit
normal n = (z', -r') (Section 3, with ' the arclength derivative and the curve
traversed counterclockwise, open curves from the south pole to the north
pole), and the speed ds/du.  The arclength weight of node k of a panel is the
Gauss-Legendre weight times ds/du.  Nothing here evaluates the method; it only
describes bodies.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
from numpy.polynomial import legendre as npleg

ORDER = 16


@dataclass
class Curve:
    name: str
    n_panels: int
    closed: bool
    r: np.ndarray
    z: np.ndarray
    nr: np.ndarray
    nz: np.ndarray
    dsdu: np.ndarray
    panel_len: np.ndarray  # arclength of each panel
    order: int = ORDER
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return self.r.size

    def arrays(self):
        return self.r, self.z, self.nr, self.nz, self.dsdu


def _from_panels(name, panels, closed, meta=None):
    """panels: list of (t_a, t_b, f) with f(t) -> (r, z, dr/dt, dz/dt)."""
    ug, _ = npleg.leggauss(ORDER)
    ug_fine, wg_fine = npleg.leggauss(40)
    R, Z, NR, NZ, DS, PL = [], [], [], [], [], []
    for ta, tb, f in panels:
        t = ta + (ug + 1) * (tb - ta) / 2
        r, z, dr, dz = f(t)
        sp = np.hypot(dr, dz)
        R.append(r)
        Z.append(z)
        NR.append(dz / sp)
        NZ.append(-dr / sp)
        DS.append(sp * (tb - ta) / 2)
        tf = ta + (ug_fine + 1) * (tb - ta) / 2
        _, _, drf, dzf = f(tf)
        PL.append(np.sum(wg_fine * np.hypot(drf, dzf)) * (tb - ta) / 2)
    cat = np.concatenate
    return Curve(name, len(panels), closed, cat(R), cat(Z), cat(NR), cat(NZ), cat(DS),
                 np.array(PL), meta=meta or {})


def spheroid(n_panels: int, c: float = 1.0, name: str | None = None,
             pole_levels: int = 0) -> Curve:
    """r = sin t, z = -c cos t, t in [0, pi]: c = 1 is the unit sphere.

    pole_levels > 0 refines the two pole panels dyadically toward the axis, where
    the 1/r and 1/r^2 factors of the modal operators amplify quadrature error.
    """
    f = lambda t: (np.sin(t), -c * np.cos(t), np.cos(t), c * np.sin(t))
    edges = np.linspace(0.0, np.pi, n_panels + 1)
    cuts = []
    for i, (a, b) in enumerate(zip(edges[:-1], edges[1:])):
        if pole_levels and i == 0:
            cuts.append(_dyadic(a, b, pole_levels, toward_b=False))
        elif pole_levels and i == n_panels - 1:
            cuts.append(_dyadic(a, b, pole_levels, toward_b=True))
        else:
            cuts.append(np.array([a, b]))
    panels = [(lo, hi, f) for cc in cuts for lo, hi in zip(cc[:-1], cc[1:])]
    return _from_panels(name or ("sphere" if c == 1.0 else f"spheroid_c{c:g}"), panels, False,
                        {"kind": "spheroid", "c": c, "pole_levels": pole_levels})


def sphere(n_panels: int = 8, pole_levels: int = 0) -> Curve:
    return spheroid(n_panels, 1.0, pole_levels=pole_levels)


def torus(n_panels: int, R0: float = 2.0, a: float = 1.0, b: float = 0.5) -> Curve:
    """r = R0 + a cos t, z = b sin t, t in [0, 2 pi): the torus of Example 1."""
    f = lambda t: (R0 + a * np.cos(t), b * np.sin(t), -a * np.sin(t), b * np.cos(t))
    edges = np.linspace(0.0, 2 * np.pi, n_panels + 1)
    panels = [(a_, b_, f) for a_, b_ in zip(edges[:-1], edges[1:])]
    return _from_panels("torus", panels, True, {"kind": "torus"})


def starfish(n_panels: int) -> Curve:
    """The rotated starfish of Example 2: r = rho cos(pi (t - 1/2)),
    z = rho sin(pi (t - 1/2)), rho = 2 + cos(5 pi (t - 1))/2, t in [0, 1]
    (pole to pole), equal panels in t."""
    def f(t):
        rho = 2.0 + 0.5 * np.cos(5 * np.pi * (t - 1.0))
        drho = -2.5 * np.pi * np.sin(5 * np.pi * (t - 1.0))
        ph = np.pi * (t - 0.5)
        c, s = np.cos(ph), np.sin(ph)
        return rho * c, rho * s, drho * c - np.pi * rho * s, drho * s + np.pi * rho * c
    edges = np.linspace(0.0, 1.0, n_panels + 1)
    panels = [(a_, b_, f) for a_, b_ in zip(edges[:-1], edges[1:])]
    return _from_panels("starfish", panels, False, {"kind": "starfish"})


def droplet(n_panels: int, tip_levels: int = 5) -> Curve:
    """The droplet of Example 3: r = sin(pi t) cos(pi (t - 3/2)/2),
    z = sin(pi t) sin(pi (t - 3/2)/2) + 1/2, t in [1/2, 1] (pole to pole), with
    a conical point on the axis at t = 1.  n_panels - tip_levels equal panels
    in t, the one ending at t = 1 refined dyadically tip_levels times toward it."""
    def f(t):
        s, c = np.sin(np.pi * t), np.cos(np.pi * t)
        a = 0.5 * np.pi * (t - 1.5)
        sa, ca = np.sin(a), np.cos(a)
        return (s * ca, s * sa + 0.5, np.pi * c * ca - 0.5 * np.pi * s * sa,
                np.pi * c * sa + 0.5 * np.pi * s * ca)
    nb = n_panels - tip_levels
    if nb < 1:
        raise ValueError("droplet needs more panels than tip levels")
    edges = np.linspace(0.5, 1.0, nb + 1)
    cuts = np.concatenate([edges[:-1], _dyadic(edges[-2], 1.0, tip_levels, True)[1:]])
    panels = [(lo, hi, f) for lo, hi in zip(cuts[:-1], cuts[1:])]
    return _from_panels("droplet", panels, False, {"kind": "droplet", "tip_levels": tip_levels})


def _segment(p0, p1):
    p0 = np.asarray(p0, float)
    p1 = np.asarray(p1, float)
    d = p1 - p0

    def f(t):
        return (p0[0] + t * d[0], p0[1] + t * d[1],
                np.full_like(t, d[0]), np.full_like(t, d[1]))
    return f


def _dyadic(a, b, levels, toward_b):
    """Split [a, b] dyadically `levels` times toward one end."""
    cuts = [a, b]
    lo, hi = a, b
    for _ in range(levels):
        mid = 0.5 * (lo + hi)
        cuts.append(mid)
        if toward_b:
            lo = mid
        else:
            hi = mid
    return np.array(sorted(cuts))


def polygon(vertices, panels_per_unit: float, corner_levels: int, name: str) -> Curve:
    """Open polygonal generating curve with both ends on the axis.

    Each segment gets equal base panels; the base panels touching an interior
    vertex (a corner of the body) are refined dyadically `corner_levels` times
    toward it (Section 5, dyadic refinement at corners).
    """
    panels = []
    nv = len(vertices)
    for s in range(nv - 1):
        p0, p1 = vertices[s], vertices[s + 1]
        length = float(np.hypot(p1[0] - p0[0], p1[1] - p0[1]))
        nb = max(1, int(round(length * panels_per_unit)))
        edges = np.linspace(0.0, 1.0, nb + 1)
        f = _segment(p0, p1)
        for i in range(nb):
            a, b = edges[i], edges[i + 1]
            at_start = (i == 0) and s > 0
            at_end = (i == nb - 1) and s < nv - 2
            if at_end and corner_levels:
                cuts = _dyadic(a, b, corner_levels, toward_b=True)
            elif at_start and corner_levels:
                cuts = _dyadic(a, b, corner_levels, toward_b=False)
            else:
                cuts = np.array([a, b])
            for lo, hi in zip(cuts[:-1], cuts[1:]):
                panels.append((lo, hi, f))
    return _from_panels(name, panels, False, {"kind": "polygon", "vertices": vertices})


def cylinder(corner_levels: int = 24, panels_per_unit: float = 8.0) -> Curve:
    """Cylinder of radius 1, height 2 (vertices of Example 4), base panels of
    length about 1/panels_per_unit (32 of 0.125 by default), the four
    corner-adjacent base panels refined toward the edges."""
    v = [(0.0, -1.0), (1.0, -1.0), (1.0, 1.0), (0.0, 1.0)]
    return polygon(v, panels_per_unit, corner_levels, "cylinder")


def random_body(rng: np.random.Generator, n_panels: int, tip_levels: int = 0) -> Curve:
    """Fourier-perturbed spheroid r = R(t) sin t, z = -c R(t) cos t with
    R = 1 + sum_j a_j cos(j t); optionally a conical north tip refined dyadically."""
    while True:
        a = rng.uniform(-0.15, 0.15, 6) / np.arange(1, 7)
        tt = np.linspace(0, np.pi, 2001)
        Rt = 1 + sum(a[j] * np.cos((j + 1) * tt) for j in range(6))
        if Rt.min() >= 0.5:
            break
    c = rng.uniform(0.5, 2.0)
    js = np.arange(1, 7)

    def f(t):
        t = np.asarray(t, float)
        Rv = 1 + np.sum(a[:, None] * np.cos(js[:, None] * t[None, :]), axis=0)
        dR = -np.sum(a[:, None] * js[:, None] * np.sin(js[:, None] * t[None, :]), axis=0)
        r = Rv * np.sin(t)
        z = -c * Rv * np.cos(t)
        dr = dR * np.sin(t) + Rv * np.cos(t)
        dz = -c * (dR * np.cos(t) - Rv * np.sin(t))
        return r, z, dr, dz
    if tip_levels == 0:
        edges = np.linspace(0.0, np.pi, n_panels + 1)
        panels = [(x0, x1, f) for x0, x1 in zip(edges[:-1], edges[1:])]
        return _from_panels("random", panels, False, {"kind": "random", "a": a, "c": c})
    # conical tip: the last stretch of the curve is a straight segment to the axis
    t_cut = np.pi * (1 - 1.0 / n_panels)
    r_c, z_c, _, _ = f(np.array([t_cut]))
    tip = (0.0, float(z_c[0]) + 0.6 * float(r_c[0]))
    edges = np.linspace(0.0, t_cut, n_panels)
    panels = [(x0, x1, f) for x0, x1 in zip(edges[:-1], edges[1:])]
    seg = _segment((float(r_c[0]), float(z_c[0])), tip)
    # segment panels about as long as the last body panel, the last one
    # refined dyadically toward the tip (neighbour length ratios <= 2)
    _, _, dr_c, dz_c = f(np.array([t_cut]))
    body_len = float(np.hypot(dr_c[0], dz_c[0])) * (t_cut / (n_panels - 1))
    seg_len = float(np.hypot(tip[0] - r_c[0], tip[1] - z_c[0]))
    k = max(1, int(round(seg_len / body_len)))
    cuts = np.linspace(0.0, 1.0, k + 1)
    for lo, hi in zip(cuts[:-2], cuts[1:-1]):
        panels.append((lo, hi, seg))
    for lo, hi in zip(*(lambda c_: (c_[:-1], c_[1:]))(_dyadic(cuts[-2], 1.0, tip_levels, True))):
        panels.append((lo, hi, seg))
    return _from_panels("random_tip", panels, False, {"kind": "random_tip", "a": a, "c": c})


def gl_weights(curve: Curve) -> np.ndarray:
    """Arclength quadrature weight per node: Gauss-Legendre weight times ds/du."""
    _, wg = npleg.leggauss(curve.order)
    return np.tile(wg, curve.n_panels) * curve.dsdu
