"""Writes extinction_cylinder_row1.json: the oracle's interior fields for the
extinction test of Section 6 on the cylinder of Example 4 at the size of
Table 4's first row (k0 = 2, k1 = 1, N_f = 9; 81 panels, the four corner
panels refined 14 dyadic levels), from the indirect system (eq. dualmullrep)
with the current-loop data (eq. loop), evaluated by eq. interior_dual on
4 sub-panels per panel at six seeded interior points.

Only oracle/ computes; workloads/ supplies the body, the rules and the loop
data.  About 6 minutes on one host core:

    python -m tests.golden.make_extinction_cylinder
"""
import json
import os

import numpy as np

from oracle import assemble, discretize, fields, modal, solve
from workloads import geometry, incident, rules

LOOP = dict(center=[0.4, 0.5, 5.0], radius=0.42)  # Section 6
K0, K1, NF = 2.0, 1.0, 9


def interior_points():
    rng = np.random.default_rng(3)
    rr, zz, th = 0.5 * np.sqrt(rng.uniform(0, 1, 6)), rng.uniform(-0.5, 0.5, 6), rng.uniform(0, 2 * np.pi, 6)
    return np.stack([rr * np.cos(th), rr * np.sin(th), zz], axis=1)


def main():
    curve = geometry.cylinder(14, 6.5)
    eps1 = (K1 / K0) ** 2
    (ys, ws), (ya, wa) = rules.load_rules()
    sup = discretize.support_points(curve, (ys, ws), (ya, wa))
    L = 64
    while not modal.KernelParams(K0, K1, NF, L, float(curve.r.max())).valid:
        L *= 2
    tab = modal.tabulate(curve, sup, modal.KernelParams(K0, K1, NF, L, float(curve.r.max())))
    w = geometry.gl_weights(curve)
    mats = [assemble.assemble_mode(curve, sup, tab, m, K0, K1, K0, 1.0, 1.0, eps1, 1.0, w, formulation="indirect")
            for m in range(NF + 1)]
    rhs = incident.loop_rhs_modes(curve, LOOP["center"], LOOP["radius"], K1, K0, 1.0, -NF, NF)
    x = solve.solve_modes(mats, w, rhs, -NF, NF)[:, 0]
    pts = interior_points()
    E, H = fields.fields(curve, w, x, -NF, pts, K0, K1, K0, 1.0, 1.0, eps1, 1.0, "interior", "indirect",
                         upsample=4)
    El, Hl = incident.current_loop(LOOP["center"], LOOP["radius"], K1, K0, 1.0)
    Er, Hr = El(pts), Hl(pts)
    err = np.sqrt((np.linalg.norm(E - Er) ** 2 + np.linalg.norm(H - Hr) ** 2)
                  / (np.linalg.norm(Er) ** 2 + np.linalg.norm(Hr) ** 2))
    c = lambda a: [[float(v.real), float(v.imag)] for v in np.asarray(a).ravel()]
    out = {"source": "oracle (tests/golden/make_extinction_cylinder.py)",
           "body": "cylinder of Example 4, 81 panels (26 base, 4 x 14 corner levels), N = %d" % curve.n,
           "k0": K0, "k1": K1, "N_f": NF, "L": L, "upsample": 4, "points": pts.tolist(),
           "E": c(E), "H": c(H), "E_error": float(err), "paper_E_error": 4.11e-9}
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "extinction_cylinder_row1.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print(path, "E_error", err)


if __name__ == "__main__":
    main()
