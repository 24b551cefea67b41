"""Support-node offsets (Section 5 near-panel quadrature) against a 40-digit
evaluation of the same degree-15 interpolant: the offsets r_s - r_t, z_s - z_t
must keep full relative precision even where z_s - z_t is a thousandth of the
distance (targets next to the axis) or the distance is 1e-10 of a panel."""
import mpmath as mp
import numpy as np
import pytest

from oracle import discretize
from workloads import geometry, rules

RULES = rules.load_rules()


def _mp_nodes():
    mp.mp.dps = 40
    roots = sorted(mp.findroot(lambda t: mp.legendre(16, t), mp.mpf(float(u)))
                   for u in np.polynomial.legendre.leggauss(16)[0])
    return [mp.mpf(float(v)) for v in roots]  # nodes rounded to double


@pytest.mark.parametrize("curve", [geometry.sphere(8), geometry.spheroid(6, 3.0)], ids=["sphere", "spheroid"])
def test_offsets_full_relative_precision(curve):
    ug = _mp_nodes()
    (ys, _), (ya, _) = RULES
    sup = discretize.support_points(curve, *RULES)
    NS = ys.shape[1]
    worst = 0.0
    for t in (0, 2, curve.n // 2, curve.n - 1):
        for s in range(0, sup.r.shape[1], 3):
            p = sup.panel[t, s]
            if p < 0:
                continue
            y = mp.mpf(ys[t % 16, s] if s < NS else ya[(s - NS) % ya.size])
            ell = []
            for k in range(16):
                v = mp.mpf(1)
                for j in range(16):
                    if j != k:
                        v *= (y - ug[j]) / (ug[k] - ug[j])
                ell.append(v)
            for arr, got in ((curve.r, sup.dr[t, s]), (curve.z, sup.dz[t, s])):
                ref = sum(ell[k] * mp.mpf(arr[16 * p + k]) for k in range(16)) - mp.mpf(arr[t])
                worst = max(worst, abs(float((got - ref) / ref)))
    assert worst < 3e-15, worst
