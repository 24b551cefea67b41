"""Pins for the near-panel quadrature rules: exact moments of the families they
are built for (Section 5, remark on generalized Gaussian quadratures)."""
import mpmath as mp
import numpy as np
import pytest
from numpy.polynomial import legendre as npleg

from workloads import rules

(YS, WS), (YA, WA) = rules.load_rules()
XG, _ = npleg.leggauss(16)


def _P(j, y):
    return npleg.legval(y, np.eye(16)[j])


@pytest.mark.parametrize("i", [0, 3, 7, 12, 15])
def test_self_rules_exact(i):
    mp.mp.dps = 30
    x = XG[i]
    for j in (0, 1, 6, 15):
        exact_log = float(mp.quad(lambda y: mp.legendre(j, y) * mp.log(abs(y - x)), [-1, x, 1]))
        exact_pol = 2.0 if j == 0 else 0.0
        assert abs(np.sum(WS[i] * _P(j, YS[i]) * np.log(np.abs(YS[i] - x))) - exact_log) < 5e-15
        assert abs(np.sum(WS[i] * _P(j, YS[i])) - exact_pol) < 5e-15


@pytest.mark.parametrize("delta,alpha", [(0.0053, 0.0), (0.0106, 0.1), (0.3, 0.7), (1.9, 0.0),
                                          (0.02, np.pi / 2), (3.9, 1.2)])
def test_adjacent_rule_exact(delta, alpha):
    """log|y - x| with x beside either endpoint, from a 2:1 refined neighbour's
    nearest node (delta ~ 0.0053) to a 2:1 coarser neighbour's farthest node,
    at angles up to a right-angle corner."""
    mp.mp.dps = 30
    for side in (1, -1):
        xr = side * (1 + delta * np.cos(alpha))
        xi = delta * np.sin(alpha)
        for j in (0, 2, 9, 15):
            f = lambda y: mp.legendre(j, y) * 0.5 * mp.log((y - xr) ** 2 + xi ** 2)
            exact = float(mp.quad(f, [-1, 0, 1]))
            got = np.sum(WA * _P(j, YA) * 0.5 * np.log((YA - xr) ** 2 + xi ** 2))
            assert abs(got - exact) < 1e-14 * max(1.0, abs(exact))


def test_self_rules_keep_their_distance():
    """No self-rule node lies within 1e-5 of its target: nodes closer than that,
    paired with weights of opposite sign, multiplied the rounding of the
    derivative kernels (which grow like 1/|x - y|) by sum |w| / |y - x| ~ 1e8."""
    for i in range(16):
        d = np.abs(YS[i] - XG[i])
        assert d.min() >= 1e-5
        assert np.sum(np.abs(WS[i]) / d) < 3e4


def test_rules_are_polynomially_exact_and_inside():
    assert np.all(np.abs(YS) < 1) and np.all(np.abs(YA) < 1)
    for j in range(16):
        assert abs(np.sum(WA * _P(j, YA)) - (2.0 if j == 0 else 0.0)) < 1e-15
