"""Pins for the special functions (Section 4 and Appendix A) against independent
library routines: scipy's elliptic integrals, mpmath's Legendre Q of
half-odd degree (toroidal functions), and direct quadrature of 1/rho^3."""
import math

import mpmath as mp
import numpy as np
import pytest
from scipy.special import ellipe, ellipk

from oracle import special


@pytest.mark.parametrize("kp2", [1e-20, 1e-12, 1e-6, 0.01, 0.5, 0.99])
def test_elliptic_against_scipy(kp2):
    K, E = special.elliptic_KE(np.array([kp2]))
    mp.mp.dps = 40
    Kref = float(mp.ellipk(1 - mp.mpf(kp2)))  # mpmath takes the parameter k^2
    Eref = float(mp.ellipe(1 - mp.mpf(kp2)))
    assert abs(K[0] - Kref) <= 1e-15 * Kref
    assert abs(E[0] - Eref) <= 2e-15 * Eref
    if kp2 > 1e-3:  # scipy (parameter form) is accurate away from k' -> 0
        assert abs(K[0] - ellipk(1.0 - kp2)) <= 1e-14 * Kref
        assert abs(E[0] - ellipe(1.0 - kp2)) <= 1e-14 * Eref


@pytest.mark.parametrize("eta", [1e-18, 1e-10, 1e-6, 1e-3, 0.03, 0.3, 3.0])
def test_legendre_q_half_against_mpmath(eta):
    nmax = 130
    fwd = (107, 3.0)
    Q, num = special.legendre_q(np.array([eta]), nmax, fwd, 20.0)
    mp.mp.dps = 40
    chi = 1 + mp.mpf(eta)
    q0 = mp.re(mp.legenq(-mp.mpf(1) / 2, 0, chi, type=3))
    for n in (0, 1, 2, 7, 30, 64, 100, 128):
        ref = mp.re(mp.legenq(n - mp.mpf(1) / 2, 0, chi, type=3))
        # normwise: relative to Q_{-1/2}, the largest of the sequence
        assert abs(Q[0, n] - float(ref)) <= 1e-14 * float(abs(q0)), n


def test_q_recurrence_seeds():
    """Q_{1/2} from the elliptic seeds equals mpmath's toroidal function."""
    mp.mp.dps = 30
    for eta in (1e-8, 0.1, 2.0):
        q0, q1, tail = special.q_half_seeds(np.array([eta]))
        ref = mp.re(mp.legenq(mp.mpf(1) / 2, 0, 1 + mp.mpf(eta), type=3))
        assert abs(q1[0] - float(ref)) <= 1e-13 * abs(float(ref)) + 1e-15 * q0[0]


@pytest.mark.parametrize("eta", [1e-4, 0.05, 0.8])
def test_rho3_spectrum_against_quadrature(eta):
    """X3_n (Lemma A.2 applied to 1/rho^3) against direct quadrature."""
    rt, rs = 0.7, 0.9
    X1, X3 = special.spectra(np.array([rt]), np.array([rs]), np.array([eta]), 40,
                             (60, 3.0), 20.0)
    mp.mp.dps = 30
    d2 = mp.mpf(eta) * 2 * rt * rs
    for n in (0, 1, 3, 10, 25):
        f3 = lambda p: mp.cos(n * p) / (d2 + 4 * rt * rs * mp.sin(p / 2) ** 2) ** 1.5
        f1 = lambda p: mp.cos(n * p) / (d2 + 4 * rt * rs * mp.sin(p / 2) ** 2) ** 0.5
        sc = mp.sqrt(eta)
        pts = [0, sc, 10 * sc, mp.pi] if 10 * sc < mp.pi else [0, sc, mp.pi]
        r3 = 2 * mp.quad(f3, pts)
        r1 = 2 * mp.quad(f1, pts)
        assert abs(X3[0, n] - float(r3)) <= 1e-13 * abs(X3[0, 0])
        assert abs(X1[0, n] - float(r1)) <= 1e-13 * abs(X1[0, 0])


def test_s_relation_holds_at_n0():
    """The n = 0 case of the S relation with Q_{-3/2} = Q_{1/2}: S_0 = -2 dP_0/dchi."""
    eta = 0.2
    X1, X3 = special.spectra(np.array([1.0]), np.array([1.0]), np.array([eta]), 5, (6, 3.0), 20.0)
    h = 1e-6
    Xp, _ = special.spectra(np.array([1.0]), np.array([1.0]), np.array([eta + h]), 5, (6, 3.0), 20.0)
    Xm, _ = special.spectra(np.array([1.0]), np.array([1.0]), np.array([eta - h]), 5, (6, 3.0), 20.0)
    # 1/rho = (2 (chi - cos))^{-1/2} for rt = rs = 1, d/dchi (1/rho) = -(1/rho^3)
    dX1 = (Xp[0, 0] - Xm[0, 0]) / (2 * h)
    assert abs(-dX1 - X3[0, 0]) <= 1e-7 * abs(X3[0, 0])
