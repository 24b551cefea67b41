"""Special functions behind the singular parts of the modal kernels.

All arrays are float64 and vectorized over node pairs.  Everything is written
in terms of eta = chi - 1 = d^2 / (2 r_t r_s) (d the distance in the (r, z)
half-plane) so that chi - 1 is never formed by subtraction.

Q_{n-1/2}(chi)   Section 4.1, eq. (lm) and the recurrence (recurform) with its
                 elliptic-integral seeds; Miller's backward algorithm where the
                 forward recurrence is unstable (Section 4.1, last paragraph).
S_n(chi)         Section 4.2, eq. (pm) and Lemma A.2:
                 S_n = sqrt(8) (1-2n) (chi Q_{n-1/2} - Q_{n-3/2}) / (chi^2 - 1),
                 used for n = 0 as well with Q_{-3/2} = Q_{1/2} (evenness of the
                 integrand in n).
"""
from __future__ import annotations

import math

import numpy as np


def acosh_chi(eta):
    """acosh(1 + eta), accurate for tiny eta."""
    eta = np.asarray(eta, float)
    return np.log1p(eta + np.sqrt(eta * (2.0 + eta)))


def elliptic_KE(kp2):
    """Complete elliptic integrals K(k), E(k) of modulus k, given k'^2 = 1 - k^2.

    Arithmetic-geometric mean started from (1, k'), so that K ~ log(4/k') is
    accurate as k' -> 0:  K = pi / (2 AGM(1, k')),
    E = K (1 - sum_n 2^(n-1) c_n^2) with c_0 = k, c_{n+1} = (a_n - b_n)/2.
    """
    kp2 = np.asarray(kp2, float)
    a = np.ones_like(kp2)
    b = np.sqrt(kp2)
    s = 0.5 * (1.0 - kp2)  # 2^{-1} c_0^2 with c_0^2 = k^2
    p = 0.5
    for _ in range(40):
        c = 0.5 * (a - b)
        a, b = 0.5 * (a + b), np.sqrt(a * b)
        p *= 2.0
        s = s + p * c * c
        if np.all(np.abs(c) <= 1e-17 * a):
            break
    K = np.pi / (2.0 * a)
    E = K * (1.0 - s)
    return K, E


def q_half_seeds(eta):
    """Q_{-1/2}(chi), Q_{1/2}(chi) from the elliptic integrals (Section 4.1).

    Modulus k = sqrt(2/(chi+1)), so k'^2 = eta / (2 + eta) and
    Q_{-1/2} = k K(k),  Q_{1/2} = chi Q_{-1/2} - sqrt(2 (chi+1)) E(k).
    Also returns sqrt(2(chi+1)) E, which equals chi Q_{-1/2} - Q_{1/2} exactly.
    """
    eta = np.asarray(eta, float)
    kp2 = eta / (2.0 + eta)
    K, E = elliptic_KE(kp2)
    k = np.sqrt(2.0 / (2.0 + eta))
    q0 = k * K
    tail = np.sqrt(2.0 * (2.0 + eta)) * E
    q1 = (1.0 + eta) * q0 - tail
    return q0, q1, tail


def legendre_q(eta, nmax, forward_limit, miller_extra):
    """Q_{n-1/2}(1 + eta), n = 0..nmax, and the numerators of S_n.

    Returns (Q, num), both [len(eta), nmax + 1], with
    num_n = chi Q_{n-1/2} - Q_{n-3/2} (num_0 uses Q_{-3/2} = Q_{1/2}).

    Pairs with acosh(chi) * forward_limit[0] <= forward_limit[1] run the
    three-term recurrence of eq. (recurform) forward.  Close to chi = 1 that
    recurrence has a double characteristic root, so it is run on the
    differences D_n = Q_{n-1/2} - Q_{n-3/2}; subtracting (n+1/2) Q_{n-1/2}
    from both sides of the recurrence gives the identical relation
        (n + 1/2) D_{n+1} = (n - 1/2) D_n + 2 n eta Q_{n-1/2},
        Q_{n+1/2} = Q_{n-1/2} + D_{n+1},
    whose rounding errors grow linearly instead of quadratically in n, and
    num_n = D_n + eta Q_{n-1/2} needs no cancelling subtraction.
    Other pairs use Miller's backward algorithm started at
    n_start = max(nmax + 2, forward_limit[0] + ceil(miller_extra / acosh chi)),
    normalized by the exact Q_{-1/2}.
    """
    eta = np.atleast_1d(np.asarray(eta, float))
    P = eta.size
    chi = 1.0 + eta
    a = acosh_chi(eta)
    q0, q1, tail = q_half_seeds(eta)
    Q = np.zeros((P, nmax + 1))
    num = np.zeros((P, nmax + 1))
    fwd = a * forward_limit[0] <= forward_limit[1]
    idx = np.nonzero(fwd)[0]
    if idx.size:
        e = eta[idx]
        Q[idx, 0] = q0[idx]
        num[idx, 0] = tail[idx]
        D = e * q0[idx] - tail[idx]  # D_1 = Q_{1/2} - Q_{-1/2}
        for n in range(1, nmax + 1):
            Q[idx, n] = Q[idx, n - 1] + D
            num[idx, n] = D + e * Q[idx, n]
            D = ((n - 0.5) * D + 2 * n * e * Q[idx, n]) / (n + 0.5)
    idx = np.nonzero(~fwd)[0]
    for i in idx:
        # Miller: backward from n_start with (Q_{n_start+1/2}, Q_{n_start-1/2}) = (0, 1)
        ns = max(nmax + 2, forward_limit[0] + int(math.ceil(miller_extra / a[i])))
        c = chi[i]
        f_hi, f = 0.0, 1.0  # f = f_{n - 1/2}, f_hi = f_{n + 1/2}, n = ns
        vals = np.zeros(nmax + 1)
        for n in range(ns, 0, -1):
            f_lo = (2 * n * c * f - (n + 0.5) * f_hi) / (n - 0.5)  # f_{n-3/2}
            f_hi, f = f, f_lo
            if n - 1 <= nmax:
                vals[n - 1] = f
            if abs(f) > 1e250:
                f_hi *= 1e-250
                f *= 1e-250
                vals *= 1e-250
        vals *= q0[i] / vals[0]
        Q[i] = vals
        num[i, 0] = tail[i]
        num[i, 1:] = c * vals[1:] - vals[:-1]
    return Q, num


def spectra(rt, rs, eta, nmax, forward_limit, miller_extra):
    """Azimuthal Fourier coefficients of 1/rho and 1/rho^3, n = 0..nmax.

    X1_n = int_0^{2pi} e^{-i n phi} / rho dphi = 2 Q_{n-1/2}(chi) / sqrt(rt rs)
    X3_n = int_0^{2pi} e^{-i n phi} / rho^3 dphi = S_n(chi) / (2 rt rs)^{3/2}
    (4 pi times the q-hat and p-hat of eqs. (lm) and (pm)).
    """
    Q, num = legendre_q(eta, nmax, forward_limit, miller_extra)
    X1 = 2.0 * Q / np.sqrt(rt * rs)[:, None]
    n = np.arange(nmax + 1)[None, :]
    den = (eta * (2.0 + eta))[:, None]
    S = math.sqrt(8.0) * (1 - 2 * n) * num / den
    X3 = S / ((2.0 * rt * rs) ** 1.5)[:, None]
    return X1, X3
