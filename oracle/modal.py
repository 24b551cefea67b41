"""Modal Green's functions and their derivatives (Section 4).

For a target (r_t, z_t) and a source (r_s, z_s) on the generating curve the
nine stored quantities per azimuthal mode m are (eq. green11 and derivatives
with respect to the target coordinates):

    0 g^{k0}_m           1 d_r g^{k0}_m           2 d_z g^{k0}_m
    3 (g^{k0}-g^{k1})_m  4 d_r (g^{k0}-g^{k1})_m  5 d_z (g^{k0}-g^{k1})_m
    6 d_rr (g^{k0}-g^{k1})_m   7 d_rz (g^{k0}-g^{k1})_m   8 d_zz (g^{k0}-g^{k1})_m

with g^k_m = int_0^{2pi} e^{ik rho}/(4 pi rho) e^{-i m phi} dphi and rho^2 =
d^2 + 4 r_t r_s sin^2(phi/2).  Only the k0 - k1 difference of the second
derivatives enters the Mueller system (Section 4.3), which removes their
hypersingularity.  The interior family is stored as the difference too:
the K operators enter only as K^{k0} - K^{k1}, N^{k1} = N^{k0} - (N^{k0} -
N^{k1}), and at the support nodes closest to a target d_r g and d_z g reach
1e9, so forming the difference from two tabulated values would keep about
7 digits of it; formed from the integrands below it keeps full precision.

Kernel splitting (Sections 4.1-4.3).  Every integrand is written as
sum(analytic factor x X) + analytic part, with X in {1/rho, 1/rho^3}:

    e^{ik rho}/rho          = cos(k rho) . 1/rho  +  i k sinc(k rho)
    (ik rho - 1) e^{ik rho} = -W_k + i Y_k,   W = cos x + x sin x,  Y = x cos x - sin x
    (3 - 3ik rho - k^2 rho^2) e^{ik rho} = U_k + i V_k,
        U = 3 cos x - x^2 cos x + 3 x sin x,  V = 3 sin x - x^2 sin x - 3 x cos x

(x = k rho).  Y/rho^3, V/rho^5, (U_{k0}-U_{k1})/rho^2, (W_{k0}-W_{k1})/rho^2 and
(cos(k0 rho) - cos(k1 rho))/rho^2 are analytic in phi, evaluated with Taylor
series for small |x| (the paper's small-rho Taylor remark in Section 4.1).
The differences of the first family are

    (g^{k0} - g^{k1}) 4 pi  = rho^2 Cd X1 + i (k0 sinc(k0 rho) - k1 sinc(k1 rho))
    d_r (g^{k0} - g^{k1}) 4 pi = r_d (-Wd X1 + i Y3d),   d_z: z_t - z_s for r_d

with Cd = k0^2 Ct(k0 rho) - k1^2 Ct(k1 rho), Ct(x) = (cos x - 1)/x^2,
Wd = k0^2 Wt(k0 rho) - k1^2 Wt(k1 rho), Y3d = k0^3 Y3(k0 rho) - k1^3 Y3(k1 rho).  The factor r_d = r_t - r_s cos(phi)
of the r-derivatives is written r_d = (rho^2 + a) / (2 r_t) with
a = r_t^2 - r_s^2 - (z_t - z_s)^2 so that no smooth factor carries a cancelling
r_d next to a singular X:

    r_d / rho^3   = (X1 + a X3) / (2 r_t)
    r_d^2 / rho^3 = (rho^2 X1 + 2 a X1 + a^2 X3) / (4 r_t^2).

For near pairs X is replaced by its band-limited version
X_L(phi) = (1/2pi) sum_{|n|<=M_q} X_n e^{i n phi}, with X_n from the Legendre-Q
spectra (eq. lm, eq. pm), and the product is transformed with an L-point FFT:
the discrete convolution of eq. (discA).  For well separated pairs X = 1/rho^p
exactly and the same L-point trapezoid rule is already exact to rounding
(Section 4, first paragraphs after eq. equrelation).
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

from . import special

NTYPES = 9


@dataclass
class KernelParams:
    """Pair classification and transform sizes shared by every pair of a body.

    N_f: azimuthal bandwidth of the analytic factors, the smallest j with
         (x/2)^(2j)/(2j)! <= 1e-16 for x = 2 max|k| r_max (a bound on the
         Bessel coefficients J_{2j}(x) of cos(k rho(phi))).
    The convolution is exact when m_hi + N_f <= M_q, m_hi = M + 1, M_q = L/2-1.
    A pair is "near" (split + convolution) iff acosh(chi) < a_min with
    a_min = TAU / (L - m_hi - N_f): otherwise the trapezoid aliasing
    exp(-(L - m - N_f) acosh chi) is below e^-TAU.
    Near pairs use the forward Q recurrence iff acosh(chi) (m_hi + N_f) <= FWD,
    else Miller's algorithm with MILLER extra e-folds.
    """
    k0: float
    k1: complex
    M: int
    L: int
    r_max: float
    TAU: float = 36.0
    FWD: float = 3.0
    MILLER: float = 20.0

    def __post_init__(self):
        self.m_hi = self.M + 1
        self.Mq = self.L // 2 - 1
        x = 2.0 * max(abs(self.k0), abs(self.k1)) * self.r_max
        j = 1
        while True:
            nu = 2 * j
            lb = nu * math.log(max(x, 1e-300) / 2.0) - math.lgamma(nu + 1.0)
            if lb <= math.log(1e-16):
                break
            j += 1
        self.Nf = j
        self.valid = self.m_hi + self.Nf <= self.Mq
        self.a_min = self.TAU / max(self.L - self.m_hi - self.Nf, 1)
        self.fwd_n = self.m_hi + self.Nf


# --------------------------------------------------------------------------
# analytic factors: series for |x| <= 2, closed forms beyond
# --------------------------------------------------------------------------
_NSER = 20
_fact = [math.factorial(i) for i in range(2 * _NSER + 8)]
_C_SINC = [(-1) ** i / _fact[2 * i + 1] for i in range(_NSER)]
_C_Y3 = [(-1) ** (i + 1) * 2 * (i + 1) / _fact[2 * i + 3] for i in range(_NSER)]
_C_WT = [(-1) ** i * (2 * i + 1) / _fact[2 * i + 2] for i in range(_NSER)]
_C_UT = [(-1) ** (i + 1) * (2 * i + 1) * (2 * i - 1) / _fact[2 * i + 2] for i in range(_NSER)]
_C_V5 = [(-1) ** i * 4 * (i + 2) * (i + 1) / _fact[2 * i + 5] for i in range(_NSER)]
_C_CT = [(-1) ** (i + 1) / _fact[2 * i + 2] for i in range(_NSER)]


def _horner(coef, y):
    acc = np.zeros_like(y) + coef[-1]
    for c in coef[-2::-1]:
        acc = acc * y + c
    return acc


def analytic_factors(x):
    """For x = k rho (real or complex array):
    cos x, sinc x, W = cos x + x sin x, Y3 = Y/x^3, Wt = (W-1)/x^2,
    Ut = (U-3)/x^2, V5 = V/x^5, Ct = (cos x - 1)/x^2."""
    x = np.asarray(x)
    c = np.cos(x)
    s = np.sin(x)
    small = np.abs(x) <= 2.0
    y = x * x
    with np.errstate(all="ignore"):
        sinc = np.where(small, _horner(_C_SINC, y), s / x)
        Y3 = np.where(small, _horner(_C_Y3, y), (x * c - s) / (x * y))
        Wt = np.where(small, _horner(_C_WT, y), (c + x * s - 1.0) / y)
        Ut = np.where(small, _horner(_C_UT, y), (3.0 * c - y * c + 3.0 * x * s - 3.0) / y)
        V5 = np.where(small, _horner(_C_V5, y), (3.0 * s - y * s - 3.0 * x * c) / (y * y * x))
        Ct = np.where(small, _horner(_C_CT, y), (c - 1.0) / y)
    W = 1.0 + y * Wt
    return c, sinc, W, Y3, Wt, Ut, V5, Ct


def sample_types(rt, dr, dz, cosphi, rho2, X1, X3, k0, k1, exact=False):
    """The nine integrands (times 4 pi) at azimuth samples.

    rt, dr = r_s - r_t, dz = z_s - z_t: [P, 1]; cosphi, rho2: [P, J] or [1, J];
    X1, X3: [P, J] samples of 1/rho and 1/rho^3, band-limited for near pairs.
    exact: X1, X3 are exactly 1/rho, 1/rho^3 (well separated pairs); then
    r_d/rho^3 and r_d^2/rho^3 are formed from r_d directly, because the identity
    r_d = (rho^2 + a)/(2 r_t) cancels badly when r_t is small and rho is not.
    Returns [9, P, J] complex.
    """
    rs = rt + dr
    zd = -dz
    a = -dr * (2.0 * rt + dr) - dz * dz
    rd = rt - rs * cosphi
    rho = np.sqrt(rho2)
    if exact:
        Xa = rd * X3
        Xaa = rd * rd * X3
    else:
        Xa = (X1 + a * X3) / (2.0 * rt)
        Xaa = (rho2 * X1 + 2.0 * a * X1 + a * a * X3) / (4.0 * rt * rt)
    c0, sinc0, W0, Y30, Wt0, Ut0, V50, Ct0 = analytic_factors(k0 * rho)
    c1, sinc1, W1, Y31, Wt1, Ut1, V51, Ct1 = analytic_factors(k1 * rho)
    k0_, k1_ = k0, k1
    g0 = c0 * X1 + 1j * k0 * sinc0
    dr0 = -W0 * Xa + 1j * k0 ** 3 * Y30 * rd
    dz0 = zd * (-W0 * X3 + 1j * k0 ** 3 * Y30)
    Pd = k0_ ** 2 * Ut0 - k1_ ** 2 * Ut1
    Wd = k0_ ** 2 * Wt0 - k1_ ** 2 * Wt1
    V5d = k0_ ** 5 * V50 - k1_ ** 5 * V51
    Y3d = k0_ ** 3 * Y30 - k1_ ** 3 * Y31
    Cd = k0_ ** 2 * Ct0 - k1_ ** 2 * Ct1
    Sd = k0_ * sinc0 - k1_ * sinc1
    dg = rho2 * Cd * X1 + 1j * Sd
    F1d = -Wd * X1 + 1j * Y3d
    out = [g0, dr0, dz0, dg, rd * F1d, zd * F1d]
    rr = Pd * Xaa - Wd * X1 + 1j * (V5d * rd * rd + Y3d)
    rz = Pd * zd * Xa + 1j * V5d * rd * zd
    zz = Pd * zd * zd * X3 - Wd * X1 + 1j * (V5d * zd * zd + Y3d)
    out += [rr, rz, zz]
    return np.stack([np.broadcast_to(o, X1.shape).astype(complex) for o in out])


def _grid(L):
    j = np.arange(L)
    phi = 2.0 * np.pi * j / L
    return phi, np.cos(phi), np.sin(phi / 2.0) ** 2


def modal_kernels(rt, zt, rs, zs, kp: KernelParams, force=None, offsets=None):
    """Modes m = 0..M+1 of the nine types for arrays of pairs: [P, 9, M+2].

    force: None (classify), "near" (always split) or "far" (always direct).
    offsets: optional (r_s - r_t, z_s - z_t) when they are known more
    accurately than the difference of the coordinates.
    """
    rt, zt, rs, zs = (np.asarray(v, float).ravel() for v in (rt, zt, rs, zs))
    if offsets is None:
        dr, dz = rs - rt, zs - zt
    else:
        dr, dz = (np.asarray(v, float).ravel() for v in offsets)
        rs = rt + dr
    P = rt.size
    L = kp.L
    phi, cphi, s2 = _grid(L)
    d2 = dr * dr + dz * dz
    eta = d2 / (2.0 * rt * rs)
    acosh = special.acosh_chi(eta)
    if force == "near":
        near = np.ones(P, bool)
    elif force == "far":
        near = np.zeros(P, bool)
    else:
        near = acosh < kp.a_min
    out = np.zeros((P, NTYPES, kp.M + 2), dtype=complex)
    col = lambda v: v[:, None]
    for sel in (np.nonzero(~near)[0], np.nonzero(near)[0]):
        if sel.size == 0:
            continue
        is_near = bool(near[sel[0]])
        for c0 in range(0, sel.size, 4096):
            idx = sel[c0:c0 + 4096]
            rho2 = col(d2[idx]) + 4.0 * col(rt[idx] * rs[idx]) * s2[None, :]
            if is_near:
                X1h, X3h = special.spectra(rt[idx], rs[idx], eta[idx], kp.Mq,
                                           (kp.fwd_n, kp.FWD), kp.MILLER)
                X1 = _synthesize(X1h, L)
                X3 = _synthesize(X3h, L)
            else:
                rho = np.sqrt(rho2)
                X1 = 1.0 / rho
                X3 = 1.0 / (rho * rho2)
            K = sample_types(col(rt[idx]), col(dr[idx]), col(dz[idx]),
                             cphi[None, :], rho2, X1, X3, kp.k0, kp.k1, exact=not is_near)
            F = np.fft.fft(K, axis=-1) * (2.0 * np.pi / L) / (4.0 * np.pi)
            out[idx] = F[..., : kp.M + 2].transpose(1, 0, 2)
    return out


def _synthesize(Xh, L):
    """X_L(phi_j) = (1/2pi) sum_{|n|<=M_q} X_n e^{i n phi_j}, X_{-n} = X_n."""
    P, nq = Xh.shape
    spec = np.zeros((P, L))
    spec[:, :nq] = Xh
    spec[:, L - nq + 1:] = Xh[:, 1:][:, ::-1]
    return np.real(np.fft.ifft(spec, axis=-1)) * L / (2.0 * np.pi)


def direct_trapezoid(rt, zt, rs, zs, k0, k1, M, Lt):
    """Reference: the unsplit integrands sampled on Lt azimuthal points
    (no series, no splitting) -- for well separated pairs and large Lt."""
    rt, zt, rs, zs = (np.asarray(v, float).ravel()[:, None] for v in (rt, zt, rs, zs))
    phi = 2 * np.pi * np.arange(Lt) / Lt
    cp = np.cos(phi)[None, :]
    rho2 = (rt - rs) ** 2 + (zt - zs) ** 2 + 4 * rt * rs * np.sin(phi / 2)[None, :] ** 2
    rho = np.sqrt(rho2)
    rd = rt - rs * cp
    zd = zt - zs
    f = {}
    for k in (k0, k1):
        E = np.exp(1j * k * rho)
        F1 = (1j * k * rho - 1) * E / (rho * rho2)
        G = E * (3 - 3j * k * rho - k * k * rho2) / (rho2 * rho2 * rho)
        f[k] = (E / rho, F1, G)
    g0, F10, _ = f[k0]
    dg = f[k0][0] - f[k1][0]
    H = f[k0][1] - f[k1][1]
    G = f[k0][2] - f[k1][2]
    out = [g0, rd * F10, zd * F10, dg, rd * H, zd * H, rd * rd * G + H, rd * zd * G, zd * zd * G + H]
    K = np.stack([np.broadcast_to(o, rho.shape) for o in out])
    F = np.fft.fft(K, axis=-1) * (2 * np.pi / Lt) / (4 * np.pi)
    return F[..., : M + 2].transpose(1, 0, 2)


def tabulate(curve, sup, kp: KernelParams, rows=None):
    """Modal-kernel table [M+2, 9, len(rows), N + S] for target rows `rows`.

    Sources 0..N-1 are the curve nodes, N..N+S-1 the target's support nodes.
    The coincident pair (target == source node) is log-singular and never used
    by the discretization (its panel is integrated with support nodes); it is
    stored as 0, as are unused support slots.
    """
    N = curve.n
    S = sup.r.shape[1]
    rows = np.arange(N) if rows is None else np.asarray(rows)
    T = rows.size
    out = np.zeros((kp.M + 2, NTYPES, T, N + S), dtype=complex)
    for i, t in enumerate(rows):
        dr = np.concatenate([curve.r - curve.r[t], sup.dr[t]])
        dz = np.concatenate([curve.z - curve.z[t], sup.dz[t]])
        valid = np.ones(N + S, bool)
        valid[t] = False
        valid[N:] = sup.wq[t] != 0.0
        idx = np.nonzero(valid)[0]
        K = modal_kernels(np.full(idx.size, curve.r[t]), np.full(idx.size, curve.z[t]),
                          None, None, kp, offsets=(dr[idx], dz[idx]))
        out[:, :, i, idx] = K.transpose(2, 1, 0)
    return out
