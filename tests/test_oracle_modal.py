"""Pins for the modal Green's functions (Section 4) and the mode-m operator
expansions (Lemma 1 and the N, K expansions of Section 3).

* brute force: mpmath quadrature of the defining phi-integrals (P1);
* well separated pairs: a 4096-point trapezoid of the unsplit integrands;
* k -> 0: g_m -> Q_{m-1/2}(chi) / (2 pi sqrt(r_t r_s)) (eq. lm);
* the modal Helmholtz equation, which ties the second-derivative types to the
  others: (d_rr + d_r / r - m^2/r^2 + d_zz + k^2) g^k_m = 0 away from the source;
* Lemma 1 and the N and K expansions against a direct 3-D surface integral and
  finite differences at an off-surface point.
"""
import mpmath as mp
import numpy as np
import pytest

from mp_brute import types_at
from oracle import assemble, modal
from workloads import geometry

KP2 = dict(k0=10.0, k1=20.0 + 0j, M=64, L=256, r_max=1.0)


@pytest.mark.slow
@pytest.mark.parametrize("dr,dz", [(-0.01, 0.02), (-1e-5, 1e-6), (0.0, 1e-9), (-0.3, -0.5)])
def test_against_brute_force(dr, dz):
    kp = modal.KernelParams(**KP2)
    rt, zt = 0.8, 0.1
    ms = [0, 1, 9, 65]
    K = modal.modal_kernels([rt], [zt], None, None, kp, offsets=([dr], [dz]))[0]
    ref = np.array(types_at(rt, zt, dr, dz, kp.k0, kp.k1, ms, dps=24))  # [ms, 9]
    scale = np.max(np.abs(K), axis=1)
    for j, m in enumerate(ms):
        err = np.abs(K[:, m] - ref[j]) / scale
        assert np.all(err < 1e-13), (m, err)


def test_far_pairs_against_dense_trapezoid():
    kp = modal.KernelParams(**KP2)
    rng = np.random.default_rng(1)
    rt = rng.uniform(0.2, 1.0, 40)
    zt = rng.uniform(-2, 2, 40)
    rs = rng.uniform(0.2, 1.0, 40)
    zs = zt + rng.choice([-1, 1], 40) * rng.uniform(0.4, 2.0, 40)
    K = modal.modal_kernels(rt, zt, rs, zs, kp)
    R = modal.direct_trapezoid(rt, zt, rs, zs, kp.k0, kp.k1, kp.M, 4096)
    err = np.max(np.abs(K - R), axis=2) / np.max(np.abs(R), axis=2)
    assert err.max() < 1e-13


def test_near_and_far_branches_agree_at_the_switch():
    """Both branches are valid around acosh(chi) = a_min: they must agree."""
    kp = modal.KernelParams(**KP2)
    rt = np.full(6, 0.6)
    a = kp.a_min * np.array([1.0, 1.2, 1.5, 2.0, 3.0, 4.0])
    eta = np.cosh(a) - 1
    d = np.sqrt(2 * rt * rt * eta)
    Kn = modal.modal_kernels(rt, np.zeros(6), rt, d, kp, force="near")
    Kf = modal.modal_kernels(rt, np.zeros(6), rt, d, kp, force="far")
    err = np.max(np.abs(Kn - Kf), axis=2) / np.max(np.abs(Kn), axis=2)
    assert err.max() < 5e-14


def test_laplace_limit_is_legendre_q():
    """k -> 0: g_m = Q_{m-1/2}(chi)/(2 pi sqrt(rt rs)) and d_z g from dQ/dchi."""
    kp = modal.KernelParams(k0=1e-9, k1=2e-9 + 0j, M=20, L=128, r_max=1.0)
    mp.mp.dps = 30
    for rt, zt, rs, zs in [(0.5, 0.0, 0.52, 0.03), (0.5, 0.0, 0.9, 0.8)]:
        K = modal.modal_kernels([rt], [zt], [rs], [zs], kp)[0]
        chi = (rt * rt + rs * rs + (zt - zs) ** 2) / (2 * rt * rs)
        for m in (0, 1, 5, 21):
            nu = m - mp.mpf(1) / 2
            Q = mp.re(mp.legenq(nu, 0, chi, type=3))
            Qm = mp.re(mp.legenq(nu - 1, 0, chi, type=3))
            g = float(Q) / (2 * np.pi * np.sqrt(rt * rs))
            dQ = float(nu * (chi * Q - Qm) / (chi * chi - 1))
            gz = dQ * (zt - zs) / (rt * rs) / (2 * np.pi * np.sqrt(rt * rs))
            assert abs(K[0, m].real - g) < 1e-13 * abs(K[0, 0])
            assert abs(K[2, m].real - gz) < 1e-12 * np.max(np.abs(K[2]))


@pytest.mark.parametrize("k1", [20.0 + 0j, 40.0 + 0.5j])
def test_modal_helmholtz_identity(k1):
    """(d_rr + d_r/r - m^2/r^2 + d_zz) (g0 - g1) + k0^2 g0 - k1^2 g1 = 0."""
    kp = modal.KernelParams(k0=10.0, k1=k1, M=64, L=512, r_max=1.0)
    rt = np.array([0.7, 0.7, 0.7])
    zt = np.zeros(3)
    rs = np.array([0.69, 0.65, 0.3])
    zs = np.array([0.005, 0.1, 0.9])
    K = modal.modal_kernels(rt, zt, rs, zs, kp)
    m = np.arange(kp.M + 2)[None, :]
    dg = K[:, 3]
    dgr = K[:, 4]
    res = K[:, 6] + dgr / rt[:, None] - m * m / rt[:, None] ** 2 * dg + K[:, 8] \
        + (kp.k0 ** 2 - kp.k1 ** 2) * K[:, 0] + kp.k1 ** 2 * K[:, 3]
    scale = np.max(np.abs(K[:, 6]), axis=1)[:, None] + np.max(np.abs(m * m * dg), axis=1)[:, None]
    assert np.max(np.abs(res) / scale) < 1e-12


def _surface_potential(curve, w, dens, m, k, X):
    T = 256
    th = 2 * np.pi * np.arange(T) / T
    rp, zp = -curve.nz, curve.nr
    out = np.zeros(3, complex)
    J1, J2 = dens
    for s in range(curve.n):
        y = np.stack([curve.r[s] * np.cos(th), curve.r[s] * np.sin(th), np.full(T, curve.z[s])], 1)
        R = np.linalg.norm(y - X, axis=1)
        G = np.exp(1j * k * R) / (4 * np.pi * R)
        t = np.stack([rp[s] * np.cos(th), rp[s] * np.sin(th), np.full(T, zp[s])], 1)
        et = np.stack([-np.sin(th), np.cos(th), np.zeros(T)], 1)
        Jv = (J1[s] * t + J2[s] * et) * np.exp(1j * m * th)[:, None]
        out += w[s] * curve.r[s] * (2 * np.pi / T) * np.sum(G[:, None] * Jv, axis=0)
    return out


@pytest.mark.slow
def test_lemma1_and_operator_expansions_against_3d():
    curve = geometry.sphere(4)
    w = geometry.gl_weights(curve)
    k0, k1, m = 1.3, 2.1, 2
    kp = modal.KernelParams(k0, k1 + 0j, 8, 128, 1.0)
    rt, zt, trt, tzt = 0.5, 0.3, 0.6, 0.8  # off-surface target, any unit tangent
    N = curve.n
    K = modal.modal_kernels(np.full(N, rt), np.full(N, zt), curve.r, curve.z, kp)
    tab = np.stack([K[:, :, abs(m - 1)], K[:, :, m], K[:, :, m + 1]]).transpose(0, 2, 1)
    B = assemble.blocks(tab, m, rt, trt, tzt, curve.r, -curve.nz, curve.nr,
                        k0, k1 + 0j, 1.0, 1.0, 1.0, 0.0, 0.0)
    dens = (np.cos(curve.z) + 0.3, np.sin(2 * curve.z) + 0.1j)
    a = np.stack(dens)
    Kop = np.einsum("abn,bn,n->a", B[2:4, 0:2], a, w)
    Nop = np.einsum("abn,bn,n->a", B[2:4, 2:4], a, w) / (-1j)
    # Lemma 1 via the g^{k0} column of the blocks is implicit; check the fields
    h = 2e-3
    X0 = np.array([rt, 0, zt])
    E = np.eye(3, dtype=int)

    def derivs(k):
        A = {}
        for i in (-1, 0, 1):
            for j in (-1, 0, 1):
                for l in (-1, 0, 1):
                    if abs(i) + abs(j) + abs(l) <= 2:
                        A[(i, j, l)] = _surface_potential(curve, w, dens, m, k, X0 + h * np.array([i, j, l]))
        d = np.zeros((3, 3), complex)
        for i in range(3):
            d[i] = (A[tuple(E[i])] - A[tuple(-E[i])]) / (2 * h)
        curl = np.array([d[1, 2] - d[2, 1], d[2, 0] - d[0, 2], d[0, 1] - d[1, 0]])

        def dd(i, j, c):
            if i == j:
                return (A[tuple(E[i])][c] - 2 * A[(0, 0, 0)][c] + A[tuple(-E[i])][c]) / h ** 2
            return (A[tuple(E[i] + E[j])][c] - A[tuple(E[i] - E[j])][c]
                    - A[tuple(-E[i] + E[j])][c] + A[tuple(-E[i] - E[j])][c]) / (4 * h * h)
        gd = np.array([sum(dd(i, j, j) for j in range(3)) for i in range(3)])
        return A[(0, 0, 0)], curl, gd

    A0, c0, gd0 = derivs(k0)
    A1, c1, gd1 = derivs(k1)
    n = np.array([tzt, 0, -trt])
    t = np.array([trt, 0, tzt])
    eth = np.array([0, 1.0, 0])
    Nv = np.cross(n, c0)
    Kv = np.cross(n, k0 ** 2 * A0 + gd0) - np.cross(n, k1 ** 2 * A1 + gd1)
    assert np.allclose(Nop, [Nv @ t, Nv @ eth], rtol=0, atol=1e-5 * np.abs(Nop).max())
    assert np.allclose(Kop, [Kv @ t, Kv @ eth], rtol=0, atol=1e-5 * np.abs(Kop).max())


@pytest.mark.slow
@pytest.mark.parametrize("dr,dz", [(-2e-4, 1e-4), (-0.3, -0.5)])
def test_against_brute_force_complex_k1(dr, dz):
    """Absorbing interior (k1 = 40 + 0.5i, the lossy cylinder's k0 = 20 with
    eps1 = 4 + 0.1i): a near and a far pair against 24-digit quadrature, every
    type, modes up to M + 1 = 129 (measured <= 1.2e-14)."""
    kp = modal.KernelParams(k0=20.0, k1=40.0 + 0.5j, M=128, L=512, r_max=1.0)
    assert kp.valid
    rt, zt = 0.8, 0.1
    ms = [0, 1, 17, 129]
    K = modal.modal_kernels([rt], [zt], None, None, kp, offsets=([dr], [dz]))[0]
    ref = np.array(types_at(rt, zt, dr, dz, kp.k0, kp.k1, ms, dps=24))
    scale = np.max(np.abs(K), axis=1)
    for j, m in enumerate(ms):
        err = np.abs(K[:, m] - ref[j]) / scale
        assert np.all(err < 1e-13), (m, err)
