"""Whole-chain pins for the oracle: mode parity, the trivial medium, the Mie
series (P8), and energy balance for a lossless sphere (P10)."""
import numpy as np
import pytest

import mie
from oracle import assemble, discretize, farfield, modal, solve
from workloads import geometry, incident, rules


def build(curve, k0, eps1, M, L, mu1=1.0):
    (ys, ws), (ya, wa) = rules.load_rules()
    sup = discretize.support_points(curve, (ys, ws), (ya, wa))
    omega = k0
    k1 = omega * np.sqrt(complex(eps1 * mu1))
    kp = modal.KernelParams(k0, k1, M, L, float(curve.r.max()))
    assert kp.valid
    tab = modal.tabulate(curve, sup, kp)
    w = geometry.gl_weights(curve)
    mats = [assemble.assemble_mode(curve, sup, tab, m, k0, k1, omega, 1.0, 1.0, eps1, mu1, w)
            for m in range(M + 1)]
    return sup, tab, w, mats


@pytest.fixture(scope="module")
def sphere_case():
    curve = geometry.sphere(8)
    M, L, k0, eps1 = 16, 64, 1.0, 2.25
    sup, tab, w, mats = build(curve, k0, eps1, M, L)
    d, p = incident.tilted_direction(30.0)
    rhs = incident.rhs_modes(curve, [(d, p)], k0, -M, M)
    x = solve.solve_modes(mats, w, rhs, -M, M)
    return dict(curve=curve, M=M, k0=k0, eps1=eps1, w=w, mats=mats, x=x, d=d, p=p)


def test_mode_parity():
    """A_{-m} = D A_m D, D = diag(1, -1, -1, 1) per node, built independently."""
    curve = geometry.sphere(4)
    (ys, ws), (ya, wa) = rules.load_rules()
    sup = discretize.support_points(curve, (ys, ws), (ya, wa))
    kp = modal.KernelParams(1.0, 1.5 + 0j, 6, 64, 1.0)
    tab = modal.tabulate(curve, sup, kp)
    w = geometry.gl_weights(curve)

    class Even:  # g_{-m} = g_m: index the table by |m|
        def __init__(self, t):
            self.t = t

        def __getitem__(self, key):
            idx, *rest = key
            return self.t[([abs(i) for i in idx], *rest)]
    D = solve.parity_diag(curve.n)
    for m in (1, 2, 5):
        Ap = assemble.assemble_mode(curve, sup, tab, m, 1.0, 1.5 + 0j, 1.0, 1.0, 1.0, 2.25, 1.0, w)
        An = assemble.assemble_mode(curve, sup, Even(tab), -m, 1.0, 1.5 + 0j, 1.0, 1.0, 1.0, 2.25, 1.0, w)
        assert np.max(np.abs(An - D[:, None] * Ap * D[None, :])) < 1e-14 * np.max(np.abs(Ap))


def test_trivial_medium_scatters_nothing():
    """eps1 = eps0, mu1 = mu0: J, M are the incident traces and E_inf = 0."""
    curve = geometry.sphere(4)
    M = 14  # plane-wave modes beyond 14 are below 1e-15 for k0 r = 1
    sup, tab, w, mats = build(curve, 1.0, 1.0, M, 64)
    d, p = incident.tilted_direction(50.0)
    rhs = incident.rhs_modes(curve, [(d, p)], 1.0, -M, M)
    x = solve.solve_modes(mats, w, rhs, -M, M)
    assert np.allclose(x, rhs / 1j, atol=1e-13 * np.abs(rhs).max())
    dirs = np.array([[0.0, 0.6, 0.8], [0.3, -0.4, np.sqrt(0.75)]])
    E = farfield.far_field(curve, w, x[:, 0], -M, 1.0, 1.0, 1.0, dirs)
    # 4 panels of length 0.79 limit the surface quadrature of the far field
    assert np.abs(E).max() < 1e-10


@pytest.mark.slow
def test_mie_far_field(sphere_case):
    c = sphere_case
    rng = np.random.default_rng(0)
    dirs = rng.standard_normal((24, 3))
    dirs /= np.linalg.norm(dirs, axis=1)[:, None]
    E = farfield.far_field(c["curve"], c["w"], c["x"][:, 0], -c["M"], c["k0"], c["k0"], 1.0, dirs)
    e = np.cross(np.cross(c["d"], c["p"]), c["d"])
    Em = mie.far_field(c["k0"], 1.0, np.sqrt(c["eps1"]), c["d"], e, dirs)
    err = np.max(np.linalg.norm(E - Em, axis=1)) / np.max(np.linalg.norm(Em, axis=1))
    # 8 equal panels on the semicircle: ~1.7e-9, limited by the rows next to the
    # axis, where the 1/r_t and 1/r_t^2 factors of the mode operators amplify
    # rounding of the kernels
    assert err < 5e-9, err


@pytest.mark.slow
def test_energy_balance_lossless(sphere_case):
    """Net time-averaged power through the surface of a lossless body is 0:
    pi sum_m int Re(M2 conj(J1) - M1 conj(J2)) r ds = 0."""
    c = sphere_case
    X = c["x"][:, 0].reshape(2 * c["M"] + 1, c["curve"].n, 4)
    J1, J2, M1, M2 = (X[:, :, i] for i in range(4))
    rw = c["curve"].r * c["w"]
    P = np.pi * np.sum(np.real(M2 * np.conj(J1) - M1 * np.conj(J2)) * rw[None, :])
    scale = np.pi * np.sum((np.abs(J1) + np.abs(J2)) * (np.abs(M1) + np.abs(M2)) * rw[None, :])
    assert abs(P) < 1e-9 * scale
