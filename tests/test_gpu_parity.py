"""GPU parity: the HIP library (through the C-ABI) against the FP64 oracle.

Tolerances: modal kernels 1e-12 relative, normwise over modes per (type,
target, source); matrices 1e-12 relative to the largest entry of the row
block; surface currents and far fields 1e-10 relative.
"""
import numpy as np
import pytest

from gpu_cases import RULES, normwise_table_error, oracle_matrix, oracle_setup, oracle_table
from oracle import farfield
from oracle import solve as osolve
from workloads import geometry, incident

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_1810_07067_amd as msv  # noqa: E402


def make_plan(curve, k0, eps1, M, L, precision=0, mu1=1.0):
    print(f"[case] {curve.name} N={curve.n} k0={k0} eps1={eps1} M={M} L={L} prec={precision}", flush=True)
    return msv.plan_from_curve(curve, RULES, k0, eps1, mu1, m_max=M, fft_len=L, precision=precision)


@pytest.fixture(scope="module")
def sphere():
    curve = geometry.sphere(8)
    k0, eps1, M, L = 1.0, 2.25, 16, 64
    sup, kp = oracle_setup(curve, k0, eps1, M, L)
    tab = oracle_table(curve, sup, kp)
    plan = make_plan(curve, k0, eps1, M, L)
    kern = plan.tabulate()
    torch.cuda.synchronize()
    return dict(curve=curve, k0=k0, eps1=eps1, M=M, L=L, sup=sup, kp=kp, tab=tab, plan=plan, kern=kern)


def test_sphere_table_parity(sphere):
    got = sphere["kern"].cpu().numpy()
    ref = sphere["tab"]
    assert got.shape == ref.shape
    err, zero_bad = normwise_table_error(got, ref)
    assert zero_bad == 0.0
    assert err < 1e-12, err


def test_sphere_matrix_parity(sphere):
    s = sphere
    A = s["plan"].assemble(s["kern"], 0, s["M"])
    torch.cuda.synchronize()
    Ag = A.cpu().numpy()
    for m in (0, 1, 2, 7, s["M"]):
        Ar = oracle_matrix(s["curve"], s["sup"], s["tab"], m, s["k0"], s["kp"].k1, s["eps1"])
        scale = np.max(np.abs(Ar))
        assert np.max(np.abs(Ag[m] - Ar)) < 1e-12 * scale, m


@pytest.mark.parametrize("precision", [0, 1])
def test_sphere_solution_and_far_field(sphere, precision):
    s = sphere
    curve, M, k0 = s["curve"], s["M"], s["k0"]
    plan = make_plan(curve, k0, s["eps1"], M, s["L"], precision=precision)
    kern = plan.tabulate()
    A = plan.assemble(kern, 0, M)
    Aref = [oracle_matrix(curve, s["sup"], s["tab"], m, k0, s["kp"].k1, s["eps1"]) for m in range(M + 1)]
    plan.factor(A, 0, M)
    d, p = incident.tilted_direction(30.0)
    rhs = incident.rhs_modes(curve, [(d, p)], k0, -M, M)
    x = plan.solve(-M, M, torch.from_numpy(rhs).cuda())
    torch.cuda.synchronize()
    xg = x.cpu().numpy()
    w = geometry.gl_weights(curve)
    xr = osolve.solve_modes(Aref, w, rhs, -M, M)
    assert np.max(np.abs(xg - xr)) < 1e-10 * np.max(np.abs(xr))
    dirs = np.array([[0.3, 0.4, np.sqrt(0.75)], [-0.6, 0.0, 0.8], [0.0, -1.0, 0.0]])
    Eg = farfield.far_field(curve, w, xg[:, 0], -M, k0, k0, 1.0, dirs)
    Er = farfield.far_field(curve, w, xr[:, 0], -M, k0, k0, 1.0, dirs)
    assert np.max(np.abs(Eg - Er)) < 1e-10 * np.max(np.abs(Er))
    if precision == 1:
        assert 1 <= plan.last_ir_iterations() <= 10


def test_negative_modes_use_parity(sphere):
    """Solving mode -m with the factors of m equals solving the directly
    assembled A_{-m} (oracle)."""
    s = sphere
    curve, M, k0 = s["curve"], s["M"], s["k0"]
    plan = s["plan"]
    A = plan.assemble(s["kern"], 0, 3)
    plan.factor(A, 0, 3)
    rng = np.random.default_rng(7)
    n = 4 * curve.n
    b = rng.standard_normal((7, 2, n)) + 1j * rng.standard_normal((7, 2, n))
    x = plan.solve(-3, 3, torch.from_numpy(b).cuda()).cpu().numpy()
    w = geometry.gl_weights(curve)
    mats = [oracle_matrix(curve, s["sup"], s["tab"], m, k0, s["kp"].k1, s["eps1"]) for m in range(4)]
    xr = osolve.solve_modes(mats, w, b, -3, 3)
    assert np.max(np.abs(x - xr)) < 1e-10 * np.max(np.abs(xr))


@pytest.mark.parametrize("which", ["torus", "cylinder", "spheroid_c3"])
def test_other_bodies_table_and_matrix(which):
    """Closed curve, corners with dyadic refinement, complex k1, elongated body."""
    if which == "torus":
        curve, k0, eps1, M, L = geometry.torus(6), 2.0, 3.0, 8, 128
    elif which == "cylinder":
        curve, k0, eps1, M, L = geometry.polygon([(0.0, -1.0), (1.0, -1.0), (1.0, 1.0), (0.0, 1.0)],
                                                 2.0, 6, "cylinder_small"), 3.0, 4.0 + 0.1j, 8, 128
    else:
        curve, k0, eps1, M, L = geometry.spheroid(6, 3.0), 2.0, 4.0, 10, 128
    sup, kp = oracle_setup(curve, k0, eps1, M, L)
    rows = np.array([0, 5, curve.n // 2, curve.n - 1])
    tab = oracle_table(curve, sup, kp, rows=rows)
    plan = make_plan(curve, k0, eps1, M, L)
    kern = plan.tabulate()
    A = plan.assemble(kern, 0, M)
    torch.cuda.synchronize()
    got = kern.cpu().numpy()[:, :, rows, :]
    err, zero_bad = normwise_table_error(got, tab)
    assert zero_bad == 0.0 and err < 1e-12, err
    Ag = A.cpu().numpy()
    for m in (0, 1, M):
        Ar = oracle_matrix(curve, sup, tab, m, k0, kp.k1, eps1, rows=rows)
        rsel = np.concatenate([np.arange(4 * t, 4 * t + 4) for t in rows])
        assert np.max(np.abs(Ag[m][rsel] - Ar)) < 1e-12 * np.max(np.abs(Ar)), (which, m)
