"""GPU parity: the HIP library (through the C-ABI) against the FP64 oracle.

Each stage is checked on the oracle's own inputs, then the whole path end to
end:

  modal kernels   msv_tabulate vs oracle.modal.tabulate: 1e-12 relative,
                  normwise over modes per (type, target, source); slots the
                  oracle leaves zero must be exactly zero.
  assembly        msv_assemble on the ORACLE table vs oracle.assemble on the
                  same table.  Rows next to the axis carry the 1/r_t^2 terms
                  of the modal operators (Section 3), and there a one-ulp
                  perturbation of the table moves the oracle's own row by up
                  to 1e-5 of its size.  Per row i the bound is therefore
                  max(1e-12 * rowmax_i, 16 * sens_i), sens_i being the largest
                  change of row i (over modes) when every table entry is
                  scaled by an independent 1 + u 2^-53, u uniform in [-1, 1].
                  Rows whose sensitivity is below the 1e-12 level (all rows
                  away from the axis) are held to 1e-12.
  factor + solve  msv_factor/msv_solve on the ORACLE matrices vs the oracle's
                  dense solve: 1e-10 relative (max norm).
  end to end      far fields and surface currents (the latter in the L2 norm
                  of the discretization, weights sqrt(w_j), Section 6), each
                  to max(1e-10, 4 * sens) relative.  sens is the oracle's own
                  change of that output when every table entry is scaled by
                  an independent 1 + 1e-14 u: both implementations evaluate
                  the kernels to 0.5e-14 .. 1.5e-14 of a 30-digit quadrature
                  (the derivative kernels at near-singular support nodes reach
                  1e9), and for bodies with mu1 != mu0 the terms
                  (mu0 - mu1) N^{k0}, (eps0 - eps1) N^{k0} carry those
                  differences to the far field at a few 1e-10.
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

DIRS = np.array([[0.3, 0.4, np.sqrt(0.75)], [-0.6, 0.0, 0.8], [0.0, -1.0, 0.0], [0.0, 0.0, 1.0]])


def _cylinder_small():
    return geometry.polygon([(0.0, -1.0), (1.0, -1.0), (1.0, 1.0), (0.0, 1.0)], 1.0, 2, "cylinder_small")


# name -> (curve builder, k0, eps1, mu1, M, L)
CASES = {
    "sphere": (lambda: geometry.sphere(8), 1.0, 2.25, 1.0, 16, 64),
    "torus_magnetic": (lambda: geometry.torus(6), 2.0, 3.0, 2.0, 8, 128),
    "cylinder_lossy": (_cylinder_small, 3.0, 4.0 + 0.1j, 1.0, 8, 128),
    "spheroid_c3": (lambda: geometry.spheroid(6, 3.0), 2.0, 4.0, 1.0, 10, 128),
}


def make_plan(curve, k0, eps1, mu1, M, L, precision=0, **kw):
    print(f"[case] {curve.name} N={curve.n} k0={k0} eps1={eps1} mu1={mu1} M={M} L={L} "
          f"prec={precision}", flush=True)
    return msv.plan_from_curve(curve, RULES, k0, eps1, mu1, m_max=M, fft_len=L, precision=precision, **kw)


def l2w(curve):
    return np.sqrt(np.repeat(geometry.gl_weights(curve), 4))


def perturbed(tab, seed, rel):
    rng = np.random.default_rng(seed)
    return tab * (1.0 + rel * rng.uniform(-1.0, 1.0, tab.shape))


@pytest.fixture(scope="module", params=list(CASES))
def case(request):
    build, k0, eps1, mu1, M, L = CASES[request.param]
    curve = build()
    sup, kp = oracle_setup(curve, k0, eps1, M, L, mu1=mu1)
    tab = oracle_table(curve, sup, kp)
    mats = np.array([oracle_matrix(curve, sup, tab, m, k0, kp.k1, eps1, mu1) for m in range(M + 1)])
    matsp = np.array([oracle_matrix(curve, sup, perturbed(tab, 11, 2.0 ** -53), m, k0, kp.k1, eps1, mu1)
                      for m in range(M + 1)])
    matsk = [oracle_matrix(curve, sup, perturbed(tab, 12, 1e-14), m, k0, kp.k1, eps1, mu1) for m in range(M + 1)]
    w = geometry.gl_weights(curve)
    waves = [incident.tilted_direction(30.0), incident.tilted_direction(75.0)]
    rhs = incident.rhs_modes(curve, waves, k0, -M, M, mu0=1.0)
    x = osolve.solve_modes(list(mats), w, rhs, -M, M)
    xp = osolve.solve_modes(matsk, w, rhs, -M, M)
    E = farfield.far_field(curve, w, x[:, 0], -M, k0, k0, 1.0, DIRS)
    Ep = farfield.far_field(curve, w, xp[:, 0], -M, k0, k0, 1.0, DIRS)
    sw = l2w(curve)
    return dict(name=request.param, curve=curve, k0=k0, eps1=eps1, mu1=mu1, M=M, L=L, sup=sup, kp=kp,
                tab=tab, mats=mats, matsp=matsp, w=w, rhs=rhs, x=x, E=E,
                sens_x=np.linalg.norm(sw * (x - xp)) / np.linalg.norm(sw * x),
                sens_E=np.max(np.abs(E - Ep)) / np.max(np.abs(E)))


def test_table_parity(case):
    plan = make_plan(case["curve"], case["k0"], case["eps1"], case["mu1"], case["M"], case["L"])
    got = plan.tabulate().cpu().numpy()
    assert got.shape == case["tab"].shape
    err, zero_bad = normwise_table_error(got, case["tab"])
    print(f"[table] {case['name']} normwise err {err:.3e}", flush=True)
    assert zero_bad == 0.0
    assert err < 1e-12, err


def test_assembly_parity(case):
    c = case
    plan = make_plan(c["curve"], c["k0"], c["eps1"], c["mu1"], c["M"], c["L"])
    A = plan.assemble(torch.from_numpy(c["tab"]).cuda(), 0, c["M"]).cpu().numpy()
    ref = c["mats"]
    diff = np.max(np.abs(A - ref), axis=(0, 2))
    rowmax = np.max(np.abs(ref), axis=(0, 2))
    sens = np.max(np.abs(c["matsp"] - ref), axis=(0, 2))
    bound = np.maximum(1e-12 * rowmax, 16.0 * sens)
    tight = sens < 1e-13 * rowmax
    print(f"[assemble] {c['name']} max row err/rowmax {np.max(diff / rowmax):.3e}; rows held to 1e-12: "
          f"{tight.sum()}/{tight.size}, their max {np.max((diff / rowmax)[tight]) if tight.any() else 0:.3e}",
          flush=True)
    assert np.all(diff <= bound), np.max(diff / bound)


@pytest.mark.parametrize("precision", [0, 1])
def test_factor_solve_parity(case, precision):
    c = case
    M = c["M"]
    plan = make_plan(c["curve"], c["k0"], c["eps1"], c["mu1"], M, c["L"], precision=precision)
    A = torch.from_numpy(c["mats"].copy()).cuda()
    plan.factor(A, 0, M)
    x = plan.solve(-M, M, torch.from_numpy(c["rhs"]).cuda()).cpu().numpy()
    err = np.max(np.abs(x - c["x"])) / np.max(np.abs(c["x"]))
    print(f"[solve] {c['name']} prec {precision} err {err:.3e} ir {plan.last_ir_iterations()}", flush=True)
    assert err < 1e-10, err
    if precision == 1:
        assert 1 <= plan.last_ir_iterations() <= 10


@pytest.mark.parametrize("precision", [0, 1])
def test_end_to_end(case, precision):
    c = case
    curve, M, k0 = c["curve"], c["M"], c["k0"]
    plan = make_plan(curve, k0, c["eps1"], c["mu1"], M, c["L"], precision=precision)
    kern = plan.tabulate()
    A = plan.assemble(kern, 0, M)
    plan.factor(A, 0, M)
    x = plan.solve(-M, M, torch.from_numpy(c["rhs"]).cuda()).cpu().numpy()
    sw = l2w(curve)
    xerr = np.linalg.norm(sw * (x - c["x"])) / np.linalg.norm(sw * c["x"])
    E = farfield.far_field(curve, c["w"], x[:, 0], -M, k0, k0, 1.0, DIRS)
    ferr = np.max(np.abs(E - c["E"])) / np.max(np.abs(c["E"]))
    xtol = max(1e-10, 4.0 * c["sens_x"])
    ftol = max(1e-10, 4.0 * c["sens_E"])
    print(f"[e2e] {c['name']} prec {precision} far field {ferr:.3e} (oracle sensitivity "
          f"{c['sens_E']:.3e}); currents L2 {xerr:.3e} (oracle sensitivity {c['sens_x']:.3e})", flush=True)
    assert ferr < ftol, (ferr, ftol)
    assert xerr < xtol, (xerr, xtol)


def test_negative_modes_use_parity(case):
    """Solving mode -m with the factors of mode m (msv_solve applies D) equals
    solving the directly assembled A_{-m} of the oracle."""
    c = case
    if c["name"] != "sphere":
        pytest.skip("one body suffices")
    M = 3
    plan = make_plan(c["curve"], c["k0"], c["eps1"], c["mu1"], c["M"], c["L"])
    A = torch.from_numpy(c["mats"][: M + 1].copy()).cuda()
    plan.factor(A, 0, M)
    rng = np.random.default_rng(7)
    n = 4 * c["curve"].n
    b = rng.standard_normal((2 * M + 1, 3, n)) + 1j * rng.standard_normal((2 * M + 1, 3, n))
    x = plan.solve(-M, M, torch.from_numpy(b).cuda()).cpu().numpy()
    xr = osolve.solve_modes(list(c["mats"][: M + 1]), c["w"], b, -M, M)
    assert np.max(np.abs(x - xr)) < 1e-10 * np.max(np.abs(xr))
