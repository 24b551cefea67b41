"""GPU edge cases and full-size checks through the C-ABI.

  ragged      N = 112 nodes (448 unknowns per mode: not a multiple of the LU's
              128-column panels or 64-row tiles), 3 right-hand sides (the
              triangular solves take 8 per workgroup), a factored mode range
              that starts above 0 and single-mode solves.
  degenerate  a single azimuthal mode (m_max = 0).
  past 8192   orders 8768 and 12288 (the largest the plan accepts), where the
              LU's panel strips hold 12 rows per thread: seeded matrices in
              both precisions, the residual of each solve and the two
              solutions against each other; N = 3088 is refused.
  (4N = 8192 and the full-size workloads are in test_gpu_fullsize.py.)
  staggered   five modes of order 4416 factored by one call (two halves on
              two streams) against one mode per call.
  errors      invalid calls return EINVAL and leave the plan usable.
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

DIRS = np.array([[0.3, 0.4, np.sqrt(0.75)], [-0.6, 0.0, 0.8], [0.0, -1.0, 0.0]])


def make_plan(curve, k0, eps1, mu1, M, L, precision=0, **kw):
    print(f"[case] {curve.name} N={curve.n} k0={k0} eps1={eps1} M={M} L={L} prec={precision}", flush=True)
    return msv.plan_from_curve(curve, RULES, k0, eps1, mu1, m_max=M, fft_len=L, precision=precision, **kw)


def l2w(curve):
    return np.sqrt(np.repeat(geometry.gl_weights(curve), 4))


def power_balance(curve, x):
    """Net power into a lossless body, relative: pi sum_m int Re(M2 J1* - M1 J2*) r ds."""
    X = x.reshape(x.shape[0], curve.n, 4)
    J1, J2, M1, M2 = (X[:, :, i] for i in range(4))
    rw = curve.r * geometry.gl_weights(curve)
    P = np.pi * np.sum(np.real(M2 * np.conj(J1) - M1 * np.conj(J2)) * rw[None, :])
    scale = np.pi * np.sum((np.abs(J1) + np.abs(J2)) * (np.abs(M1) + np.abs(M2)) * rw[None, :])
    return abs(P) / scale


@pytest.mark.parametrize("precision", [0, 1])
def test_ragged_sizes_and_mode_ranges(precision):
    curve, k0, eps1, M, L = geometry.sphere(7), 1.5, 2.0 + 0.05j, 5, 64
    sup, kp = oracle_setup(curve, k0, eps1, M, L)
    tab = oracle_table(curve, sup, kp)
    mats = [oracle_matrix(curve, sup, tab, m, k0, kp.k1, eps1) for m in range(M + 1)]
    w = geometry.gl_weights(curve)
    plan = make_plan(curve, k0, eps1, 1.0, M, L, precision=precision)
    err, zero_bad = normwise_table_error(plan.tabulate().cpu().numpy(), tab)
    assert zero_bad == 0.0 and err < 1e-12, err
    A = torch.from_numpy(np.array(mats[2:]).copy()).cuda()
    plan.factor(A, 2, M)
    waves = [incident.tilted_direction(a) for a in (10.0, 50.0, 120.0)]
    for lo, hi in ((-M, -2), (2, M), (3, 3), (-4, -4)):
        rhs = incident.rhs_modes(curve, waves, k0, lo, hi)
        x = plan.solve(lo, hi, torch.from_numpy(rhs).cuda()).cpu().numpy()
        xr = osolve.solve_modes(mats, w, rhs, lo, hi)
        err = np.max(np.abs(x - xr)) / np.max(np.abs(xr))
        print(f"[ragged] modes {lo}..{hi} err {err:.3e}", flush=True)
        assert err < 1e-10, (lo, hi, err)


def test_ragged_row_blocks_reproduce_the_table_and_matrices():
    """Row blocks of 48 target rows (the last one 16) tabulate the same table,
    and assemble the same matrices, bit for bit as the whole table."""
    curve = geometry.sphere(7)
    plan = make_plan(curve, 1.5, 2.0 + 0.05j, 1.0, 5, 64, precision=1)
    full = plan.tabulate()
    parts = [plan.tabulate_rows(t0, min(48, curve.n - t0)) for t0 in range(0, curve.n, 48)]
    assert torch.equal(torch.cat(parts, dim=2), full)
    A_full = plan.assemble(full, 0, 5)
    A_blocks = plan.assemble_streamed(0, 5, rows_per_block=48)
    assert torch.equal(A_blocks, A_full)
    A_default = plan.assemble_streamed(0, 5)  # 128-row blocks: one block for 112 nodes
    assert torch.equal(A_default, A_full)


def test_single_mode():
    curve, k0, eps1, M, L = geometry.sphere(7), 0.5, 3.0, 0, 32
    sup, kp = oracle_setup(curve, k0, eps1, M, L)
    tab = oracle_table(curve, sup, kp)
    A0 = oracle_matrix(curve, sup, tab, 0, k0, kp.k1, eps1)
    plan = make_plan(curve, k0, eps1, 1.0, M, L)
    kern = plan.tabulate()
    err, zero_bad = normwise_table_error(kern.cpu().numpy(), tab)
    assert zero_bad == 0.0 and err < 1e-12, err
    A = plan.assemble(kern, 0, 0)
    plan.factor(A, 0, 0)
    rhs = incident.rhs_modes(curve, [incident.tilted_direction(40.0)], k0, 0, 0)
    x = plan.solve(0, 0, torch.from_numpy(rhs).cuda()).cpu().numpy()
    w = geometry.gl_weights(curve)
    xr = osolve.solve_modes([A0], w, rhs, 0, 0)
    E = farfield.far_field(curve, w, x[:, 0], 0, k0, k0, 1.0, DIRS)
    Er = farfield.far_field(curve, w, xr[:, 0], 0, k0, k0, 1.0, DIRS)
    assert np.max(np.abs(E - Er)) < 1e-10 * np.max(np.abs(Er))


def test_invalid_calls_raise_einval():
    curve = geometry.sphere(4)
    plan = make_plan(curve, 1.0, 2.25, 1.0, 3, 32)
    kern = plan.tabulate()

    def einval(fn):
        with pytest.raises(msv.MsvError) as e:
            fn()
        assert e.value.status == msv.MSV_EINVAL

    n = plan.n
    einval(lambda: plan.tabulate(out=torch.empty(10, dtype=torch.complex128, device="cuda")))
    einval(lambda: plan.assemble(kern, 2, 4))          # m_hi > m_max
    rhs = torch.zeros((1, 1, n), dtype=torch.complex128, device="cuda")
    einval(lambda: plan.solve(0, 0, rhs))             # nothing factored yet
    A = plan.assemble(kern, 1, 2)
    plan.factor(A, 1, 2)
    einval(lambda: plan.solve(0, 0, rhs))             # mode 0 not factored
    einval(lambda: plan.solve(3, 3, rhs))             # mode 3 not factored
    einval(lambda: plan.solve(1, 1, torch.zeros((1, 0, n), dtype=torch.complex128, device="cuda")))
    # the plan still works after the errors
    x = plan.solve(-2, -1, torch.ones((2, 1, n), dtype=torch.complex128, device="cuda"))
    assert torch.isfinite(torch.view_as_real(x)).all()


def _seeded_system(n, seed=7):
    """Complex Gaussian entries over sqrt(n), plus 1.5 on a random permutation
    of the diagonal positions (condition ~5, every column needs an
    interchange), and one right-hand side."""
    g = torch.Generator(device="cuda")
    g.manual_seed(seed)
    A = torch.randn((1, n, n), dtype=torch.complex128, device="cuda", generator=g)
    A.mul_(1.0 / np.sqrt(n))
    perm = torch.randperm(n, device="cuda", generator=g)
    A[0, perm, torch.arange(n, device="cuda")] += 1.5
    b = torch.randn((1, 1, n), dtype=torch.complex128, device="cuda", generator=g)
    return A, b


@pytest.mark.parametrize("n_nodes", [2192, 3072])
def test_orders_past_8192(n_nodes):
    """A seeded matrix of order 4 n_nodes factored with the complex64 LU +
    refinement and with the complex128 LU: each solution's relative residual
    (of the weighted system the solve works on) below 1e-12, the two within
    1e-10 of each other."""
    curve = geometry.sphere(n_nodes // 16)
    p1 = make_plan(curve, 1.0, 2.0, 1.0, 0, 64, precision=1)
    n = p1.n
    assert n == 4 * n_nodes
    A, b = _seeded_system(n)
    # the library solves the L2-weighted system: sqrt(w) x from sqrt(w) b
    sw = torch.from_numpy(l2w(curve)).cuda()
    rel = lambda M, x: (torch.linalg.vector_norm(sw * b[0, 0] - M[0] @ (sw * x[0, 0]))
                        / torch.linalg.vector_norm(sw * b[0, 0])).item()
    p1.factor(A, 0, 0)  # complex64 factors of their own; A is kept
    x1 = p1.solve(0, 0, b)
    r1 = rel(A, x1)
    print(f"[order {n}] complex64 + refinement: residual {r1:.3e} after {p1.last_ir_iterations()} steps",
          flush=True)
    p1.close()
    p0 = make_plan(curve, 1.0, 2.0, 1.0, 0, 64, precision=0)
    p0.factor(A, 0, 0)  # the complex128 LU factors A in place
    x0 = p0.solve(0, 0, b)
    p0.close()
    A, _ = _seeded_system(n)
    r0 = rel(A, x0)
    d = (torch.linalg.vector_norm(x0 - x1) / torch.linalg.vector_norm(x0)).item()
    print(f"[order {n}] complex128: residual {r0:.3e}; the solutions differ by {d:.3e}", flush=True)
    assert r1 < 1e-12 and r0 < 1e-12, (r1, r0)
    assert d < 1e-10, d


@pytest.mark.parametrize("precision", [0, 1])
def test_staggered_factorization_matches_one_mode_at_a_time(precision):
    """Five seeded matrices of order 4416 (above the order from which a plan
    staggers its factorization) factored by one call (two halves of 3 and 2
    on two streams, the second half's panels after the first's, the last
    outer panels narrower than the others) and one mode per call (one
    stream): complex128 solutions bit-identical, complex64 + refinement within
    1e-12 of each other."""
    curve = geometry.sphere(69)
    plan = make_plan(curve, 1.0, 2.0, 1.0, 4, 64, precision=precision)
    n = plan.n
    assert n == 4416
    mats, rhs = zip(*(_seeded_system(n, seed=20 + m) for m in range(5)))
    A = torch.cat(mats)
    b = torch.cat(rhs)
    A_all = A.clone()  # the complex128 LU factors in place; the plan keeps the buffer
    plan.factor(A_all, 0, 4)
    x_all = plan.solve(0, 4, b)
    for m in range(5):
        A_one = A[m:m + 1].clone()
        plan.factor(A_one, m, m)
        x_one = plan.solve(m, m, b[m:m + 1])
        d = (torch.linalg.vector_norm(x_one[0] - x_all[m]) / torch.linalg.vector_norm(x_all[m])).item()
        print(f"[stagger] precision {precision} mode {m}: difference {d:.3e}", flush=True)
        if precision == 0:
            assert torch.equal(x_one[0], x_all[m]), (m, d)
        else:
            assert d < 1e-12, (m, d)


def test_order_past_12288_is_refused():
    with pytest.raises(msv.MsvError) as exc:
        make_plan(geometry.sphere(193), 1.0, 2.0, 1.0, 0, 64)
    assert exc.value.status == msv.MSV_EINVAL
