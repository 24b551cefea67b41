"""The allocation-free solve (msv_solve_noalloc) through the C-ABI against
msv_solve: two calls in a row on the shared static workspace, the second
smaller than the first, in both precisions; a call that needs more workspace
than the static array is refused; and the calls allocate no device memory."""
import numpy as np
import pytest

from gpu_cases import RULES
from workloads import geometry, incident

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_1810_07067_amd as msv  # noqa: E402


@pytest.mark.parametrize("precision", [0, 1])
def test_noalloc_solve_matches_msv_solve(precision):
    curve, k0, eps1, M, L = geometry.spheroid(8, 2.0), 2.0, 3.0 + 0.1j, 8, 64
    print(f"[noalloc] {curve.name} N={curve.n} M={M} precision={precision}", flush=True)
    p = msv.plan_from_curve(curve, RULES, k0, eps1, 1.0, m_max=M, fft_len=L, precision=precision,
                            ir_tol=1e-13, ir_max_iter=20)
    A = p.assemble(p.tabulate(), 0, M)
    p.factor(A, 0, M)
    calls = [(-M, M, [incident.tilted_direction(a) for a in (10.0, 50.0, 100.0, 160.0)]),
             (2, 5, [incident.tilted_direction(70.0)])]  # the second call is smaller
    ins = [torch.from_numpy(incident.rhs_modes(curve, w, k0, lo, hi)).cuda() for lo, hi, w in calls]
    refs = [p.solve(lo, hi, b).cpu().numpy() for (lo, hi, _), b in zip(calls, ins)]
    outs = [torch.empty_like(b) for b in ins]
    torch.cuda.synchronize()
    held = p.device_bytes
    free0 = torch.cuda.mem_get_info()[0]
    for (lo, hi, _), b, o in zip(calls, ins, outs):
        p.solve_noalloc(lo, hi, b, o)
    torch.cuda.synchronize()
    free1 = torch.cuda.mem_get_info()[0]
    assert p.device_bytes == held
    assert abs(free1 - free0) <= (2 << 20), (free0, free1)
    for (lo, hi, _), o, ref in zip(calls, outs, refs):
        got = o.cpu().numpy()
        err = np.max(np.abs(got - ref)) / np.max(np.abs(ref))
        print(f"[noalloc] modes {lo}..{hi}: max |noalloc - msv_solve| / max = {err:.2e}", flush=True)
        assert err <= 1e-14, (lo, hi, err)
    p.close()


def test_noalloc_refuses_oversize_solve():
    curve, k0, eps1, M, L = geometry.sphere(16), 1.0, 2.25, 8, 64
    p = msv.plan_from_curve(curve, RULES, k0, eps1, 1.0, m_max=M, fft_len=L, precision=1)
    A = p.assemble(p.tabulate(), 0, M)
    p.factor(A, 0, M)
    cap = int(p.lib.msv_solve_noalloc_max_bytes())
    # (2M+1) modes x n_rhs vectors of order 1024 at 64 bytes per element exceed the array
    n_rhs = cap // ((2 * M + 1) * p.n * 64) + 2
    b = torch.zeros((2 * M + 1, n_rhs, p.n), dtype=torch.complex128, device="cuda")
    o = torch.empty_like(b)
    with pytest.raises(msv.MsvError) as e:
        p.solve_noalloc(-M, M, b, o)
    assert e.value.status == msv.MSV_EINVAL and "workspace" in str(e.value)
    p.close()
