"""The boundary's resource contract on the GPU, through the C-ABI:

  workspace   msv_workspace_bytes bounds what a plan allocates, and
              msv_plan_device_bytes matches the device memory that disappears
              while a plan is created, factored and solved;
  streams     back-to-back solves of different mode ranges on one non-default
              stream, with no host wait between them, give the results of the
              same solves run one at a time (the solve's batch table is written
              in stream order);
  pinning     a batch pins its plans: factoring more modes than the batch
              holds is refused, and destroying a plan before its batch defers
              the free until the batch goes.
  allocator   with msv_set_allocator routing the library's buffers through
              torch's caching allocator, the plan's storage is counted by
              torch while the plan lives and handed back when it is destroyed,
              the solution equals the one on hipMalloc'd storage, and the hooks
              cannot change while a plan exists.
"""
import gc

import numpy as np
import pytest

from gpu_cases import RULES
from workloads import geometry, incident

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_1810_07067_amd as msv  # noqa: E402


def make(curve, k0, eps1, M, L, precision):
    print(f"[case] {curve.name} N={curve.n} M={M} L={L} prec={precision}", flush=True)
    return msv.plan_from_curve(curve, RULES, k0, eps1, 1.0, m_max=M, fft_len=L, precision=precision,
                               ir_tol=1e-13, ir_max_iter=20)


def free_bytes():
    torch.cuda.synchronize()
    return torch.cuda.mem_get_info()[0]


@pytest.mark.parametrize("precision", [0, 1])
def test_workspace_bytes_bound_allocations(precision):
    curve, k0, eps1, M, L = geometry.sphere(16), 2.0, 2.25, 8, 64
    p = make(curve, k0, eps1, M, L, precision)
    A = p.assemble(p.tabulate(), 0, M)
    waves = [incident.tilted_direction(a) for a in (20.0, 80.0, 140.0)]
    rhs = torch.from_numpy(incident.rhs_modes(curve, waves, k0, -M, M)).cuda()
    x = torch.empty_like(rhs)
    A2 = A.clone()
    before = free_bytes()
    q = make(curve, k0, eps1, M, L, precision)
    q.factor(A2, 0, M)
    q.solve(-M, M, rhs, out=x)
    after = free_bytes()
    held = q.device_bytes
    bound = msv.workspace_bytes(q.N, q.S, L, M + 1, (2 * M + 1) * len(waves), precision)
    print(f"[workspace] held {held} bound {bound} device delta {before - after}", flush=True)
    spec_max = min(q.N * (q.N + q.S), 262144) * (L // 2 + 1) * 16  # spectra scratch if every pair were near
    assert held <= bound <= held + 8 * q.N * (q.N + q.S) + spec_max + (M + 1) * 72 + 256
    # the runtime rounds allocations up; each of ~30 buffers by at most 2 MiB
    assert 0.98 * held <= before - after <= held + (64 << 20)
    q.close()


@pytest.mark.parametrize("precision", [0, 1])
def test_back_to_back_solves_on_a_side_stream(precision):
    curve, k0, eps1, M, L = geometry.spheroid(8, 2.0), 2.0, 3.0 + 0.1j, 6, 64
    p = make(curve, k0, eps1, M, L, precision)
    A = p.assemble(p.tabulate(), 0, M)
    p.factor(A, 0, M)
    waves = [incident.tilted_direction(a) for a in (10.0, 60.0)]
    ranges = [(-M, M), (2, 4), (-3, -1), (0, 0)]
    rhs = [torch.from_numpy(incident.rhs_modes(curve, waves, k0, lo, hi)).cuda() for lo, hi in ranges]
    alone = []
    for (lo, hi), b in zip(ranges, rhs):
        alone.append(p.solve(lo, hi, b).cpu().numpy())
        torch.cuda.synchronize()
    s = torch.cuda.Stream()
    outs = [torch.empty_like(b) for b in rhs]
    with torch.cuda.stream(s):
        for (lo, hi), b, o in zip(ranges, rhs, outs):
            p.solve(lo, hi, b, out=o, stream=s)
    s.synchronize()
    for (lo, hi), o, ref in zip(ranges, outs, alone):
        err = np.max(np.abs(o.cpu().numpy() - ref)) / np.max(np.abs(ref))
        print(f"[streams] modes {lo}..{hi}: {err:.2e}", flush=True)
        assert err < 1e-12, (lo, hi, err)


def test_batch_pins_its_plans():
    M = 2
    plans, mats = [], []
    for curve, k0, eps1 in ((geometry.sphere(8), 1.0, 2.25), (geometry.spheroid(4, 2.0), 1.5, 3.0)):
        p = make(curve, k0, eps1, 3, 64, 1)
        plans.append(p)
        mats.append(p.assemble(p.tabulate(), 0, M))
    batch = msv.Batch(plans, mats, 0, M)
    p0 = plans[0]
    A3 = p0.assemble(p0.tabulate(), 0, 3)
    with pytest.raises(msv.MsvError) as e:
        p0.factor(A3, 0, 3)  # would grow the factor storage the batch's graph points into
    assert e.value.status == msv.MSV_EINVAL and "batch" in str(e.value)
    p0.factor(A3[:M + 1].contiguous(), 0, M)  # within the batch's storage: allowed
    # destroy a plan before its batch: deferred, the replay still runs on live storage
    held = plans[1].device_bytes
    plans[1].close()
    batch.factor()
    torch.cuda.synchronize()
    before = free_bytes()
    batch.close()
    after = free_bytes()
    print(f"[pinning] plan held {held} B; freed at batch destroy {after - before} B", flush=True)
    assert after - before >= 0.9 * held


def test_plans_allocate_from_a_caller_pool():
    curve, k0, eps1, M, L = geometry.sphere(8), 1.0, 2.25, 16, 64
    d, p = incident.tilted_direction(30.0)
    rhs = torch.from_numpy(incident.rhs_modes(curve, [(d, p)], k0, -M, M)).cuda()

    def run():
        plan = make(curve, k0, eps1, M, L, 1)
        A = plan.assemble(plan.tabulate(), 0, M)
        x = torch.empty_like(rhs)
        torch.cuda.synchronize()
        before = torch.cuda.memory_allocated()
        plan.factor(A, 0, M)
        plan.solve(-M, M, rhs, out=x)
        torch.cuda.synchronize()
        return plan, x, torch.cuda.memory_allocated() - before

    gc.collect()
    msv.use_torch_allocator(False)
    p0, x0, grown0 = run()
    p0.close()
    msv.use_torch_allocator(True)
    try:
        p1, x1, grown1 = run()
        with pytest.raises(msv.MsvError):
            msv.use_torch_allocator(False)  # a plan is alive
        live = torch.cuda.memory_allocated()
        p1.close()
        freed = live - torch.cuda.memory_allocated()
    finally:
        gc.collect()
        msv.use_torch_allocator(False)
    n = 4 * curve.n
    fac = (M + 1) * n * n * 8  # the complex64 factors alone
    diff = float((x1 - x0).abs().max() / x0.abs().max())
    print(f"[allocator] torch counts {grown1} B for the factor and solve (hipMalloc: {grown0} B), "
          f"{freed} B back at destroy; solutions differ by {diff:.1e}", flush=True)
    assert grown0 == 0
    assert grown1 >= fac
    assert freed >= grown1
    assert diff < 1e-14
