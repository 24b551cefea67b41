"""Serving form on the GPU: every request's currents are the same when it is
served alone and when it is served in a Poisson mix with other requests
(overlapping on four streams, factorizations shared through the cache), also
under a memory budget that forces evictions; each is checked against the plain
complex128 path of its body."""
import numpy as np
import pytest

from gpu_cases import RULES
from workloads import geometry, incident

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_1810_07067_amd.serve import Request, Server, entry_bytes, latency_stats, poisson_arrivals  # noqa: E402

BODIES = {
    "sphere": (geometry.sphere(4), 1.0, 2.25, 6, 64),
    "spheroid": (geometry.spheroid(4, 2.0), 1.5, 3.0, 5, 64),
    "torus": (geometry.torus(4), 1.0, 2.0 + 0.05j, 4, 64),
}


def make_requests(seed=11, count=12, qps=200.0):
    rng = np.random.default_rng(seed)
    names = list(BODIES)
    t = poisson_arrivals(rng, count, qps)
    reqs = []
    for i in range(count):
        name = names[rng.integers(len(names))]
        curve, k0, eps1, M, L = BODIES[name]
        nw = int(rng.integers(1, 5))
        waves = incident.random_directions(int(rng.integers(1 << 30)), nw)
        reqs.append(Request(i, name, curve, k0, eps1, M, L, waves, float(t[i])))
    return reqs


def one_body_budget():
    """Room for the largest body while it is built, and for no second one."""
    S = RULES[0][0].shape[1] + 2 * RULES[1][0].size
    return max(sum(entry_bytes(c, M, L, 1, S)) for c, _, _, M, L in BODIES.values())


def test_results_alone_equal_results_in_the_mix():
    reqs = make_requests()
    alone = {}
    for r in reqs:
        srv = Server(RULES, hbm_budget=8 << 30, slots=1)
        res, _ = srv.run([Request(r.rid, r.body, r.curve, r.k0, r.eps1, r.m_max, r.fft_len, r.waves, 0.0)],
                         realtime=False)
        alone[r.rid] = res[r.rid].x
    srv = Server(RULES, hbm_budget=8 << 30, slots=4)
    mix, wall = srv.run(reqs, realtime=True)
    st = latency_stats(mix)
    print(f"[serve] {len(mix)} requests in {wall:.3f} s, hits {srv.hits} misses {srv.misses}, "
          f"p50 {st['p50_ms']:.2f} ms p99 {st['p99_ms']:.2f} ms", flush=True)
    assert srv.hits > 0 and len(mix) == len(reqs)
    for r in reqs:
        d = np.max(np.abs(mix[r.rid].x - alone[r.rid])) / np.max(np.abs(alone[r.rid]))
        assert d <= 1e-12, (r.rid, d)
    # against the plain complex128 path of each body
    import paper_1810_07067_amd as msv
    for name, (curve, k0, eps1, M, L) in BODIES.items():
        p0 = msv.plan_from_curve(curve, RULES, k0, eps1, 1.0, m_max=M, fft_len=L, precision=0)
        A = p0.assemble(p0.tabulate(), 0, M)
        p0.factor(A, 0, M)
        for r in (q for q in reqs if q.body == name):
            rhs = torch.from_numpy(incident.rhs_modes(curve, r.waves, k0, -M, M)).cuda()
            ref = p0.solve(-M, M, rhs).cpu().numpy()
            d = np.max(np.abs(mix[r.rid].x - ref)) / np.max(np.abs(ref))
            assert d < 1e-10, (name, r.rid, d)


def test_eviction_under_a_small_budget():
    reqs = make_requests(seed=12, count=10, qps=400.0)
    srv = Server(RULES, hbm_budget=one_body_budget(), slots=3)
    res, _ = srv.run(reqs, realtime=True)
    print(f"[serve] small budget: hits {srv.hits} misses {srv.misses} evictions {srv.evictions}", flush=True)
    assert srv.evictions > 0 and len(res) == len(reqs)
    ref_srv = Server(RULES, hbm_budget=8 << 30, slots=1)
    ref, _ = ref_srv.run([Request(r.rid, r.body, r.curve, r.k0, r.eps1, r.m_max, r.fft_len, r.waves, 0.0)
                          for r in reqs], realtime=False)
    for r in reqs:
        d = np.max(np.abs(res[r.rid].x - ref[r.rid].x)) / np.max(np.abs(ref[r.rid].x))
        assert d <= 1e-12, (r.rid, d)
