"""Host logic of the serving loop (no GPU): footprints, admission in arrival
order with cache hits passing a request that waits for memory, least-recently-
used eviction of idle factorizations only."""
import threading
import time

import numpy as np

from paper_1810_07067_amd.serve import Request, Result, Server, entry_bytes, poisson_arrivals
from workloads import geometry, incident, rules


def _req(rid, curve, body, k0=1.0):
    return Request(rid, body, curve, k0, 2.25, 4, 64, [incident.tilted_direction(10.0)], 0.0)


RULES = rules.load_rules()
S = RULES[0][0].shape[1] + 2 * RULES[1][0].size


def test_entry_bytes_counts_matrices_plan_workspace_and_table():
    """The held part is the caller's complex128 matrices, the library's bound
    on the plan's own memory (factors, LU workspace, inverses, solve workspace
    for 2M+1 modes x 32 waves) and the request's right-hand sides and
    solutions; the transient part is the modal-kernel table."""
    import paper_1810_07067_amd as msv
    c = geometry.sphere(4)
    N, n, M = c.n, 4 * c.n, 4
    vec = (2 * M + 1) * 32
    keep, table = entry_bytes(c, M, 64, 1, S)
    plan = msv.workspace_bytes(N, S, 64, M + 1, vec, 1)
    assert keep == 5 * n * n * 16 + plan + 2 * vec * n * 16
    assert plan > 5 * n * n * 8 + vec * n * 64  # complex64 factors + solve workspace
    assert table == 6 * 9 * N * (N + S) * 16
    keep0, _ = entry_bytes(c, M, 64, 0, S)
    assert keep0 == 5 * n * n * 16 + msv.workspace_bytes(N, S, 64, M + 1, vec, 0) + 2 * vec * n * 16 < keep


def test_admission_hits_and_lru_eviction():
    a, b = geometry.sphere(4), geometry.spheroid(4, 2.0)
    keep, table = entry_bytes(a, 4, 64, 1, S)
    srv = Server(rules=RULES, hbm_budget=keep + table + keep // 2, slots=2)
    e1, built1, t1 = srv._try_admit(_req(0, a, "a"))
    assert built1 and srv.used == keep + table
    srv.used -= t1  # as the builder does once the table is freed
    e1.ready.set()
    e2, built2, _ = srv._try_admit(_req(1, a, "a"))  # same body: a hit, no memory
    assert not built2 and e2 is e1 and srv.hits == 1
    # a second body does not fit while the first is in use
    assert srv._try_admit(_req(2, b, "b")) is False
    e1.users = 0
    e3, built3, t3 = srv._try_admit(_req(3, b, "b"))  # now the idle entry is evicted
    assert built3 and srv.evictions == 1 and ("a", 1.0, 2.25, 1.0, 4, 64) not in srv.cache


def test_poisson_arrivals_rate():
    t = poisson_arrivals(np.random.default_rng(5), 4000, 50.0)
    assert np.all(np.diff(t) > 0)
    assert abs(len(t) / t[-1] - 50.0) < 3.0


class _StubPlan:
    def close(self, wait=True):
        pass


class _StubServer(Server):
    """The scheduler with the GPU work replaced: a build marks the entry ready
    and gives its table back; every request holds its slot for `hold` s."""

    def __init__(self, budget, hold=0.2):
        super().__init__(rules=RULES, hbm_budget=budget, slots=2, torch_pool=False)
        self.hold = hold
        self.order = []
        self._order_mu = threading.Lock()

    def _new_streams(self):
        return [object() for _ in range(self.slots)]

    def _serve_one(self, req, admitted, t0, slot_streams):
        e, builder, table = admitted
        stream = slot_streams.get()
        try:
            with self._order_mu:
                self.order.append(req.rid)
            if builder:
                e.plan = _StubPlan()
                with self._mu:
                    self.used -= table
                e.ready.set()
            else:
                e.ready.wait()
            time.sleep(self.hold)
            return Result(req.rid, None, time.perf_counter() - t0 - req.arrival, not builder, 0, 1)
        finally:
            with self._mu:
                e.users -= 1
                e.last_used = time.perf_counter()
            slot_streams.put(stream)


def test_cache_hits_pass_a_request_waiting_for_memory():
    """Budget for one body: request 1 (a second body) must wait until body a is
    idle, and request 2 (body a again, in the cache) goes ahead of it."""
    a, b = geometry.sphere(4), geometry.spheroid(4, 2.0)
    keep, table = entry_bytes(a, 4, 64, 1, S)
    keep_b, table_b = entry_bytes(b, 4, 64, 1, S)
    srv = _StubServer(budget=max(keep + table, keep_b + table_b) + keep // 4)
    reqs = [_req(0, a, "a"), _req(1, b, "b"), _req(2, a, "a")]
    results, _ = srv.run(reqs, realtime=False)
    assert sorted(results) == [0, 1, 2]
    assert srv.order == [0, 2, 1], srv.order
    assert results[2].cached and not results[1].cached
    assert srv.hits == 1 and srv.misses == 2 and srv.evictions == 1


def test_close_keeps_the_memory_in_torchs_cache_unless_asked(monkeypatch):
    """close() drops every entry and closes its plan; the memory goes back to
    the driver only with release=True (memory returned and taken again by the
    next server of the process made its builds slower)."""
    import torch
    calls = []
    monkeypatch.setattr(torch.cuda, "synchronize", lambda *a, **k: calls.append("sync"))
    monkeypatch.setattr(torch.cuda, "empty_cache", lambda *a, **k: calls.append("empty"))
    closed = []

    class _Plan:
        def close(self, wait=True):
            closed.append(wait)

    for release, expect in ((False, ["sync"]), (True, ["sync", "empty"])):
        calls.clear()
        closed.clear()
        srv = Server(rules=RULES, hbm_budget=1 << 30, slots=1, torch_pool=False)
        e, built, _ = srv._try_admit(_req(0, geometry.sphere(4), "a"))
        e.plan, e.A = _Plan(), object()
        if release:
            srv.close(release=True)
        else:
            srv.close()  # the default keeps the cache
        assert calls == expect and closed == [True]
        assert not srv.cache and srv.used == 0 and e.plan is None and e.A is None
