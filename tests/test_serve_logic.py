"""Host logic of the serving loop (no GPU): footprints, admission in arrival
order, least-recently-used eviction of idle factorizations only."""
import numpy as np

from paper_1810_07067_amd.serve import Request, Server, entry_bytes, poisson_arrivals
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
