"""The two AI-systems forms measured beside the step, and single pieces of
the step for hardware counters (see bench.py).

  batching  the per-mode LUs of many bodies of uneven order in one captured
            launch sequence, against the same bodies factored one at a time
  serving   a request stream of mixed bodies, wavenumbers and plane-wave
            counts through the continuous-batching server (paper_1810_07067_amd.serve)
"""
from __future__ import annotations

import sys

import numpy as np

from bench import valid_fft_len, workload


def bench_batching(rules, seed=4, n_bodies=16, M=16):
    """Batching form: modes 0..M of n_bodies random bodies (Fourier-perturbed
    spheroids, about a quarter with a conical tip, 8..32 panels) factored one
    body after another vs. by the batch's captured launch sequence."""
    import torch
    import paper_1810_07067_amd as msv
    from workloads import geometry
    rng = np.random.default_rng(seed)
    plans, mats, orders = [], [], []
    for b in range(n_bodies):
        npan = int(rng.integers(4, 17)) * 2
        tip = rng.random() < 0.25
        curve = geometry.random_body(rng, npan, tip_levels=4 if tip else 0)
        k0, eps1 = float(rng.uniform(1.0, 5.0)), float(rng.uniform(1.5, 6.0))
        L = valid_fft_len(curve, k0, eps1, M)
        try:
            p = msv.plan_from_curve(curve, rules, k0, eps1, 1.0, m_max=M, fft_len=L, precision=1)
        except msv.MsvError:
            continue  # a tip body whose panels grade too steeply
        A = p.assemble(p.tabulate(), 0, M)
        plans.append(p)
        mats.append(A)
        orders.append(p.n)
    torch.cuda.synchronize()
    ev = lambda: torch.cuda.Event(enable_timing=True)
    e0, e1 = ev(), ev()
    for p, A in zip(plans, mats):  # warm
        p.factor(A, 0, M)
    e0.record()
    for p, A in zip(plans, mats):
        p.factor(A, 0, M)
    e1.record()
    torch.cuda.synchronize()
    seq_ms = e0.elapsed_time(e1)
    batch = msv.Batch(plans, mats, 0, M)
    batch.factor()
    torch.cuda.synchronize()
    e0.record()
    batch.factor()
    e1.record()
    torch.cuda.synchronize()
    bat_ms = e0.elapsed_time(e1)
    flops = sum((8.0 / 3.0) * n ** 3 * (M + 1) for n in orders)
    return {"bodies": len(plans), "orders": orders, "modes_per_body": M + 1,
            "one_by_one_factor_ms": seq_ms, "batched_factor_ms": bat_ms, "speedup": seq_ms / bat_ms,
            "panel": batch.panel, "tuned_ms": {str(w): batch.tuned_ms(w) for w in (64, 128, 256, 512)},
            "per_mode_factorizations_per_s": len(plans) * (M + 1) / (bat_ms * 1e-3),
            "tflops": flops / (bat_ms * 1e-3) / 1e12}


def serving_requests(seed, count, arrivals):
    """Mixed stream: sphere (8 panels, k0 = 1, eps 2.25, |m| <= 16), prolate
    spheroid 1:3 (16 panels, k0 = 4, eps 4), cylinder with dyadic corners
    (eps 4 + 0.1i, k0 = 3); k0 from {base, 1.5 base}; 1..32 plane waves."""
    from paper_1810_07067_amd.serve import Request
    from workloads import geometry, incident
    cyl = geometry.polygon([(0.0, -1.0), (1.0, -1.0), (1.0, 1.0), (0.0, 1.0)], 1.0, 6, "cylinder")
    base = {"sphere": (geometry.sphere(8), 1.0, 2.25, 16),
            "spheroid": (geometry.spheroid(16, 3.0), 4.0, 4.0, 16),
            "cylinder": (cyl, 3.0, 4.0 + 0.1j, 16)}
    rng = np.random.default_rng(seed)
    names = list(base)
    reqs = []
    for i in range(count):
        name = names[int(rng.choice(3, p=[0.5, 1 / 3, 1 / 6]))]
        curve, k0, eps1, M = base[name]
        k0 = k0 * (1.5 if rng.random() < 0.5 else 1.0)
        L = valid_fft_len(curve, k0, eps1, M)
        waves = incident.random_directions(int(rng.integers(1 << 30)), int(rng.integers(1, 33)))
        reqs.append(Request(i, name, curve, k0, eps1, M, L, waves, float(arrivals[i])))
    return reqs


def bench_serving(rules, precision, count=48, seed=5, load=0.8):
    """Closed-loop capacity first (all requests at t = 0), then a Poisson stream
    at `load` times that rate; p50/p99 latency, mode-solves/s, cache hit rate."""
    from paper_1810_07067_amd.serve import Server, latency_stats, poisson_arrivals
    srv = Server(rules, hbm_budget=64 << 30, slots=4, precision=precision)
    reqs = serving_requests(seed, count, np.zeros(count))
    res, wall = srv.run(reqs, realtime=False)
    cap = count / wall
    srv2 = Server(rules, hbm_budget=64 << 30, slots=4, precision=precision)
    t = poisson_arrivals(np.random.default_rng(seed + 1), count, load * cap)
    reqs = serving_requests(seed, count, t)
    res, wall = srv2.run(reqs, realtime=True)
    st = latency_stats(res)
    solves = sum(r.mode_solves for r in res.values())
    return {"requests": count, "closed_loop_requests_per_s": cap, "qps": load * cap, **st,
            "mode_solves_per_s": solves / wall, "requests_per_s": count / wall,
            "cache_hit_rate": srv2.hits / max(1, srv2.hits + srv2.misses), "wall_s": wall}


def run_form(form):
    from workloads import rules
    rls = rules.load_rules()
    if form == "batching":
        return {"form": "batching", **bench_batching(rls)}
    return {"form": "serving", "complex64_lu_refined": bench_serving(rls, 1), "complex128_lu": bench_serving(rls, 0)}


def profile_target(what, config, modes=None):
    """One piece of the step, once, for rocprofv3 counter runs.  `modes`
    limits the LU to modes 0..modes-1 (each matrix's factorization is
    independent of the others in the batch)."""
    import torch
    import paper_1810_07067_amd as msv
    if what == "copy":
        x = torch.empty(1 << 28, dtype=torch.float32, device="cuda")
        x.fill_(1.0)
        y = torch.empty_like(x)
        torch.cuda.synchronize()
        y.copy_(x)
        torch.cuda.synchronize()
        print("copied 1 GiB", flush=True)
        return
    curve, rls, waves, cfg = workload(config)
    M = cfg["M"]
    plan = msv.plan_from_curve(curve, rls, cfg["k0"], cfg["eps1"], cfg["mu1"], m_max=M, fft_len=cfg["L"],
                               precision=1)
    nb = cfg["rows_per_block"] or curve.n
    block = torch.empty(plan.table_rows_shape(nb), dtype=torch.complex128, device="cuda")
    if what == "tabulate":
        for t0 in range(0, plan.N, nb):
            nt = min(nb, plan.N - t0)
            kb = block.view(-1)[: (M + 2) * 9 * nt * (plan.N + plan.S)].view(plan.table_rows_shape(nt))
            plan.tabulate_rows(t0, nt, out=kb)
            print(f"tabulated rows {t0}..{t0 + nt - 1}", file=sys.stderr, flush=True)
    else:
        mh = M if modes is None else min(M, int(modes) - 1)
        A = plan.assemble_streamed(0, mh, rows_per_block=nb, block=block)
        del block
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
        print(f"assembled modes 0..{mh}", file=sys.stderr, flush=True)
        plan.factor(A, 0, mh)
    torch.cuda.synchronize()
    print(f"{what} done", flush=True)
