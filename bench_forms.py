"""The forms measured beside the step (batching, serving, and the paper's
extinction experiment), and single pieces of the step for hardware counters
(see bench.py).

  batching  the per-mode LUs of many bodies of uneven order in one captured
            launch sequence, against the same bodies factored one at a time
  serving   a request stream of mixed bodies, wavenumbers and plane-wave
            counts through the continuous-batching server (paper_1810_07067_amd.serve)
  extinction the accuracy experiment of Section 6 (indirect system, current
            loop) at the sizes of Tables 1-4, with the tables' phases
"""
from __future__ import annotations

import sys
import time

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
            "plane_min": batch.plane_min,
            "tuned_plane_ms": {str(q): batch.tuned_plane_ms(q) for q in (256, 512, 1024)},
            "per_mode_factorizations_per_s": len(plans) * (M + 1) / (bat_ms * 1e-3),
            "tflops": flops / (bat_ms * 1e-3) / 1e12}


def random_bodies(seed=4, n_bodies=64):
    """The batched workload at its stated size: n_bodies seeded random bodies
    (Fourier-perturbed spheroids, about a quarter with a dyadically refined
    conical tip) with 256..2048 nodes, k0 uniform in [1, 30], eps1 uniform in
    [1.5, 6]."""
    from workloads import geometry
    out = []
    for b in range(n_bodies):
        rng = np.random.default_rng([seed, b])
        npan = max(16, int(rng.integers(256, 2049)) // 16)
        tip = rng.random() < 0.25
        k0, eps1 = float(rng.uniform(1.0, 30.0)), float(rng.uniform(1.5, 6.0))
        while True:  # a tip adds panels: stay within 2048 nodes
            curve = geometry.random_body(np.random.default_rng([seed, b, 1]), npan, tip_levels=4 if tip else 0)
            if curve.n <= 2048:
                break
            npan -= 1
        out.append((curve, k0, eps1))
    return out


def bench_batching_random_bodies(rules, M=64, budget=200e9, seed=4, n_bodies=64):
    """Batching form at the stated size: all modes |m| <= M of every body.
    The bodies do not fit in HBM together, so they stream through in groups
    whose matrices and plan memory fit `budget`; each group is tabulated and
    assembled body by body (row blocks as the serving form takes them), then
    factored one body after another and again as one batch (one captured
    launch sequence over all (body, mode) matrices, outer panel width tuned),
    and solved for one plane wave.  Per group the faster of the two schedules
    is kept (the batch's outer panels can only be as wide as every smaller
    order's divisor, 64 for these mixed orders, while a lone body uses 512).
    The smallest body of each group is also solved with the complex128 LU, and
    the two solutions compared.  A body whose mixed-precision refinement does
    not converge is refactored with the complex128 LU, timed apart."""
    import torch
    import paper_1810_07067_amd as msv
    from paper_1810_07067_amd import serve
    from workloads import incident
    bodies = random_bodies(seed, n_bodies)
    ev = lambda: torch.cuda.Event(enable_timing=True)
    S = rules[0][0].shape[1] + 2 * rules[1][0].size

    def need(curve, k0, eps1):
        L = valid_fft_len(curve, k0, eps1, M)
        n = 4 * curve.n
        return L, (M + 1) * n * n * 16 + msv.workspace_bytes(curve.n, S, L, M + 1, 2 * (2 * M + 1), 1)
    # the batch also holds, per (body, mode) matrix, the inverse slots and the
    # bf16 planes of one trailing update at the group's largest order
    def batch_ws(nmax, nmat):
        R = (nmax + 127) // 128 * 128
        return nmat * (8 * 64 * 64 * 8 + 2 * 4 * R * 512 * 2)
    groups, cur, used, nmax = [], [], 0, 0
    for bd in bodies:
        L, b = need(*bd)
        nm = max(nmax, 4 * bd[0].n)
        if cur and used + b + batch_ws(nm, (len(cur) + 1) * (M + 1)) > budget:
            groups.append(cur)
            cur, used, nm = [], 0, 4 * bd[0].n
        cur.append((bd, L))
        used += b
        nmax = nm
    groups.append(cur)
    tot_solo = tot_batch = tot_sched = flops = fallback_ms = 0.0
    rows, parity, skipped, noconv = [], [], 0, 0
    for gi, grp in enumerate(groups):
        plans, mats, meta = [], [], []
        for (curve, k0, eps1), L in grp:
            try:
                p = msv.plan_from_curve(curve, rules, k0, eps1, 1.0, m_max=M, fft_len=L, precision=1)
            except msv.MsvError:
                skipped += 1  # a tip whose panels grade too steeply, or L beyond 1024
                continue
            nb = serve.table_block_rows(curve, M, S) or curve.n
            mats.append(p.assemble_streamed(0, M, rows_per_block=nb))
            plans.append(p)
            meta.append((curve, k0, eps1, L))
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
        for p, A in zip(plans, mats):  # warm, and the factor storage
            p.factor(A, 0, M)
        e0, e1 = ev(), ev()
        e0.record()
        for p, A in zip(plans, mats):
            p.factor(A, 0, M)
        e1.record()
        torch.cuda.synchronize()
        solo = e0.elapsed_time(e1)
        batch = msv.Batch(plans, mats, 0, M)
        batch.factor()
        torch.cuda.synchronize()
        e0.record()
        batch.factor()
        e1.record()
        torch.cuda.synchronize()
        bat = e0.elapsed_time(e1)
        gflops = sum((8.0 / 3.0) * p.n ** 3 * (M + 1) for p in plans)
        tot_solo += solo
        tot_batch += bat
        flops += gflops
        # one plane wave per body, all modes, from the batched factors; where
        # the refinement does not converge (the system too ill-conditioned for
        # the split-bf16 factors) the body is refactored with the complex128 LU
        sols, gpar, gfall = [], None, 0
        for j, (p, (curve, k0, eps1, L)) in enumerate(zip(plans, meta)):
            rhs = torch.from_numpy(incident.rhs_modes(curve, [incident.paper_default_direction()], k0, -M, M)).cuda()
            try:
                sols.append(p.solve(-M, M, rhs))
            except msv.MsvError as exc:
                if exc.status != msv.MSV_ENOCONV:
                    raise
                noconv += 1
                gfall += 1
                pf = msv.plan_from_curve(curve, rules, k0, eps1, 1.0, m_max=M, fft_len=L, precision=0)
                e0.record()
                pf.factor(mats[j], 0, M)  # in place: the matrices are not needed again
                e1.record()
                xf = pf.solve(-M, M, rhs)
                torch.cuda.synchronize()
                fallback_ms += e0.elapsed_time(e1)
                assert bool(torch.isfinite(xf).all())
                sols.append(None)  # (kept out of the parity check below)
                pf.close()
                del xf
        # the smallest body of the group against its complex128 LU
        i = min(range(len(plans)), key=lambda j: plans[j].n)
        if sols[i] is not None:
            curve, k0, eps1, L = meta[i]
            pref = msv.plan_from_curve(curve, rules, k0, eps1, 1.0, m_max=M, fft_len=L, precision=0)
            A0 = mats[i].clone()
            pref.factor(A0, 0, M)
            rhs = torch.from_numpy(incident.rhs_modes(curve, [incident.paper_default_direction()], k0, -M, M)).cuda()
            xr = pref.solve(-M, M, rhs)
            gpar = float(((sols[i] - xr).abs().max() / xr.abs().max()).item())
            parity.append(gpar)
            pref.close()
            del A0, xr
        rows.append({"group": gi, "bodies": len(plans), "orders": [p.n for p in plans],
                     "one_by_one_factor_ms": solo, "batched_factor_ms": bat, "speedup": solo / bat,
                     "complex128_fallback": gfall, "parity_vs_complex128": gpar, "panel": batch.panel,
                     "plane_min": batch.plane_min, "scheduled": "batched" if bat < solo else "one by one",
                     "scheduled_tflops": gflops / (min(bat, solo) * 1e-3) / 1e12})
        tot_sched += min(bat, solo)
        print(f"[bodies] group {gi}: {len(plans)} bodies, orders {min(p.n for p in plans)}..{max(p.n for p in plans)}, "
              f"one by one {solo:.1f} ms, batched {bat:.1f} ms, complex128 fallback {gfall}, parity {gpar}",
              file=sys.stderr, flush=True)
        del batch, sols
        for p in plans:
            p.close()
        del plans, mats
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
    nb = sum(r["bodies"] for r in rows)
    return {"bodies": nb, "skipped": skipped, "groups": rows,
            "modes_per_body": M + 1, "one_by_one_factor_ms": tot_solo, "batched_factor_ms": tot_batch,
            "scheduled_factor_ms": tot_sched, "scheduled_tflops": flops / (tot_sched * 1e-3) / 1e12,
            "per_mode_factorizations_per_s": nb * (M + 1) / (tot_sched * 1e-3),
            "refinement_not_converged": noconv, "complex128_fallback_factor_ms": fallback_ms,
            "max_parity_vs_complex128": max(parity) if parity else None}


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


SERVING_BODIES = {  # the three workloads at their full sizes: curve, k0, eps1, M, smallest L
    "sphere": (lambda g: g.sphere(8), 1.0, 2.25, 16, 64),
    "spheroid": (lambda g: g.spheroid(64, 3.0), 10.0, 4.0, 64, 256),
    "cylinder": (lambda g: g.cylinder(24), 20.0, 4.0 + 0.1j, 128, 512),
}
POOL_WAVES = 32


def serving_pools(seed, factors=(1.0, 1.5)):
    """Per (body, k0 factor): the body and the incident modes of a seeded pool
    of 32 plane waves, [2M+1, 32, 4N] (a request's incident data is an input:
    it brings its modes, a subset of its body's pool)."""
    from workloads import geometry, incident
    pools = {}
    for name, (mk, k0, eps1, M, L0) in SERVING_BODIES.items():
        curve = mk(geometry)
        for f in factors:
            k = k0 * f
            L = valid_fft_len(curve, k, eps1, M, lo=L0)
            waves = incident.random_directions(seed * 100 + len(pools), POOL_WAVES)
            t0 = time.perf_counter()
            rhs = incident.rhs_modes(curve, waves, k, -M, M)
            print(f"[serving] pool {name} k0={k}: {rhs.shape}, {time.perf_counter() - t0:.1f} s on the host",
                  file=sys.stderr, flush=True)
            pools[(name, f)] = (curve, k, eps1, M, L, waves, rhs)
    return pools


def serving_requests_full(pools, seed, count, arrivals, factors=(1.0, 1.5)):
    """Poisson-stream requests over the three full-size bodies (sphere 1/2,
    spheroid 1/3, cylinder 1/6), k0 = base times one of `factors`, 1..32
    plane waves drawn from the body's pool."""
    from paper_1810_07067_amd.serve import Request
    rng = np.random.default_rng(seed)
    names = list(SERVING_BODIES)
    reqs = []
    for i in range(count):
        name = names[int(rng.choice(3, p=[0.5, 1 / 3, 1 / 6]))]
        f = factors[int(rng.integers(len(factors)))]
        curve, k, eps1, M, L, waves, pool = pools[(name, f)]
        idx = np.sort(rng.permutation(POOL_WAVES)[: int(rng.integers(1, POOL_WAVES + 1))])
        reqs.append(Request(i, name, curve, k, eps1, M, L, [waves[j] for j in idx], float(arrivals[i]),
                            rhs=np.ascontiguousarray(pool[:, idx, :])))
    return reqs


def bench_serving_full(rules, count=36, seed=9, loads=(0.5, 0.8, 0.95), budget=250 << 30, slots=4,
                       factors=(1.0, 1.5)):
    """Serving at the full body sizes, both precisions: the closed-loop rate
    (every request at t = 0), the two precisions' currents compared request by
    request, then Poisson streams at `loads` times each precision's own
    closed-loop rate (cold cache each run).  `factors`: the k0 multiples a
    body is requested at (more of them, fewer repeated bodies)."""
    from paper_1810_07067_amd.serve import Server, latency_stats, poisson_arrivals
    pools = serving_pools(seed, factors)
    mk = lambda arrivals: serving_requests_full(pools, seed, count, arrivals, factors)
    names = {r.rid: r.body for r in mk(np.zeros(count))}

    def per_body(res):
        """Mean build, wait and solve seconds per body, and the builds."""
        out = {}
        for b in SERVING_BODIES:
            rs = [r for r in res.values() if names[r.rid] == b]
            built = [r.build_s for r in rs if not r.cached]
            out[b] = {"requests": len(rs), "builds": len(built),
                      "mean_build_s": float(np.mean(built)) if built else None,
                      "mean_wait_s": float(np.mean([r.wait_s for r in rs])) if rs else None,
                      "mean_solve_s": float(np.mean([r.solve_s for r in rs])) if rs else None}
        return out
    out, ref = {}, {}
    for precision in (0, 1):
        tag = "complex128_lu" if precision == 0 else "complex64_lu_refined"
        srv = Server(rules, hbm_budget=budget, slots=slots, precision=precision)
        res, wall = srv.run(mk(np.zeros(count)), realtime=False)
        srv.close()
        cap = count / wall
        row = {"closed_loop_requests_per_s": cap, "closed_loop_wall_s": wall,
               "closed_loop_mode_solves_per_s": sum(r.mode_solves for r in res.values()) / wall,
               "cache_hits": srv.hits, "cache_misses": srv.misses, "evictions": srv.evictions,
               "complex128_fallbacks": srv.fallbacks, "per_body": per_body(res)}
        if precision == 0:
            ref = {rid: np.array(r.x) for rid, r in res.items()}  # copies, independent of the server's buffers
        else:
            row["max_rel_diff_vs_complex128"] = max(
                float(np.max(np.abs(r.x - ref[rid])) / np.max(np.abs(ref[rid]))) for rid, r in res.items())
            ref = {}
        del res
        print(f"[serving] {tag} closed loop: {row}", file=sys.stderr, flush=True)
        for load in loads:
            t = poisson_arrivals(np.random.default_rng(seed + 1), count, load * cap)
            srv = Server(rules, hbm_budget=budget, slots=slots, precision=precision)
            res, wall = srv.run(mk(t), realtime=True)
            srv.close()
            st = latency_stats(res)
            row[f"load_{load}"] = {"qps": load * cap, **st, "requests_per_s": count / wall,
                                   "mode_solves_per_s": sum(r.mode_solves for r in res.values()) / wall,
                                   "cache_hit_rate": srv.hits / max(1, srv.hits + srv.misses),
                                   "evictions": srv.evictions, "wall_s": wall}
            print(f"[serving] {tag} load {load}: {row[f'load_{load}']}", file=sys.stderr, flush=True)
            del res
        out[tag] = row
    return {"requests": count, "slots": slots, "hbm_budget_bytes": budget, "k0_factors": list(factors), **out}


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


# Section 6, Tables 1 and 2: (k0, k1, N_f, N_pts) and the printed E_error
TABLE1_TORUS = [(1, 2, 13, 64, 2.32e-9), (1, 5, 16, 160, 4.61e-9), (1, 10, 21, 320, 3.11e-8),
                (5, 2, 13, 160, 1.01e-9), (5, 10, 21, 320, 3.84e-9), (5, 20, 30, 640, 4.63e-9),
                (10, 5, 17, 320, 1.61e-9), (10, 20, 30, 640, 2.08e-9), (10, 40, 45, 640, 2.66e-8),
                (20, 5, 17, 320, 4.78e-9), (20, 10, 22, 640, 3.37e-9), (20, 40, 45, 640, 1.10e-8)]
TABLE2_STARFISH = [(5, 2, 10, 224, 1.24e-9), (5, 10, 16, 304, 3.44e-10), (5, 20, 21, 464, 1.51e-9),
                   (10, 5, 13, 304, 2.04e-10), (10, 20, 21, 464, 9.74e-10), (10, 40, 30, 784, 1.45e-8),
                   (20, 5, 13, 464, 1.05e-10), (20, 10, 16, 464, 4.41e-10), (20, 40, 30, 784, 4.60e-9),
                   (40, 5, 13, 784, 3.39e-10), (40, 10, 16, 784, 3.58e-9), (40, 20, 21, 784, 3.01e-9)]
TABLE3_DROPLET = [(5, 2, 7, 224, 2.71e-10), (5, 10, 10, 320, 1.86e-9), (5, 20, 11, 480, 5.11e-9),
                  (10, 5, 9, 320, 1.24e-10), (10, 20, 11, 480, 2.59e-9), (10, 40, 14, 800, 6.76e-9),
                  (20, 5, 9, 480, 5.81e-10), (20, 10, 10, 480, 1.31e-10), (20, 40, 14, 800, 3.43e-9),
                  (40, 5, 9, 800, 3.48e-10), (40, 10, 10, 800, 6.12e-10), (40, 20, 12, 800, 1.45e-10)]
TABLE4_CYLINDER = [(2, 1, 9, 1312, 4.11e-9), (2, 5, 11, 1440, 2.56e-8), (2, 10, 14, 1696, 9.32e-7),
                   (5, 2, 10, 1440, 1.54e-8), (5, 10, 14, 1696, 5.92e-8), (5, 20, 17, 2208, 9.74e-7),
                   (10, 2, 10, 1696, 1.91e-8), (10, 5, 11, 1696, 3.95e-8), (10, 20, 17, 2208, 2.24e-6),
                   (20, 2, 10, 2208, 3.54e-8), (20, 5, 11, 2208, 1.39e-7), (20, 10, 14, 2208, 1.32e-7)]
LOOP = dict(center=[0.4, 0.5, 5.0], radius=0.42)  # Section 6
CYLINDER_CORNER_LEVELS = 14  # corner panels of 1/(base panels per unit)/2^14, about 1e-5 (Example 4)
CYLINDER_MAX_LEVELS = 24     # the deepest corner grading the full-size cylinder checks (7.45e-9 panels)


def cylinder_split(npts, k):
    """Base panels per unit length and corner levels for a cylinder of about
    npts nodes: base panels no longer than half a wavelength at wavenumber k
    (at least 2 per unit), every other panel spent on dyadic corner levels
    (at most CYLINDER_MAX_LEVELS), the base panels then filling the rest."""
    npan = npts // 16
    p_min = max(2.0, k / np.pi)
    levels = int(min(CYLINDER_MAX_LEVELS, (npan - 4 * p_min) // 4))
    base = lambda q: sum(max(1, int(round(ln * q))) for ln in (1.0, 2.0, 1.0))  # as geometry.polygon
    p = npan / 4 - levels
    while base(p) + 4 * levels > npan:
        p -= 0.25
    return p, levels


def extinction_body(body, npts, k=None):
    """The generating curve of Tables 1-4 with about npts nodes (16 per panel).
    For the cylinder with k given, the nodes go to the corners as far as
    cylinder_split allows; without k, the corner panels end near 1e-5 as in
    Example 4."""
    from workloads import geometry
    npan = npts // 16
    if body == "torus":
        return geometry.torus(npan)
    if body == "starfish":
        return geometry.starfish(npan)
    if body == "droplet":
        return geometry.droplet(npan)
    if body == "cylinder":
        # 4 p base panels over the perimeter (bottom 1, side 2, top 1) and the
        # four corner panels split `levels` times each
        if k is None:
            return geometry.cylinder(CYLINDER_CORNER_LEVELS, npan / 4 - CYLINDER_CORNER_LEVELS)
        p, levels = cylinder_split(npts, k)
        return geometry.cylinder(levels, p)
    raise ValueError(body)


def _interior_points(body, rng, P):
    if body == "torus":  # within half of the cross-section of r = 2 + cos t, z = sin(t)/2
        rho = 0.5 * np.sqrt(rng.uniform(0, 1, P))
        ph, th = rng.uniform(0, 2 * np.pi, P), rng.uniform(0, 2 * np.pi, P)
        rr, zz = 2 + rho * np.cos(ph), 0.5 * rho * np.sin(ph)
        return np.stack([rr * np.cos(th), rr * np.sin(th), zz], axis=1)
    th = rng.uniform(0, 2 * np.pi, P)
    if body == "starfish":  # the starfish contains the ball of radius 1.5
        v = rng.standard_normal((P, 3))
        return v / np.linalg.norm(v, axis=1)[:, None] * rng.uniform(0, 0.75, (P, 1))
    if body == "droplet":  # z increases along the curve: (s r(t), z(t)) lies inside for s < 1
        t = rng.uniform(0.6, 0.9, P)
        sc = rng.uniform(0.0, 0.5, P)
        rr = sc * np.sin(np.pi * t) * np.cos(0.5 * np.pi * (t - 1.5))
        zz = np.sin(np.pi * t) * np.sin(0.5 * np.pi * (t - 1.5)) + 0.5
        return np.stack([rr * np.cos(th), rr * np.sin(th), zz], axis=1)
    if body == "cylinder":
        rr, zz = 0.5 * np.sqrt(rng.uniform(0, 1, P)), rng.uniform(-0.5, 0.5, P)
        return np.stack([rr * np.cos(th), rr * np.sin(th), zz], axis=1)
    raise ValueError(body)


def bench_extinction(rules, body, rows, precision=1, seed=3, n_points=6, corner_first=False):
    """The accuracy experiment of Section 6 on the GPU: the indirect system
    (eq. dualmullrep) with the current-loop data of eq. loop, at the sizes of
    Tables 1-4 (torus, rotated starfish, droplet, cylinder); E_error over random interior
    points (eq. interior_dual, evaluated on 4 sub-panels per panel) and the
    four phases of the tables: T_kernel
    (tabulation), T_matgen (assembly), T_solve (factor and solve all modes),
    T_add (one more right-hand side).  corner_first: the cylinder's nodes go
    to the corners first (cylinder_split) instead of the paper's 1e-5 grading."""

    import torch
    import paper_1810_07067_amd as msv
    from workloads import geometry, incident
    out = []
    for k0, k1, Nf, npts, paper_err in rows:
        curve = extinction_body(body, npts, max(k0, k1) if corner_first else None)
        eps1 = (k1 / k0) ** 2
        L = valid_fft_len(curve, k0, eps1, Nf)
        rhs_h = incident.loop_rhs_modes(curve, LOOP["center"], LOOP["radius"], k1, k0, 1.0, -Nf, Nf)
        tail = float(np.abs(rhs_h[[0, -1]]).max() / np.abs(rhs_h).max())  # data beyond N_f
        rhs = torch.from_numpy(rhs_h).cuda()
        pts = _interior_points(body, np.random.default_rng(seed), n_points)

        def phase(fn):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            r = fn()
            torch.cuda.synchronize()
            return r, time.perf_counter() - t0
        used = precision
        for prec in (precision, 0) if precision else (0,):
            # complex64 factors whose refinement does not converge (the
            # system too ill-conditioned for them) fall back to complex128
            plan = msv.plan_from_curve(curve, rules, k0, eps1, 1.0, m_max=Nf, fft_len=L, precision=prec,
                                       formulation=1)
            kern, t_kernel = phase(plan.tabulate)
            A, t_matgen = phase(lambda: plan.assemble(kern, 0, Nf))
            del kern
            try:
                x, t_solve = phase(lambda: (plan.factor(A, 0, Nf), plan.solve(-Nf, Nf, rhs))[1])
            except msv.MsvError as exc:
                if exc.status != msv.MSV_ENOCONV or prec == 0:
                    raise
                plan.close()
                del A
                continue
            used = prec
            break
        _, t_add = phase(lambda: plan.solve(-Nf, Nf, rhs))
        E, H = plan.fields(-Nf, Nf, x, pts, "interior", upsample=4)
        El, Hl = incident.current_loop(LOOP["center"], LOOP["radius"], k1, k0, 1.0)
        Er, Hr = El(pts), Hl(pts)
        E, H = E[0].cpu().numpy(), H[0].cpu().numpy()
        err = np.sqrt((np.linalg.norm(E - Er) ** 2 + np.linalg.norm(H - Hr) ** 2)
                      / (np.linalg.norm(Er) ** 2 + np.linalg.norm(Hr) ** 2))
        out.append({"k0": k0, "k1": k1, "N_f": Nf, "N_pts": curve.n, "paper_N_pts": npts, "L": L,
                    "data_tail": tail, "smallest_panel": float(curve.panel_len.min()), "T_kernel_s": t_kernel,
                    "T_matgen_s": t_matgen, "T_solve_s": t_solve, "T_add_s": t_add, "E_error": float(err),
                    "paper_E_error": paper_err, "precision": used,
                    "ir_iterations": plan.last_ir_iterations() if used else 0})
        print(f"[extinction] {body} {out[-1]}", file=sys.stderr, flush=True)
        plan.close()
        del A, x
        torch.cuda.empty_cache()
    return out


def run_form(form):
    from workloads import rules
    rls = rules.load_rules()
    if form == "batching":
        return {"form": "batching", "small_bodies": bench_batching(rls),
                "random_bodies_all_modes": bench_batching_random_bodies(rls)}
    if form == "extinction":
        return {"form": "extinction", "precision": "complex64 LU + complex128 refinement",
                "torus_table1": bench_extinction(rls, "torus", TABLE1_TORUS),
                "starfish_table2": bench_extinction(rls, "starfish", TABLE2_STARFISH),
                "droplet_table3": bench_extinction(rls, "droplet", TABLE3_DROPLET),
                "cylinder_table4": bench_extinction(rls, "cylinder", TABLE4_CYLINDER, corner_first=True),
                "cylinder_table4_panels_to_1e-5": bench_extinction(rls, "cylinder", TABLE4_CYLINDER)}
    return {"form": "serving", "full_size": bench_serving_full(rls),
            "full_size_mostly_new_bodies": bench_serving_full(rls, loads=(), factors=(1.0, 1.1, 1.2, 1.3, 1.4, 1.5)),
            "small_bodies": {"complex64_lu_refined": bench_serving(rls, 1), "complex128_lu": bench_serving(rls, 0)}}


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
