"""Benchmark: one step = the whole hot path on one body.

Workload (prolate spheroid, axes 1:3): 64 panels x 16 Gauss-Legendre nodes
(1024 nodes, 4096 unknowns per mode), modes |m| <= 64, azimuthal FFT length 256,
k0 = 10, eps1 = 4, mu1 = 1, eight plane waves with directions drawn from seed 2.
A step is

  tabulate  modal Green's functions, all pairs incl. near-panel support nodes
  assemble  per-mode Mueller-Nystrom matrices, m = 0..64
  factor    complex64 LU on MFMA, all 65 modes
  solve     complex128-refined solves for m = -64..64, 8 right-hand sides

with every input already resident in HBM.  Prints one JSON line.
Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP32_MFMA_PEAK_TF = 157.3
BF16_MFMA_PEAK_TF = 2500.0  # dense
FP64_PEAK_TF = 78.6


def lu_traffic():
    """HBM bytes of one factorization from the committed rocprofv3 counter
    summary, while the LU source is the one the counters were taken on
    (its SHA-256 is recorded there); None otherwise."""
    import hashlib
    import re
    here = os.path.dirname(os.path.abspath(__file__))
    try:
        text = open(os.path.join(here, "profiles", "lu_spheroid1024_m64_traffic.md")).read()
        src = open(os.path.join(here, "paper_1810_07067_amd", "csrc", "lu.hip"), "rb").read()
    except OSError:
        return None
    h = re.search(r"lu\.hip sha256 = ([0-9a-f]{64})", text)
    b = re.search(r"lu traffic bytes per factorization = (\d+)", text)
    if not h or not b or h.group(1) != hashlib.sha256(src).hexdigest():
        return None
    return int(b.group(1))


def workload():
    from workloads import geometry, incident, rules
    curve = geometry.spheroid(64, 3.0)
    cfg = dict(k0=10.0, eps1=4.0, mu1=1.0, M=64, L=256, n_dirs=8, seed=2)
    waves = incident.random_directions(cfg["seed"], cfg["n_dirs"])
    return curve, rules.load_rules(), waves, cfg


def cpu_baseline(curve, rls, cfg, budget_s=15.0):
    """The FP64 oracle on the host: modal-kernel entries/s on a row sample."""
    from oracle import discretize, modal
    sup = discretize.support_points(curve, *rls)
    k1 = cfg["k0"] * np.sqrt(cfg["eps1"] * cfg["mu1"]) + 0j
    kp = modal.KernelParams(cfg["k0"], k1, cfg["M"], cfg["L"], float(curve.r.max()))
    rows_done, entries, t0 = 0, 0, time.perf_counter()
    rng = np.random.default_rng(0)
    rows = rng.permutation(curve.n)
    while time.perf_counter() - t0 < budget_s and rows_done < len(rows):
        tab = modal.tabulate(curve, sup, kp, rows=[rows[rows_done]])
        entries += tab.size
        rows_done += 1
    dt = time.perf_counter() - t0
    return dict(value=entries / dt, unit="modal-kernel entries/s", cores=1, kind="oracle",
                sample=f"{rows_done} random target rows x {curve.n + sup.r.shape[1]} sources x "
                       f"{cfg['M'] + 2} modes x 9 types ({dt:.1f} s, numpy FP64)")


def valid_fft_len(curve, k0, eps1, M, lo=64):
    """Smallest power of two L >= lo with M + 1 + N_f <= L/2 - 1 (the plan's rule)."""
    import math
    k = max(k0, abs(k0 * np.sqrt(complex(eps1))))
    x = 2.0 * k * float(curve.r.max())
    j = 1
    while 2 * j * math.log(max(x, 1e-300) / 2.0) - math.lgamma(2 * j + 1.0) > math.log(1e-16):
        j += 1
    L = lo
    while M + 1 + j > L // 2 - 1:
        L *= 2
    return L


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


def profile_target(what):
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
    curve, rls, waves, cfg = workload()
    M = cfg["M"]
    plan = msv.plan_from_curve(curve, rls, cfg["k0"], cfg["eps1"], cfg["mu1"], m_max=M, fft_len=cfg["L"],
                               precision=1)
    kern = plan.tabulate()
    if what == "lu":
        A = plan.assemble(kern, 0, M)
        del kern
        torch.cuda.synchronize()
        plan.factor(A, 0, M)
    torch.cuda.synchronize()
    print(f"{what} done", flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-forms", action="store_true", help="skip the batching and serving measurements")
    ap.add_argument("--profile-target", choices=["lu", "tabulate", "copy"],
                    help="run one piece once for hardware counters and exit: the LU of the benchmark "
                         "workload, its tabulation, or a 1 GiB device copy (counter calibration)")
    args = ap.parse_args()
    if args.profile_target:
        profile_target(args.profile_target)
        return
    if args.gpus != 1:
        print(f"bench.py runs on exactly one GPU (got --gpus {args.gpus}); the modes shard "
              "across GPUs without communication but that path is not built here", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1810_07067_amd as msv

    curve, rls, waves, cfg = workload()
    M, L = cfg["M"], cfg["L"]
    from workloads import incident
    rhs_h = incident.rhs_modes(curve, waves, cfg["k0"], -M, M)
    print(f"[bench] N={curve.n} M={M} L={L} rhs={rhs_h.shape}", file=sys.stderr, flush=True)

    plan = msv.plan_from_curve(curve, rls, cfg["k0"], cfg["eps1"], cfg["mu1"], m_max=M, fft_len=L,
                               precision=1, ir_tol=1e-12, ir_max_iter=20)
    dev = torch.device("cuda:0")
    kern = torch.empty(plan.table_shape, dtype=torch.complex128, device=dev)
    A = torch.empty((M + 1, plan.n, plan.n), dtype=torch.complex128, device=dev)
    rhs = torch.from_numpy(rhs_h).to(dev)
    x = torch.empty_like(rhs)
    entries = plan.table_entries
    n = plan.n

    ev = lambda: torch.cuda.Event(enable_timing=True)

    def step(record=None):
        e = [ev() for _ in range(5)]
        e[0].record()
        plan.tabulate(out=kern)
        e[1].record()
        plan.assemble(kern, 0, M, out=A)
        e[2].record()
        plan.factor(A, 0, M)
        e[3].record()
        plan.solve(-M, M, rhs, out=x)
        e[4].record()
        if record is not None:
            record.append(e)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    recs = []
    t0 = time.perf_counter()
    for i in range(args.steps):
        step(recs)
        print(f"[bench] step {i} done", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    phases = np.array([[a.elapsed_time(b) for a, b in zip(e[:-1], e[1:])] for e in recs])  # ms
    step_ms = phases.sum(axis=1)
    ms_per_step = wall * 1e3 / args.steps
    tab_ms, asm_ms, fac_ms, sol_ms = phases.mean(axis=0)

    # accuracy guard: far-field-relevant relative residual of the refined solves
    ir_iters = plan.last_ir_iterations()

    # rooflines (algorithmic): tabulation writes 16 B per entry; complex LU
    # (8/3) n^3 real flops per mode, against the dense bf16 MFMA peak (the
    # trailing updates, most of the flops, run as bf16 products)
    tab_gbs = entries * 16 / (tab_ms * 1e-3) / 1e9
    lu_flops = (8.0 / 3.0) * n ** 3 * (M + 1)
    lu_tfs = lu_flops / (fac_ms * 1e-3) / 1e12
    roof_tab = dict(bound="hbm", achieved=round(tab_gbs, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                    frac=round(tab_gbs / HBM_PEAK_GBS, 4), traffic=None,
                    kernel="msv_tabulate (tabulate_kernel far + near launches)",
                    algorithmic_bytes=entries * 16)
    roof_lu = dict(bound="mfma", achieved=round(lu_tfs, 2), peak=BF16_MFMA_PEAK_TF, unit="TFLOP/s",
                   frac=round(lu_tfs / BF16_MFMA_PEAK_TF, 4), traffic=lu_traffic(),
                   kernel="msv_factor (complex64 LU: gemm_update_planes on bf16 MFMA, base_panel, laswp, trsm)",
                   algorithmic_flops=lu_flops, fp32_mfma_frac=round(lu_tfs / FP32_MFMA_PEAK_TF, 4))
    dominant = roof_lu if fac_ms >= tab_ms else roof_tab

    line = {
        "metric": "modal-kernel entries/s; per-mode solves/s and p99 latency at 1e-10 rel err",
        "value": entries / (ms_per_step * 1e-3),
        "unit": "modal-kernel entries/s (whole step)",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64 kernels/assembly/residual; complex64 LU, trailing updates as split-bf16 MFMA products",
        "data": "synthetic (closed-form body, seeded plane waves)",
        "config": {"workload": "prolate spheroid 1:3, 64 panels x 16 nodes (N=1024, 4096 unknowns/mode), "
                               "|m|<=64, L=256, k0=10, eps=4, mu=1, 8 plane waves seed 2, "
                               "complex64 LU + complex128 refinement",
                   "modes_factored": M + 1, "mode_solves": 2 * M + 1, "rhs": len(waves),
                   "table_entries": entries, "parallelism": "single GPU"},
        "phases_ms": {"tabulate": tab_ms, "assemble": asm_ms, "factor": fac_ms, "solve": sol_ms},
        "tabulation_entries_per_s": entries / (tab_ms * 1e-3),
        "per_mode_solves_per_s": (M + 1) / (ms_per_step * 1e-3),
        "step_latency_ms": {"p50": float(np.percentile(step_ms, 50)), "p99": float(np.percentile(step_ms, 99))},
        "ir_iterations": ir_iters,
        "roofline": dominant,
        "roofline_tabulate": roof_tab,
        "roofline_lu": roof_lu,
    }
    if not args.no_forms:
        del kern, A, x
        plan.close()
        torch.cuda.empty_cache()
        # the plain complex128 path on the same workload (precision form baseline)
        p0 = msv.plan_from_curve(curve, rls, cfg["k0"], cfg["eps1"], cfg["mu1"], m_max=M, fft_len=L, precision=0)
        k0t = torch.empty(p0.table_shape, dtype=torch.complex128, device=dev)
        A0 = torch.empty((M + 1, n, n), dtype=torch.complex128, device=dev)
        x0 = torch.empty_like(rhs)
        times = []
        for it in range(2):
            e = [ev() for _ in range(5)]
            e[0].record()
            p0.tabulate(out=k0t)
            e[1].record()
            p0.assemble(k0t, 0, M, out=A0)
            e[2].record()
            p0.factor(A0, 0, M)
            e[3].record()
            p0.solve(-M, M, rhs, out=x0)
            e[4].record()
            torch.cuda.synchronize()
            times.append([a.elapsed_time(b) for a, b in zip(e[:-1], e[1:])])
        t = times[-1]
        line["complex128_path"] = {"phases_ms": dict(zip(("tabulate", "assemble", "factor", "solve"), t)),
                                   "ms_per_step": sum(t), "per_mode_solves_per_s": (M + 1) / (sum(t) * 1e-3),
                                   "factor_tflops": lu_flops / (t[2] * 1e-3) / 1e12}
        del k0t, A0, x0, rhs
        p0.close()
        torch.cuda.empty_cache()
        print("[bench] batching form", file=sys.stderr, flush=True)
        line["batching"] = bench_batching(rls)
        torch.cuda.empty_cache()
        print("[bench] serving form", file=sys.stderr, flush=True)
        line["serving"] = {"complex64_lu_refined": bench_serving(rls, 1), "complex128_lu": bench_serving(rls, 0)}
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(curve, rls, cfg)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
