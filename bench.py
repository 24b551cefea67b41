"""Benchmark: one step = the whole hot path on one body, inputs resident in HBM.

Headline workload (the largest single-GPU configuration): a finite cylinder of
radius 1 and height 2 with its four corner-adjacent panels refined dyadically
24 times toward the edges (128 panels x 16 Gauss-Legendre nodes, N = 2048,
8192 unknowns per mode), modes |m| <= 128, azimuthal FFT length 512, k0 = 20,
eps1 = 4 + 0.1i, mu1 = 1, one plane wave at the paper's default angles.  A
step is

  tabulate + assemble   modal Green's functions for every pair incl. the
                        near-panel support nodes, streamed in blocks of 512
                        target rows through one table block, each block
                        assembled into its rows of the 129 per-mode
                        Mueller-Nystrom matrices (m = 0..128)
  factor                complex64 LU on MFMA of all 129 modes
  solve                 complex128-refined solves for m = -128..128

The whole 87 GB table never coexists with the 138 GB of complex128 matrices
and the 69 GB of complex64 factors.  `--config spheroid` runs the prolate
spheroid 1:3 (64 panels, N = 1024, |m| <= 64, L = 256, k0 = 10, eps1 = 4,
eight plane waves from seed 2) instead.  Prints one JSON line.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--config cylinder|spheroid]
                       [--no-cpu-baseline] [--no-forms]
       python bench.py --form batching|serving|extinction   (the batching and serving forms, the accuracy experiment)
       python bench.py --profile-target lu|tabulate|copy [--config ...]   (one piece, for counters)
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

METRIC = "modal-kernel entries/s; per-mode solves/s and p99 latency at 1e-10 rel err"


def workload(name="cylinder"):
    """Curve, rules, plane waves and parameters of a named workload."""
    from workloads import geometry, incident, rules
    if name == "cylinder":
        curve = geometry.cylinder(24)
        cfg = dict(name=name, k0=20.0, eps1=4.0 + 0.1j, mu1=1.0, M=128, L=512, rows_per_block=128,
                   desc="finite cylinder r=1, h=2, corner panels refined 24 times toward the edges "
                        "(128 panels x 16 nodes, N=2048, 8192 unknowns/mode), |m|<=128, L=512, k0=20, "
                        "eps=4+0.1i, mu=1, 1 plane wave at the paper's default angles, complex64 LU + "
                        "complex128 refinement, table streamed in 128-row blocks")
        waves = [incident.paper_default_direction()]
    elif name == "spheroid":
        curve = geometry.spheroid(64, 3.0)
        cfg = dict(name=name, k0=10.0, eps1=4.0, mu1=1.0, M=64, L=256, rows_per_block=128,
                   desc="prolate spheroid 1:3, 64 panels x 16 nodes (N=1024, 4096 unknowns/mode), |m|<=64, "
                        "L=256, k0=10, eps=4, mu=1, 8 plane waves seed 2, complex64 LU + complex128 refinement, "
                        "table streamed in 128-row blocks")
        waves = incident.random_directions(2, 8)
    else:
        raise ValueError(name)
    return curve, rules.load_rules(), waves, cfg


def _internal_constant(name):
    """The value of an integer constant of csrc/msv_internal.h (a constexpr,
    or the default of a macro), as written there."""
    import re
    text = open(os.path.join(ROOT, "paper_1810_07067_amd", "csrc", "msv_internal.h")).read()
    m = re.search(rf"(?:constexpr int {name} =|#define {name}) (\d+)", text)
    return m.group(1) if m else None


def _counted_bytes(profile, source, constants, label, rows=None):
    """HBM bytes recorded under `label` in a committed counter summary, while
    the kernel source (SHA-256), the launch constants and (if given) the
    table rows per block recorded with them are the current ones; None
    otherwise."""
    import hashlib
    import re
    try:
        text = open(os.path.join(ROOT, "profiles", profile)).read()
        src = open(os.path.join(ROOT, "paper_1810_07067_amd", "csrc", source), "rb").read()
        values = {c: _internal_constant(c) for c in constants}
    except OSError:
        return None
    h = re.search(rf"{re.escape(source)} sha256 = ([0-9a-f]{{64}})", text)
    b = re.search(rf"{label} = (\d+)", text)
    if not h or not b or h.group(1) != hashlib.sha256(src).hexdigest():
        return None
    for c, v in values.items():
        m = re.search(rf"{c} = (\d+)", text)
        if not m or m.group(1) != v:
            return None
    if rows is not None:
        r = re.search(r"rows per block = (\d+)", text)
        if not r or int(r.group(1)) != rows:
            return None
    return int(b.group(1))


def lu_traffic(config):
    """HBM bytes of one factorization (committed rocprofv3 counter summary of
    this workload, while the LU source, its number of stream groups and the
    smallest order it staggers are the ones counted), else None."""
    return _counted_bytes(f"lu_{config}_traffic.md", "lu.hip", ("MSV_LU_GROUPS", "kStaggerMinOrder"),
                          "lu traffic bytes per factorization")


def tab_traffic(config):
    """HBM bytes of one tabulation (committed counter summary, while the
    tabulation source, its spectra chunk and the workload's table rows per
    block are the ones counted), else None."""
    rows = workload(config)[3]["rows_per_block"]
    return _counted_bytes(f"tabulate_{config}_counters.md", "tabulate.hip", ("kSpecCap",), "tabulation traffic bytes",
                          rows=rows)


# --------------------------------------------------------------------------
# CPU baseline: the FP64 oracle on the host, phases as in the paper's tables
# (T_kernel, T_matgen, T_solve), on bounded samples of the same workload.
# --------------------------------------------------------------------------
def _oracle_rows_worker(args):
    import numpy as _np
    from oracle import discretize, modal
    name, rows, budget_s = args
    curve, rls, _, cfg = workload(name)
    sup = discretize.support_points(curve, *rls)
    k1 = cfg["k0"] * _np.sqrt(complex(cfg["eps1"] * cfg["mu1"]))
    kp = modal.KernelParams(cfg["k0"], k1, cfg["M"], cfg["L"], float(curve.r.max()))
    done, entries, t0 = 0, 0, time.perf_counter()
    for r in rows:
        if time.perf_counter() - t0 > budget_s:
            break
        entries += modal.tabulate(curve, sup, kp, rows=[int(r)]).size
        done += 1
    return done, entries, time.perf_counter() - t0


def host_cores():
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(n, 16))


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(name, kernel_s=8.0):
    """Oracle throughput on the host: modal-kernel entries/s on random target
    rows (one process per core, and one core alone), assembled matrix rows/s
    for a few modes, and the per-mode LU (numpy/LAPACK, all cores) at full
    order on a seeded matrix of the workload's size."""
    import multiprocessing as mp

    from threadpoolctl import threadpool_limits

    from oracle import assemble as oasm
    from oracle import discretize, modal
    from oracle import solve as osolve
    from workloads import geometry

    curve, rls, _, cfg = workload(name)
    N, M = curve.n, cfg["M"]
    n = 4 * N
    cores = host_cores()
    rng = np.random.default_rng(0)
    rows = rng.permutation(N)
    # T_kernel, one core
    with threadpool_limits(1):
        d1, e1, t1 = _oracle_rows_worker((name, rows[:64], kernel_s))
    one_core = e1 / t1
    # T_kernel, every core: disjoint row samples, one process each
    chunks = [rows[64 + i::cores][:64] for i in range(cores)]
    ctx = mp.get_context("spawn")
    t0 = time.perf_counter()
    with ctx.Pool(cores) as pool:
        res = pool.map(_oracle_rows_worker, [(name, c, kernel_s) for c in chunks])
    wall = time.perf_counter() - t0
    rows_all = sum(r[0] for r in res)
    ent_all = sum(r[1] for r in res)
    # per process the rate is entries / its own time; the aggregate is the sum
    all_cores = sum(r[1] / r[2] for r in res if r[2] > 0)
    # T_matgen: oracle assembly of sampled rows (its own table rows) for 2 modes
    sup = discretize.support_points(curve, *rls)
    k1 = cfg["k0"] * np.sqrt(complex(cfg["eps1"] * cfg["mu1"]))
    kp = modal.KernelParams(cfg["k0"], k1, M, cfg["L"], float(curve.r.max()))
    srows = rows[:4]
    tab = modal.tabulate(curve, sup, kp, rows=srows)
    w = geometry.gl_weights(curve)
    t0 = time.perf_counter()
    for m in (0, M // 2):
        oasm.assemble_mode(curve, sup, tab, m, cfg["k0"], k1, cfg["k0"], 1.0, 1.0, cfg["eps1"], cfg["mu1"], w,
                           rows=srows)
    tmat = time.perf_counter() - t0
    matrows_per_s = 2 * len(srows) / tmat
    # T_solve: one mode's dense solve (seeded matrix) at order <= 4096,
    # extrapolated as n^3 to the workload's order
    nl = min(n, 4096)
    A = rng.standard_normal((nl, nl)) + 1j * rng.standard_normal((nl, nl)) + 8 * np.sqrt(nl) * np.eye(nl)
    b = rng.standard_normal((1, 1, nl)) + 0j
    t0 = time.perf_counter()
    osolve.solve_modes([A], np.ones(nl // 4), b, 0, 0)
    tlu_s = time.perf_counter() - t0
    flops = (8.0 / 3.0) * nl ** 3
    tlu = tlu_s * (n / nl) ** 3
    return dict(
        value=all_cores, unit="modal-kernel entries/s", cores=cores, kind="oracle",
        cpu=cpu_model(),
        sample=f"{rows_all} random target rows x {N + sup.r.shape[1]} sources x {M + 2} modes x 9 types, one "
               f"process per core ({wall:.1f} s wall); numpy FP64",
        one_core=dict(value=one_core, unit="modal-kernel entries/s", sample=f"{d1} rows ({t1:.1f} s)"),
        phases=dict(
            T_kernel_s_extrapolated=(M + 2) * 9 * N * (N + sup.r.shape[1]) / all_cores,
            T_matgen_s_extrapolated=(M + 1) * N / matrows_per_s / cores,
            T_solve_s_extrapolated=(M + 1) * tlu,
            note=f"T_kernel from the all-core row rate; T_matgen from {2 * len(srows)} target-row x mode "
                 f"assemblies ({tmat * 1e3:.0f} ms, one core) divided over {cores} cores; T_solve = (M+1) x one "
                 f"{nl}x{nl} complex128 LAPACK solve ({tlu_s:.1f} s, {flops / tlu_s / 1e9:.0f} GFLOP/s, OpenBLAS "
                 f"threads = {cores}) scaled by ({n}/{nl})^3; all extrapolated from the samples"),
    )


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


# --------------------------------------------------------------------------
# the step
# --------------------------------------------------------------------------
class Step:
    """Buffers and the launch sequence of one step of a workload."""

    def __init__(self, name, precision, torch, msv):
        self.torch = torch
        curve, rls, waves, cfg = workload(name)
        self.curve, self.waves, self.cfg = curve, waves, cfg
        M = cfg["M"]
        self.M = M
        from workloads import incident
        rhs_h = incident.rhs_modes(curve, waves, cfg["k0"], -M, M)
        self.plan = msv.plan_from_curve(curve, rls, cfg["k0"], cfg["eps1"], cfg["mu1"], m_max=M, fft_len=cfg["L"],
                                        precision=precision, ir_tol=1e-12, ir_max_iter=20)
        dev = torch.device("cuda:0")
        p = self.plan
        self.nb = cfg["rows_per_block"] or curve.n
        self.kblock = torch.empty(p.table_rows_shape(self.nb), dtype=torch.complex128, device=dev)
        self.A = torch.empty((M + 1, p.n, p.n), dtype=torch.complex128, device=dev)
        self.rhs = torch.from_numpy(rhs_h).to(dev)
        self.x = torch.empty_like(self.rhs)
        self.entries = p.table_entries

    def run(self):
        """Enqueue one step; returns the events [tab/asm per block..., factor, solve]."""
        torch, p, M = self.torch, self.plan, self.M
        ev = lambda: torch.cuda.Event(enable_timing=True)
        marks = []
        for t0 in range(0, p.N, self.nb):
            nt = min(self.nb, p.N - t0)
            kb = self.kblock.view(-1)[: (M + 2) * 9 * nt * (p.N + p.S)].view(p.table_rows_shape(nt))
            e = [ev(), ev(), ev()]
            e[0].record()
            p.tabulate_rows(t0, nt, out=kb)
            e[1].record()
            p.assemble_rows(kb, t0, nt, 0, M, self.A)
            e[2].record()
            marks.append(e)
        f = [ev(), ev(), ev()]
        f[0].record()
        p.factor(self.A, 0, M)
        f[1].record()
        p.solve(-M, M, self.rhs, out=self.x)
        f[2].record()
        return marks, f

    @staticmethod
    def phases(rec):
        marks, f = rec
        tab = sum(e[0].elapsed_time(e[1]) for e in marks)
        asm = sum(e[1].elapsed_time(e[2]) for e in marks)
        return tab, asm, f[0].elapsed_time(f[1]), f[1].elapsed_time(f[2])

    def close(self):
        self.plan.close()
        del self.kblock, self.A, self.rhs, self.x
        self.torch.cuda.empty_cache()


def run_steps(name, precision, steps, warmup, torch, msv, verbose=True):
    st = Step(name, precision, torch, msv)
    print(f"[bench] {name}: N={st.curve.n} M={st.M} L={st.cfg['L']} precision={precision} "
          f"rhs={tuple(st.rhs.shape)}", file=sys.stderr, flush=True)
    for i in range(warmup):
        st.run()
        torch.cuda.synchronize()
        if verbose:
            print(f"[bench] warmup {i} done", file=sys.stderr, flush=True)
    recs = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        recs.append(st.run())
        if verbose:
            print(f"[bench] step {i} enqueued", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ph = np.array([Step.phases(r) for r in recs])  # ms
    return st, wall, ph


def rooflines(st, ph, config):
    n, M = st.plan.n, st.M
    tab_ms, asm_ms, fac_ms, sol_ms = ph.mean(axis=0)
    tab_gbs = st.entries * 16 / (tab_ms * 1e-3) / 1e9
    lu_flops = (8.0 / 3.0) * n ** 3 * (M + 1)
    lu_tfs = lu_flops / (fac_ms * 1e-3) / 1e12
    tt = tab_traffic(config)
    roof_tab = dict(bound="hbm", achieved=round(tab_gbs, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                    frac=round(tab_gbs / HBM_PEAK_GBS, 4), traffic=tt,
                    kernel="msv_tabulate_rows (tabulate_kernel far + near launches, all row blocks)",
                    algorithmic_bytes=st.entries * 16)
    roof_lu = dict(bound="mfma", achieved=round(lu_tfs, 2), peak=BF16_MFMA_PEAK_TF, unit="TFLOP/s",
                   frac=round(lu_tfs / BF16_MFMA_PEAK_TF, 4), traffic=lu_traffic(config),
                   kernel="msv_factor (complex64 LU: gemm_update_planes on bf16 MFMA, base_panel, laswp, trsm)",
                   algorithmic_flops=lu_flops, fp32_mfma_frac=round(lu_tfs / FP32_MFMA_PEAK_TF, 4))
    return roof_tab, roof_lu


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", choices=["cylinder", "spheroid"], default="cylinder")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-forms", action="store_true",
                    help="skip the complex128-path comparison and the secondary workload")
    ap.add_argument("--form", choices=["batching", "serving", "extinction"],
                    help="measure the batching, serving or extinction form instead of the step (separate JSON line)")
    ap.add_argument("--modes", type=int, default=None,
                    help="with --profile-target lu: factor modes 0..modes-1 only")
    ap.add_argument("--profile-target", choices=["lu", "tabulate", "copy"],
                    help="run one piece once for hardware counters and exit: the LU of the workload, "
                         "its tabulation, or a 1 GiB device copy (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on exactly one GPU (got --gpus {args.gpus}); the modes shard "
              "across GPUs without communication but that path is not built here", file=sys.stderr)
        sys.exit(2)
    if args.profile_target:
        from bench_forms import profile_target
        profile_target(args.profile_target, args.config, args.modes)
        return
    if args.form:
        from bench_forms import run_form
        print(json.dumps(run_form(args.form)), flush=True)
        return

    # the oracle runs first, in worker processes started before this process
    # touches the GPU
    cpu = None
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline", file=sys.stderr, flush=True)
        cpu = cpu_baseline(args.config)

    import torch
    import paper_1810_07067_amd as msv

    st, wall, ph = run_steps(args.config, 1, args.steps, args.warmup, torch, msv)
    step_ms = ph.sum(axis=1)
    ms_per_step = wall * 1e3 / args.steps
    tab_ms, asm_ms, fac_ms, sol_ms = ph.mean(axis=0)
    roof_tab, roof_lu = rooflines(st, ph, args.config)
    dominant = roof_lu if fac_ms >= tab_ms else roof_tab
    M, cfg = st.M, st.cfg
    line = {
        "metric": METRIC,
        "value": st.entries / (ms_per_step * 1e-3),
        "unit": "modal-kernel entries/s (whole step)",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64 kernels/assembly/residual; complex64 LU, trailing updates as split-bf16 MFMA products",
        "data": "synthetic (closed-form body, plane waves)",
        "config": {"workload": cfg["desc"], "modes_factored": M + 1, "mode_solves": 2 * M + 1,
                   "rhs": len(st.waves), "table_entries": st.entries, "parallelism": "single GPU"},
        "phases_ms": {"tabulate": tab_ms, "assemble": asm_ms, "factor": fac_ms, "solve": sol_ms},
        "tabulation_entries_per_s": st.entries / (tab_ms * 1e-3),
        "per_mode_solves_per_s": (M + 1) / (ms_per_step * 1e-3),
        "step_latency_ms": {"p50": float(np.percentile(step_ms, 50)), "p99": float(np.percentile(step_ms, 99))},
        "ir_iterations": st.plan.last_ir_iterations(),
        "roofline": dominant,
        "roofline_tabulate": roof_tab,
        "roofline_lu": roof_lu,
    }
    st.close()
    del st
    torch.cuda.empty_cache()
    if not args.no_forms:
        # the plain complex128 path on the same workload (the precision form's baseline)
        print("[bench] complex128 path", file=sys.stderr, flush=True)
        s0, wall0, ph0 = run_steps(args.config, 0, 1, 0, torch, msv)
        t = ph0.mean(axis=0)
        line["complex128_path"] = {
            "phases_ms": dict(zip(("tabulate", "assemble", "factor", "solve"), t.tolist())),
            "ms_per_step": float(t.sum()), "per_mode_solves_per_s": (M + 1) / (t.sum() * 1e-3),
            "factor_tflops": (8.0 / 3.0) * s0.plan.n ** 3 * (M + 1) / (t[2] * 1e-3) / 1e12,
            "factor_fp64_frac": (8.0 / 3.0) * s0.plan.n ** 3 * (M + 1) / (t[2] * 1e-3) / 1e12 / FP64_PEAK_TF}
        s0.close()
        del s0
        torch.cuda.empty_cache()
        other = "spheroid" if args.config == "cylinder" else "cylinder"
        if other == "spheroid":
            print("[bench] secondary workload", file=sys.stderr, flush=True)
            s2, wall2, ph2 = run_steps(other, 1, 5, 1, torch, msv, verbose=False)
            rt, rl = rooflines(s2, ph2, other)
            t2 = ph2.mean(axis=0)
            line["secondary"] = {"workload": s2.cfg["desc"], "ms_per_step": wall2 * 1e3 / 5,
                                 "phases_ms": dict(zip(("tabulate", "assemble", "factor", "solve"), t2.tolist())),
                                 "value": s2.entries / (wall2 / 5), "roofline_tabulate": rt, "roofline_lu": rl}
            s2.close()
            del s2
            torch.cuda.empty_cache()
    if cpu is not None:
        line["cpu_baseline"] = cpu
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
