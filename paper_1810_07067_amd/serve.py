"""Serving form: a request loop over the msv C-ABI.

A request is one scattering solve: a body (generating curve), k0, the
interior material, a mode range and 1..32 incident plane waves.  The server

* keeps, per (body, k0, material, modes), the assembled complex128 matrices and
  their factors resident in HBM (a factorization cache): a repeated body only
  needs right-hand sides and solves (the paper's observation that further
  right-hand sides are cheap once the modes are factored, Section 6);
* admits requests continuously, in arrival order, as soon as a slot (a worker
  with its own HIP stream) and HBM budget are free -- requests that arrive
  while others are on the GPU start without waiting for them, and their
  kernels overlap on the device;
* evicts idle cache entries, least recently used first, when a new body does
  not fit the budget;
* records per request the latency from arrival to currents on the host.

All numerical work is done by the library (tabulate, assemble, factor, solve);
this module only schedules.  The plane-wave right-hand sides are synthesized
on the host (workloads.incident).
"""
from __future__ import annotations

import heapq
import threading
import time
from concurrent.futures import FIRST_COMPLETED, ThreadPoolExecutor, wait
from dataclasses import dataclass, field

import numpy as np


@dataclass
class Request:
    rid: int
    body: str                 # name of the geometry (cache key part)
    curve: object             # workloads.geometry.Curve
    k0: float
    eps1: complex
    m_max: int
    fft_len: int
    waves: list               # [(d, p)] plane waves
    arrival: float = 0.0      # seconds after the start of the stream
    mu1: complex = 1.0


@dataclass
class Result:
    rid: int
    x: np.ndarray             # [2M+1, n_waves, 4N] currents
    latency: float            # arrival -> currents on the host, seconds
    cached: bool              # factors came from the cache
    ir_iterations: int
    mode_solves: int          # (2M+1) x n_waves


MAX_WAVES = 32  # plane waves per request


def entry_bytes(curve, m_max, fft_len, precision, n_support):
    """HBM held by a cache entry, and the transient extra while it is built.

    Held: the caller-owned complex128 matrices of modes 0..M plus everything
    the plan owns once factored and after its largest solve (2M+1 modes x
    MAX_WAVES vectors), as bounded by the library (msv_workspace_bytes:
    geometry, pivots, LU workspace, complex64 factors, block inverses, solve
    workspace), plus the request's right-hand sides and solutions.
    Transient: the modal-kernel table, freed once the matrices are assembled."""
    import paper_1810_07067_amd as msv
    N = curve.n
    n = 4 * N
    nm = m_max + 1
    vectors = (2 * m_max + 1) * MAX_WAVES
    mats = nm * n * n * 16
    plan = msv.workspace_bytes(N, n_support, fft_len, nm, vectors, precision)
    io = 2 * vectors * n * 16
    table = (m_max + 2) * 9 * N * (N + n_support) * 16
    return mats + plan + io, table


@dataclass
class _Entry:
    key: tuple
    plan: object = None
    A: object = None
    bytes: int = 0
    users: int = 0
    last_used: float = 0.0
    ready: threading.Event = field(default_factory=threading.Event)
    lock: threading.Lock = field(default_factory=threading.Lock)  # one solve at a time per plan
    error: BaseException | None = None


class Server:
    """Continuous-batching scheduler with a resident factorization cache."""

    def __init__(self, rules, hbm_budget, slots=4, precision=1, ir_tol=1e-12, ir_max_iter=20):
        self.rules = rules
        self.budget = int(hbm_budget)
        self.slots = int(slots)
        self.precision = int(precision)
        self.ir_tol = ir_tol
        self.ir_max_iter = ir_max_iter
        self.cache: dict[tuple, _Entry] = {}
        self.used = 0            # bytes held by cache entries and transient tables
        self.hits = 0
        self.misses = 0
        self.evictions = 0
        self._mu = threading.Lock()
        self._streams = None

    # ------------------------------------------------------------------ keys
    @staticmethod
    def key(req: Request):
        return (req.body, float(req.k0), complex(req.eps1), complex(req.mu1), int(req.m_max), int(req.fft_len))

    # ------------------------------------------------------------- admission
    def _footprint(self, req):
        """Bytes a request needs admitted: 0 for a cached (or in-build) body."""
        if self.key(req) in self.cache:
            return 0, 0
        (ys, _), (ya, _) = self.rules
        keep, table = entry_bytes(req.curve, req.m_max, req.fft_len, self.precision, ys.shape[1] + 2 * ya.size)
        return keep, table

    def _try_admit(self, req):
        """Reserve memory for req; evict idle entries if needed.  Under _mu."""
        keep, table = self._footprint(req)
        need = keep + table
        if need > self.budget:
            raise MemoryError(f"request {req.rid} needs {need} B, budget {self.budget} B")
        while self.used + need > self.budget:
            idle = [e for e in self.cache.values() if e.users == 0 and e.ready.is_set()]
            if not idle:
                return False
            victim = min(idle, key=lambda e: e.last_used)
            del self.cache[victim.key]
            self.used -= victim.bytes
            if victim.plan is not None:
                victim.plan.close()
            victim.plan = None
            victim.A = None
            self.evictions += 1
        k = self.key(req)
        if k not in self.cache:
            self.cache[k] = _Entry(key=k, bytes=keep)
            self.used += need  # the table part is returned once the entry is built
            self.misses += 1
            builder = True
        else:
            self.hits += 1
            builder = False
        e = self.cache[k]
        e.users += 1
        return (e, builder, table)

    # ---------------------------------------------------------------- worker
    def _build(self, e, req, table_bytes, stream):
        import torch

        import paper_1810_07067_amd as msv
        try:
            plan = msv.plan_from_curve(req.curve, self.rules, req.k0, req.eps1, req.mu1, m_max=req.m_max,
                                       fft_len=req.fft_len, precision=self.precision, ir_tol=self.ir_tol,
                                       ir_max_iter=self.ir_max_iter)
            torch.cuda.empty_cache()  # matrices of evicted entries go back to the device
            with torch.cuda.stream(stream):
                kern = plan.tabulate(stream=stream)
                A = plan.assemble(kern, 0, req.m_max, stream=stream)
                stream.synchronize()
                # hand the table back to the device before the factor storage
                # is allocated (at the largest bodies the two do not fit together)
                del kern
                torch.cuda.empty_cache()
                with self._mu:
                    self.used -= table_bytes
                    table_bytes = 0
                plan.factor(A, 0, req.m_max, stream=stream)
                stream.synchronize()
            e.plan, e.A = plan, A
        except BaseException as exc:  # reported to every user of the entry
            e.error = exc
        finally:
            with self._mu:
                self.used -= table_bytes
            e.ready.set()

    def _serve_one(self, req, admitted, t0, slot_streams):
        import torch

        from workloads import incident
        e, builder, table_bytes = admitted
        stream = slot_streams.get()
        try:
            if builder:
                self._build(e, req, table_bytes, stream)
            else:
                e.ready.wait()
            if e.error is not None:
                raise e.error
            M = req.m_max
            rhs_h = incident.rhs_modes(req.curve, req.waves, req.k0, -M, M)
            with e.lock:
                with torch.cuda.stream(stream):
                    rhs = torch.from_numpy(rhs_h).to("cuda", non_blocking=False)
                    x = e.plan.solve(-M, M, rhs, stream=stream)
                    xh = x.cpu().numpy()
                    iters = e.plan.last_ir_iterations()
            done = time.perf_counter() - t0
            return Result(req.rid, xh, done - req.arrival, not builder, iters, (2 * M + 1) * len(req.waves))
        finally:
            with self._mu:
                e.users -= 1
                e.last_used = time.perf_counter()
            slot_streams.put(stream)

    # ------------------------------------------------------------------- run
    def run(self, requests, realtime=True):
        """Serve `requests` (arrival times in seconds from now).  realtime=False
        treats every request as already arrived.  Returns results by rid and
        the wall time."""
        import queue

        import torch
        if self._streams is None:
            self._streams = [torch.cuda.Stream() for _ in range(self.slots)]
        slot_streams = queue.Queue()
        for s in self._streams:
            slot_streams.put(s)
        pending = [(r.arrival if realtime else 0.0, r.rid, r) for r in requests]
        heapq.heapify(pending)
        results = {}
        t0 = time.perf_counter()
        if not realtime:
            for r in requests:
                r.arrival = 0.0
        inflight = set()
        with ThreadPoolExecutor(max_workers=self.slots) as pool:
            while pending or inflight:
                now = time.perf_counter() - t0
                # admit in arrival order while a slot and memory are free
                while pending and pending[0][0] <= now and len(inflight) < self.slots:
                    req = pending[0][2]
                    with self._mu:
                        adm = self._try_admit(req)
                    if not adm:
                        break
                    heapq.heappop(pending)
                    inflight.add(pool.submit(self._serve_one, req, adm, t0, slot_streams))
                timeout = None
                if pending and len(inflight) < self.slots:
                    timeout = max(0.0, pending[0][0] - (time.perf_counter() - t0))
                if inflight:
                    done, _ = wait(inflight, timeout=timeout if timeout is not None else 0.5,
                                   return_when=FIRST_COMPLETED)
                    for f in done:
                        inflight.discard(f)
                        res = f.result()
                        results[res.rid] = res
                elif timeout:
                    time.sleep(min(timeout, 0.05))
        wall = time.perf_counter() - t0
        return results, wall


def latency_stats(results):
    lat = np.array([r.latency for r in results.values()])
    return {"p50_ms": float(np.percentile(lat, 50) * 1e3), "p99_ms": float(np.percentile(lat, 99) * 1e3),
            "mean_ms": float(lat.mean() * 1e3)}


def poisson_arrivals(rng, n, qps):
    """n arrival times of a Poisson stream at rate qps (seconds)."""
    return np.cumsum(rng.exponential(1.0 / qps, size=n))
