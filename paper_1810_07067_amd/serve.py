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
  kernels overlap on the device; while the oldest request waits for memory,
  requests for bodies already in the cache go ahead of it;
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
    rhs: object = None        # [2M+1, n_waves, 4N] incident modes (host); synthesized from waves if None


@dataclass
class Result:
    rid: int
    x: np.ndarray             # [2M+1, n_waves, 4N] currents
    latency: float            # arrival -> currents on the host, seconds
    cached: bool              # factors came from the cache
    ir_iterations: int
    mode_solves: int          # (2M+1) x n_waves
    build_s: float = 0.0      # tabulate, assemble and factor (the request that built the entry)
    wait_s: float = 0.0       # waiting for another request's build of the entry
    solve_s: float = 0.0      # upload, solve (and refinement), download
    host: object = None       # the pinned host tensor that x views, held for as long as x is


MAX_WAVES = 32  # plane waves per request
# a modal-kernel table larger than this is never resident: the body is
# tabulated and assembled in target-row blocks through one reused block
TABLE_BLOCK_BYTES = 8 << 30
# The tabulation runs faster in blocks of ~128 target rows than of 512 or of
# the whole table (each block's table is [mode][type][row][source], and its
# per-(mode, type) planes lie closer together in memory)
TABLE_BLOCK_ROWS = 128
MAX_SPLIT_MB = 2048  # cached allocator blocks above this are never split


def table_block_rows(curve, m_max, n_support):
    """Target rows per tabulate/assemble block, or None for the whole table:
    TABLE_BLOCK_ROWS, fewer where that many rows exceed TABLE_BLOCK_BYTES."""
    row = (m_max + 2) * 9 * (curve.n + n_support) * 16
    rows = min(TABLE_BLOCK_ROWS, max(16, TABLE_BLOCK_BYTES // row))
    return None if rows >= curve.n else rows


def entry_bytes(curve, m_max, fft_len, precision, n_support):
    """HBM held by a cache entry, and the transient extra while it is built.

    Held: the caller-owned complex128 matrices of modes 0..M plus everything
    the plan owns once factored and after its largest solve (2M+1 modes x
    MAX_WAVES vectors), as bounded by the library (msv_workspace_bytes:
    geometry, pivots, LU workspace, complex64 factors, block inverses, solve
    workspace), plus the request's right-hand sides and solutions.
    Transient: the modal-kernel table, or the one row block of it that a
    large body is assembled through, freed once the matrices are assembled."""
    import paper_1810_07067_amd as msv
    N = curve.n
    n = 4 * N
    nm = m_max + 1
    vectors = (2 * m_max + 1) * MAX_WAVES
    mats = nm * n * n * 16
    plan = msv.workspace_bytes(N, n_support, fft_len, nm, vectors, precision)
    io = 2 * vectors * n * 16
    rows = table_block_rows(curve, m_max, n_support) or N
    table = (m_max + 2) * 9 * rows * (N + n_support) * 16
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

    def __init__(self, rules, hbm_budget, slots=4, precision=1, ir_tol=1e-12, ir_max_iter=20, torch_pool=True):
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
        self.fallbacks = 0       # entries refactored with the complex128 LU
        self._mu = threading.Lock()
        self._streams = None
        # Entries come and go in sizes from megabytes to a third of the
        # device.  The caching allocator must not carve a freed entry's block
        # into pieces for smaller ones: a block it may not split is handed
        # back whole when a larger allocation fails, and the retry succeeds.
        import torch
        setting = f"max_split_size_mb:{MAX_SPLIT_MB}"
        if hasattr(torch._C, "_accelerator_setAllocatorSettings"):
            torch._C._accelerator_setAllocatorSettings(setting)
        else:
            torch.cuda.memory._set_allocator_settings(setting)
        # The library's own buffers (LU factors, workspaces) from the same pool
        # as the entries' matrices: memory that an evicted entry gives back is
        # taken again as it is.  (Returned to the driver instead, a block of
        # tens of GB has to be cleared again before the next allocation gets
        # it, about a second per 70 GB.)  Not possible while plans exist.
        self.torch_pool = False
        if torch_pool:
            import paper_1810_07067_amd as msv
            try:
                msv.use_torch_allocator()
                self.torch_pool = True
            except msv.MsvError:
                pass

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
                # every use of an idle entry ended with its stream synchronized
                victim.plan.close(wait=False)
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
            if not self.torch_pool:
                torch.cuda.empty_cache()  # matrices of evicted entries go back to the device
            rows = table_block_rows(req.curve, req.m_max, plan.S)
            # the matrices from the default stream's pool, where evicted
            # entries' memory goes back (every use of an entry has finished
            # before it is evicted)
            with torch.cuda.stream(torch.cuda.default_stream()):
                A = torch.empty((req.m_max + 1, plan.n, plan.n), dtype=torch.complex128, device="cuda")
            with torch.cuda.stream(stream):
                if rows is None:
                    kern = plan.tabulate(stream=stream)
                    plan.assemble(kern, 0, req.m_max, out=A, stream=stream)
                else:
                    plan.assemble_streamed(0, req.m_max, out=A, rows_per_block=rows, stream=stream)
                    kern = None
                stream.synchronize()
                # hand the table back before the factor storage is allocated
                # (at the largest bodies the two do not fit together; a pooled
                # allocation that fails releases the cached blocks and retries)
                del kern
                if not self.torch_pool:
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
        import paper_1810_07067_amd as msv
        e, builder, table_bytes = admitted
        stream = slot_streams.get()
        try:
            ts = time.perf_counter()
            if builder:
                self._build(e, req, table_bytes, stream)
            else:
                e.ready.wait()
            tb = time.perf_counter()
            if e.error is not None:
                raise e.error
            M = req.m_max
            rhs_h = req.rhs if req.rhs is not None else incident.rhs_modes(req.curve, req.waves, req.k0, -M, M)
            with e.lock:
                with torch.cuda.stream(stream):
                    rhs = torch.from_numpy(rhs_h).to("cuda", non_blocking=False)
                    try:
                        x = e.plan.solve(-M, M, rhs, stream=stream)
                    except msv.MsvError as exc:
                        if exc.status != msv.MSV_ENOCONV:
                            raise
                        self._fallback(e, req, stream)
                        x = e.plan.solve(-M, M, rhs, stream=stream)
                    # through pinned host memory (torch's host cache): a
                    # pageable copy of a gigabyte of currents runs at 4 GB/s
                    xp = torch.empty(x.shape, dtype=x.dtype, pin_memory=True)
                    xp.copy_(x, non_blocking=True)
                    stream.synchronize()
                    xh = xp.numpy()
                    iters = e.plan.last_ir_iterations()
            te = time.perf_counter()
            return Result(req.rid, xh, te - t0 - req.arrival, not builder, iters, (2 * M + 1) * len(req.waves),
                          build_s=tb - ts if builder else 0.0, wait_s=0.0 if builder else tb - ts,
                          solve_s=te - tb, host=xp)
        finally:
            with self._mu:
                e.users -= 1
                e.last_used = time.perf_counter()
            slot_streams.put(stream)

    def _fallback(self, e, req, stream):
        """The entry's refinement did not converge (its matrices too
        ill-conditioned for the complex64 factors): refactor them in place with
        the complex128 LU, which also shrinks the entry.  Under e.lock."""
        import paper_1810_07067_amd as msv
        e.plan.close()
        e.plan = None
        plan = msv.plan_from_curve(req.curve, self.rules, req.k0, req.eps1, req.mu1, m_max=req.m_max,
                                   fft_len=req.fft_len, precision=0)
        plan.factor(e.A, 0, req.m_max, stream=stream)
        e.plan = plan
        (ys, _), (ya, _) = self.rules
        keep, _ = entry_bytes(req.curve, req.m_max, req.fft_len, 0, ys.shape[1] + 2 * ya.size)
        with self._mu:
            self.used -= e.bytes - keep
            e.bytes = keep
            self.fallbacks += 1

    def close(self, release=False):
        """Drop every cache entry (plans and matrices).  Their memory stays in
        torch's caching allocator for the next server or tensor of the
        process; release=True also returns it to the driver (memory returned
        and taken again has made the next builds several times slower)."""
        import torch
        with self._mu:
            for e in self.cache.values():
                if e.plan is not None:
                    e.plan.close()
                e.plan = None
                e.A = None
            self.cache.clear()
            self.used = 0
        torch.cuda.synchronize()
        if release:
            torch.cuda.empty_cache()

    # ------------------------------------------------------------------- run
    def _new_streams(self):
        """One HIP stream per slot."""
        import torch
        return [torch.cuda.Stream() for _ in range(self.slots)]

    def run(self, requests, realtime=True):
        """Serve `requests` (arrival times in seconds from now).  realtime=False
        treats every request as already arrived.  Returns results by rid and
        the wall time."""
        import queue

        if self._streams is None:
            self._streams = self._new_streams()
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
        arrived = []  # arrived and not yet admitted, in arrival order
        with ThreadPoolExecutor(max_workers=self.slots) as pool:
            while pending or arrived or inflight:
                now = time.perf_counter() - t0
                while pending and pending[0][0] <= now:
                    arrived.append(heapq.heappop(pending)[2])
                # admit in arrival order while a slot and memory are free; while
                # the oldest request waits for memory, requests for bodies
                # already in the cache (they need none) go ahead of it
                i = 0
                while i < len(arrived) and len(inflight) < self.slots:
                    req = arrived[i]
                    if i > 0 and self.key(req) not in self.cache:
                        i += 1
                        continue
                    with self._mu:
                        adm = self._try_admit(req)
                    if not adm:
                        i += 1
                        continue
                    arrived.pop(i)
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
