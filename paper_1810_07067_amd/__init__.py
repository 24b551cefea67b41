"""Python binding of the msv C-ABI (include/msv.h): argument marshalling only.

Every step of the method runs in the HIP library libmsv.so built from csrc/
(see build.py); PyTorch provides device memory and streams.  Importing this
package does not load the library; the first Plan does, and fails loudly if it
has not been built.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmsv.so")

MSV_OK, MSV_EINVAL, MSV_ENOMEM, MSV_EHIP, MSV_ESINGULAR, MSV_ENOCONV = range(6)
_STATUS = {1: "EINVAL", 2: "ENOMEM", 3: "EHIP", 4: "ESINGULAR", 5: "ENOCONV"}

EXPORTS = ["msv_plan_create", "msv_plan_destroy", "msv_last_error", "msv_num_nodes",
           "msv_num_support", "msv_table_entries", "msv_matrix_order", "msv_tabulate",
           "msv_assemble", "msv_factor", "msv_solve", "msv_last_ir_iterations",
           "msv_batch_create", "msv_batch_factor", "msv_batch_destroy", "msv_batch_last_error",
           "msv_batch_panel", "msv_batch_tuned_ms", "msv_workspace_bytes", "msv_plan_device_bytes", "msv_set_allocator",
           "msv_batch_plane_min", "msv_batch_tuned_plane_ms", "msv_batch_tuned_from_table",
           "msv_tabulate_rows", "msv_assemble_rows", "msv_solve_noalloc", "msv_solve_noalloc_max_bytes",
           "msv_far_field", "msv_fields"]


class MsvError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"msv {_STATUS.get(status, status)}: {msg}")
        self.status = status


class c128(ctypes.Structure):
    _fields_ = [("re", ctypes.c_double), ("im", ctypes.c_double)]


class Curve(ctypes.Structure):
    _fields_ = [("n_panels", ctypes.c_int32), ("order", ctypes.c_int32), ("closed", ctypes.c_int32),
                ("h_r", ctypes.c_void_p), ("h_z", ctypes.c_void_p), ("h_nr", ctypes.c_void_p),
                ("h_nz", ctypes.c_void_p), ("h_dsdu", ctypes.c_void_p)]


class Rules(ctypes.Structure):
    _fields_ = [("n_self", ctypes.c_int32), ("h_self_u", ctypes.c_void_p), ("h_self_w", ctypes.c_void_p),
                ("n_adj", ctypes.c_int32), ("h_adj_u", ctypes.c_void_p), ("h_adj_w", ctypes.c_void_p)]


class Desc(ctypes.Structure):
    _fields_ = [("k0", ctypes.c_double), ("eps0", c128), ("mu0", c128), ("eps1", c128), ("mu1", c128),
                ("m_max", ctypes.c_int32), ("fft_len", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("ir_tol", ctypes.c_double), ("ir_max_iter", ctypes.c_int32), ("formulation", ctypes.c_int32)]


_lib = None


def load_library(path: str = LIB_PATH):
    """Load libmsv.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: run `python -m paper_1810_07067_amd.build` first")
    lib = ctypes.CDLL(path)
    P = ctypes.c_void_p
    lib.msv_plan_create.argtypes = [ctypes.POINTER(P), ctypes.POINTER(Curve), ctypes.POINTER(Rules),
                                    ctypes.POINTER(Desc), P]
    lib.msv_plan_create.restype = ctypes.c_int
    lib.msv_plan_destroy.argtypes = [P]
    lib.msv_plan_destroy.restype = None
    lib.msv_last_error.argtypes = [P]
    lib.msv_last_error.restype = ctypes.c_char_p
    for f in ("msv_num_nodes", "msv_num_support", "msv_matrix_order", "msv_last_ir_iterations"):
        getattr(lib, f).argtypes = [P]
        getattr(lib, f).restype = ctypes.c_int32
    lib.msv_table_entries.argtypes = [P]
    lib.msv_table_entries.restype = ctypes.c_size_t
    lib.msv_tabulate.argtypes = [P, P, ctypes.c_size_t, P]
    lib.msv_tabulate.restype = ctypes.c_int
    lib.msv_assemble.argtypes = [P, P, ctypes.c_int32, ctypes.c_int32, P, P]
    lib.msv_assemble.restype = ctypes.c_int
    lib.msv_factor.argtypes = [P, P, ctypes.c_int32, ctypes.c_int32, P]
    lib.msv_factor.restype = ctypes.c_int
    lib.msv_solve.argtypes = [P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, P, P, P]
    lib.msv_solve.restype = ctypes.c_int
    lib.msv_solve_noalloc.argtypes = [P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, P, P, P]
    lib.msv_solve_noalloc.restype = ctypes.c_int
    lib.msv_far_field.argtypes = [P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, P, ctypes.c_int32, P, P, P]
    lib.msv_far_field.restype = ctypes.c_int
    lib.msv_fields.argtypes = [P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, P, ctypes.c_int32, P,
                               ctypes.c_int32, ctypes.c_int32, P, P, P]
    lib.msv_fields.restype = ctypes.c_int
    lib.msv_solve_noalloc_max_bytes.argtypes = []
    lib.msv_solve_noalloc_max_bytes.restype = ctypes.c_size_t
    lib.msv_batch_create.argtypes = [ctypes.POINTER(P), ctypes.POINTER(P), ctypes.POINTER(P), ctypes.c_int32,
                                     ctypes.c_int32, ctypes.c_int32, P]
    lib.msv_batch_create.restype = ctypes.c_int
    lib.msv_batch_factor.argtypes = [P, P]
    lib.msv_batch_factor.restype = ctypes.c_int
    lib.msv_batch_destroy.argtypes = [P]
    lib.msv_batch_destroy.restype = None
    lib.msv_batch_last_error.argtypes = [P]
    lib.msv_batch_last_error.restype = ctypes.c_char_p
    lib.msv_batch_panel.argtypes = [P]
    lib.msv_batch_panel.restype = ctypes.c_int32
    lib.msv_batch_tuned_ms.argtypes = [P, ctypes.c_int32]
    lib.msv_batch_tuned_ms.restype = ctypes.c_float
    lib.msv_batch_plane_min.argtypes = [P]
    lib.msv_batch_plane_min.restype = ctypes.c_int32
    lib.msv_batch_tuned_plane_ms.argtypes = [P, ctypes.c_int32]
    lib.msv_batch_tuned_plane_ms.restype = ctypes.c_float
    lib.msv_batch_tuned_from_table.argtypes = [P]
    lib.msv_batch_tuned_from_table.restype = ctypes.c_int32
    lib.msv_tabulate_rows.argtypes = [P, ctypes.c_int32, ctypes.c_int32, P, ctypes.c_size_t, P]
    lib.msv_tabulate_rows.restype = ctypes.c_int
    lib.msv_assemble_rows.argtypes = [P, P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, P, P]
    lib.msv_assemble_rows.restype = ctypes.c_int
    lib.msv_workspace_bytes.argtypes = [ctypes.c_int32] * 6
    lib.msv_workspace_bytes.restype = ctypes.c_size_t
    lib.msv_plan_device_bytes.argtypes = [P]
    lib.msv_plan_device_bytes.restype = ctypes.c_size_t
    lib.msv_set_allocator.argtypes = [P, P, P]
    lib.msv_set_allocator.restype = ctypes.c_int
    _lib = lib
    return lib


_ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int32, ctypes.c_void_p)
_FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p)
_hooks = None  # the registered callbacks, kept alive while the library may call them


def use_torch_allocator(enable=True):
    """Route the library's own device allocations through torch's caching
    allocator (msv_set_allocator), or back to hipMalloc / hipFree.  Every block
    is taken on the device's default stream, so that memory a destroyed plan
    gives back can serve any later plan or tensor allocated there.  Raises
    MsvError while plans or batches exist."""
    global _hooks
    lib = load_library()
    if not enable:
        st = lib.msv_set_allocator(None, None, None)
        if st:
            raise MsvError(st, lib.msv_last_error(None).decode())
        _hooks = None
        return
    import torch

    def alloc(nbytes, device, ctx):
        try:
            return torch.cuda.caching_allocator_alloc(int(nbytes), int(device),
                                                      torch.cuda.default_stream(int(device)))
        except RuntimeError:  # out of memory: the library reports MSV_ENOMEM
            return None

    def free(ptr, device, ctx):
        torch.cuda.caching_allocator_delete(ptr)
    hooks = (_ALLOC_FN(alloc), _FREE_FN(free))
    st = lib.msv_set_allocator(ctypes.cast(hooks[0], ctypes.c_void_p), ctypes.cast(hooks[1], ctypes.c_void_p), None)
    if st:
        raise MsvError(st, lib.msv_last_error(None).decode())
    _hooks = hooks


def _c(z):
    z = complex(z)
    return c128(z.real, z.imag)


def _stream_handle(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


class Plan:
    """A body, its discretization and physical parameters (msv_plan_create)."""

    def __init__(self, r, z, nr, nz, dsdu, n_panels, closed, self_u, self_w, adj_u, adj_w,
                 k0, eps1, mu1=1.0, eps0=1.0, mu0=1.0, m_max=16, fft_len=64, precision=0,
                 ir_tol=1e-13, ir_max_iter=10, formulation=0, stream=None, lib=None):
        self.lib = lib or load_library()
        f64 = lambda a: np.ascontiguousarray(np.asarray(a, dtype=np.float64))
        self._keep = [f64(a) for a in (r, z, nr, nz, dsdu, self_u, self_w, adj_u, adj_w)]
        a = self._keep
        ptr = lambda x: x.ctypes.data_as(ctypes.c_void_p)
        curve = Curve(int(n_panels), 16, int(bool(closed)), ptr(a[0]), ptr(a[1]), ptr(a[2]), ptr(a[3]), ptr(a[4]))
        ns = a[5].size // 16
        rules = Rules(int(ns), ptr(a[5]), ptr(a[6]), int(a[7].size), ptr(a[7]), ptr(a[8]))
        desc = Desc(float(k0), _c(eps0), _c(mu0), _c(eps1), _c(mu1), int(m_max), int(fft_len),
                    int(precision), float(ir_tol), int(ir_max_iter), int(formulation))
        self._h = ctypes.c_void_p()
        st = self.lib.msv_plan_create(ctypes.byref(self._h), ctypes.byref(curve), ctypes.byref(rules),
                                      ctypes.byref(desc), None)
        if st != MSV_OK:
            raise MsvError(st, self.lib.msv_last_error(None).decode())
        self.M = int(m_max)
        self.N = self.lib.msv_num_nodes(self._h)
        self.S = self.lib.msv_num_support(self._h)
        self.n = self.lib.msv_matrix_order(self._h)
        self.precision = int(precision)
        self.formulation = int(formulation)
        self._factored = None

    def _sh(self, stream):
        """The call's stream handle; the stream is remembered for close()."""
        import torch
        self._last_stream = stream if stream is not None else torch.cuda.current_stream()
        return ctypes.c_void_p(self._last_stream.cuda_stream)

    def close(self, wait=True):
        """Destroy the plan.  With a caller pool the library does not wait at
        destroy: the plan's last call must have finished, which close() makes
        sure of by synchronizing that call's stream unless the caller knows
        it has (wait=False)."""
        if getattr(self, "_h", None) and self._h.value:
            last = getattr(self, "_last_stream", None)
            if wait and _hooks is not None and last is not None:
                last.synchronize()
            self.lib.msv_plan_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, st):
        if st != MSV_OK:
            raise MsvError(st, self.lib.msv_last_error(self._h).decode())

    @property
    def table_entries(self) -> int:
        return int(self.lib.msv_table_entries(self._h))

    @property
    def table_shape(self):
        return (self.M + 2, 9, self.N, self.N + self.S)

    @property
    def device_bytes(self) -> int:
        return int(self.lib.msv_plan_device_bytes(self._h))

    def last_ir_iterations(self) -> int:
        return int(self.lib.msv_last_ir_iterations(self._h))

    def tabulate(self, out=None, stream=None):
        import torch
        if out is None:
            out = torch.empty(self.table_shape, dtype=torch.complex128, device="cuda")
        assert out.dtype == torch.complex128 and out.is_cuda and out.is_contiguous()
        self._check(self.lib.msv_tabulate(self._h, ctypes.c_void_p(out.data_ptr()), out.numel(),
                                          self._sh(stream)))
        return out

    def table_rows_shape(self, nt):
        return (self.M + 2, 9, int(nt), self.N + self.S)

    def tabulate_rows(self, t0, nt, out=None, stream=None):
        import torch
        if out is None:
            out = torch.empty(self.table_rows_shape(nt), dtype=torch.complex128, device="cuda")
        assert out.dtype == torch.complex128 and out.is_cuda and out.is_contiguous()
        self._check(self.lib.msv_tabulate_rows(self._h, int(t0), int(nt), ctypes.c_void_p(out.data_ptr()),
                                               out.numel(), self._sh(stream)))
        return out

    def assemble_rows(self, kern, t0, nt, m_lo, m_hi, out, stream=None):
        import torch
        nm = m_hi - m_lo + 1
        assert out.dtype == torch.complex128 and out.is_contiguous() and out.shape == (nm, self.n, self.n)
        assert kern.is_contiguous() and tuple(kern.shape) == self.table_rows_shape(nt)
        self._check(self.lib.msv_assemble_rows(self._h, ctypes.c_void_p(kern.data_ptr()), int(t0), int(nt),
                                               int(m_lo), int(m_hi), ctypes.c_void_p(out.data_ptr()),
                                               self._sh(stream)))
        return out

    def assemble_streamed(self, m_lo, m_hi, out=None, rows_per_block=None, block=None, stream=None):
        """Tabulate and assemble in target-row blocks through one reused table
        block, so the whole table is never resident.  Blocks of 128 rows by
        default: the tabulation's stores into a block's [mode][type][row]
        [source] table merge better than into larger blocks."""
        import torch
        nm = m_hi - m_lo + 1
        if out is None:
            out = torch.empty((nm, self.n, self.n), dtype=torch.complex128, device="cuda")
        nb = min(int(rows_per_block or 128), self.N)
        if block is None:
            block = torch.empty(self.table_rows_shape(nb), dtype=torch.complex128, device="cuda")
        for t0 in range(0, self.N, nb):
            nt = min(nb, self.N - t0)
            kb = block.view(-1)[: (self.M + 2) * 9 * nt * (self.N + self.S)].view(self.table_rows_shape(nt))
            self.tabulate_rows(t0, nt, out=kb, stream=stream)
            self.assemble_rows(kb, t0, nt, m_lo, m_hi, out, stream=stream)
        return out

    def assemble(self, kern, m_lo, m_hi, out=None, stream=None):
        import torch
        nm = m_hi - m_lo + 1
        if out is None:
            out = torch.empty((nm, self.n, self.n), dtype=torch.complex128, device="cuda")
        assert out.dtype == torch.complex128 and out.is_contiguous() and out.shape == (nm, self.n, self.n)
        assert kern.is_contiguous() and tuple(kern.shape) == self.table_shape
        self._check(self.lib.msv_assemble(self._h, ctypes.c_void_p(kern.data_ptr()), int(m_lo), int(m_hi),
                                          ctypes.c_void_p(out.data_ptr()), self._sh(stream)))
        return out

    def factor(self, A, m_lo, m_hi, stream=None):
        assert A.is_contiguous() and A.shape == (m_hi - m_lo + 1, self.n, self.n)
        self._check(self.lib.msv_factor(self._h, ctypes.c_void_p(A.data_ptr()), int(m_lo), int(m_hi),
                                        self._sh(stream)))
        self._factored = A  # the library keeps using this buffer
        return A

    def solve(self, m_lo, m_hi, rhs, out=None, stream=None):
        import torch
        nm = m_hi - m_lo + 1
        assert rhs.dtype == torch.complex128 and rhs.is_contiguous() and rhs.shape[0] == nm
        assert rhs.shape[2] == self.n
        if out is None:
            out = torch.empty_like(rhs)
        self._check(self.lib.msv_solve(self._h, int(m_lo), int(m_hi), int(rhs.shape[1]),
                                       ctypes.c_void_p(rhs.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                                       self._sh(stream)))
        return out


    def solve_noalloc(self, m_lo, m_hi, rhs, out, stream=None):
        """msv_solve with the library's static workspace (no device allocation;
        `out` must be preallocated)."""
        import torch
        nm = m_hi - m_lo + 1
        assert rhs.dtype == torch.complex128 and rhs.is_contiguous() and rhs.shape[0] == nm
        assert rhs.shape[2] == self.n and out.shape == rhs.shape and out.is_contiguous()
        self._check(self.lib.msv_solve_noalloc(self._h, int(m_lo), int(m_hi), int(rhs.shape[1]),
                                               ctypes.c_void_p(rhs.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                                               self._sh(stream)))
        return out


    def far_field(self, m_lo, m_hi, x, dirs, stream=None):
        """msv_far_field: E_inf [n_vec, n_dirs, 3] of the currents x
        [m_hi - m_lo + 1, n_vec, 4N] at unit directions dirs [n_dirs, 3]."""
        import torch
        nm = m_hi - m_lo + 1
        assert x.dtype == torch.complex128 and x.is_contiguous() and x.shape[0] == nm and x.shape[2] == self.n
        dirs = torch.as_tensor(dirs, dtype=torch.float64, device=x.device).contiguous()
        assert dirs.ndim == 2 and dirs.shape[1] == 3
        out = torch.empty((x.shape[1], dirs.shape[0], 3), dtype=torch.complex128, device=x.device)
        self._check(self.lib.msv_far_field(self._h, int(m_lo), int(m_hi), int(x.shape[1]),
                                           ctypes.c_void_p(x.data_ptr()), int(dirs.shape[0]),
                                           ctypes.c_void_p(dirs.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                                           self._sh(stream)))
        return out

    def fields(self, m_lo, m_hi, x, points, region, upsample=1, stream=None):
        """msv_fields: E, H [n_vec, n_points, 3] at points [n_points, 3] of
        `region` ("exterior" or "interior"), the currents interpolated to
        `upsample` sub-panels per panel."""
        import torch
        nm = m_hi - m_lo + 1
        assert x.dtype == torch.complex128 and x.is_contiguous() and x.shape[0] == nm and x.shape[2] == self.n
        pts = torch.as_tensor(points, dtype=torch.float64, device=x.device).contiguous()
        assert pts.ndim == 2 and pts.shape[1] == 3
        reg = {"exterior": 0, "interior": 1}[region]
        E = torch.empty((x.shape[1], pts.shape[0], 3), dtype=torch.complex128, device=x.device)
        H = torch.empty_like(E)
        self._check(self.lib.msv_fields(self._h, int(m_lo), int(m_hi), int(x.shape[1]),
                                        ctypes.c_void_p(x.data_ptr()), int(pts.shape[0]),
                                        ctypes.c_void_p(pts.data_ptr()), reg, int(upsample),
                                        ctypes.c_void_p(E.data_ptr()),
                                        ctypes.c_void_p(H.data_ptr()), self._sh(stream)))
        return E, H


class Batch:
    """Per-mode systems of several plans factored by one captured launch
    sequence (msv_batch_create / msv_batch_factor)."""

    def __init__(self, plans, mats, m_lo, m_hi, stream=None):
        self.lib = plans[0].lib
        for p, A in zip(plans, mats):
            assert A.is_contiguous() and tuple(A.shape) == (m_hi - m_lo + 1, p.n, p.n)
        self._plans = list(plans)
        self._mats = list(mats)  # the library keeps using these buffers
        P = ctypes.c_void_p
        ph = (P * len(plans))(*[p._h.value for p in plans])
        ah = (P * len(mats))(*[A.data_ptr() for A in mats])
        self._h = P()
        st = self.lib.msv_batch_create(ctypes.byref(self._h), ph, ah, len(plans), int(m_lo), int(m_hi),
                                       _stream_handle(stream))
        if st != MSV_OK:
            raise MsvError(st, self.lib.msv_batch_last_error(None).decode())

    @property
    def panel(self) -> int:
        return int(self.lib.msv_batch_panel(self._h))

    def tuned_ms(self, panel: int) -> float:
        return float(self.lib.msv_batch_tuned_ms(self._h, int(panel)))

    @property
    def plane_min(self) -> int:
        return int(self.lib.msv_batch_plane_min(self._h))

    def tuned_plane_ms(self, plane_min: int) -> float:
        return float(self.lib.msv_batch_tuned_plane_ms(self._h, int(plane_min)))

    @property
    def from_table(self) -> bool:
        return bool(self.lib.msv_batch_tuned_from_table(self._h))

    def factor(self, stream=None):
        st = self.lib.msv_batch_factor(self._h, _stream_handle(stream))
        if st != MSV_OK:
            raise MsvError(st, self.lib.msv_batch_last_error(self._h).decode())

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            self.lib.msv_batch_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def workspace_bytes(n_nodes, n_support, fft_len, n_modes, n_solve_vectors, precision, lib=None):
    """Upper bound on a plan's own device memory (msv_workspace_bytes)."""
    lib = lib or load_library()
    return int(lib.msv_workspace_bytes(int(n_nodes), int(n_support), int(fft_len), int(n_modes),
                                       int(n_solve_vectors), int(precision)))


def plan_from_curve(curve, rules, k0, eps1, mu1=1.0, m_max=16, fft_len=64, precision=0, **kw):
    """Convenience: a Plan from a workloads.geometry.Curve and loaded rules."""
    (ys, ws), (ya, wa) = rules
    return Plan(curve.r, curve.z, curve.nr, curve.nz, curve.dsdu, curve.n_panels, curve.closed,
                ys.ravel(), ws.ravel(), ya, wa, k0, eps1, mu1, m_max=m_max, fft_len=fft_len,
                precision=precision, **kw)
