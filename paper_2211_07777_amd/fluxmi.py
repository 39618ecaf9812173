"""ctypes binding of libfluxmi.so (include/fluxmi.h).

Argument marshalling only: every step of a solve runs in the HIP library.  Device
memory and streams come from PyTorch (``tensor.data_ptr()``,
``torch.cuda.current_stream().cuda_stream``).  If the library is missing this module
raises; there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfluxmi.so")

EVEN, ODD, PER, UNB = 0, 1, 2, 3
CELL, NODE = 0, 1
CHAT2, CHAT2_VOL = 0, 1
HEJ2, HEJ4, HEJ6, HEJ8, HEJ10, HEJ0 = 2, 3, 4, 5, 6, 7  # regularised kernels (Sec. IV)
LGF2 = 8  # lattice Green's function of the second-difference Laplacian (Sec. IV)
F64, F32 = 0, 1
POISSON, BIOT_SAVART, BIOT_SAVART_FD2, BIOT_SAVART_FD4, BIOT_SAVART_FD6 = 0, 1, 2, 3, 4
CLASS_NAMES = ["P", "EE", "OO", "EO", "OE", "UU", "EU", "OU", "UE", "UO"]
EXPORTED = [
    "fm_plan_create", "fm_plan_destroy", "fm_plan_workspace_bytes", "fm_plan_shape",
    "fm_solve", "fm_solve_passes", "fm_solve_batched", "fm_batched_workspace_bytes", "fm_plan_inspect",
    "fm_error_string", "fm_last_hip_error", "fm_batch_prepare", "fm_batch_run", "fm_batch_destroy",
    "fm_plan_tune", "fm_plan_tiling", "fm_plan_device_bytes",
    "fm_server_create", "fm_server_submit", "fm_server_progress", "fm_server_wait_all",
    "fm_server_get_stats", "fm_server_destroy", "fm_solve_static", "fm_plan_set_tiling",
    "fm_plan_spectrum_layout", "fm_fft_forward", "fm_fft_backward", "fm_plan_tuned_from_cache",
    "fm_plan_create_vector",
]
STATIC_WORKSPACE_BYTES = 128 << 20  # FM_STATIC_WORKSPACE_BYTES


class ServerStats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_longlong), ("finished", ctypes.c_longlong),
                ("plan_hits", ctypes.c_longlong), ("plan_misses", ctypes.c_longlong),
                ("plan_evictions", ctypes.c_longlong), ("peak_workspace_bytes", ctypes.c_size_t),
                ("peak_inflight", ctypes.c_int), ("cached_plans", ctypes.c_int), ("waiting", ctypes.c_int),
                ("running", ctypes.c_int), ("plan_bytes", ctypes.c_size_t), ("failed", ctypes.c_longlong)]


class FluxmiError(RuntimeError):
    def __init__(self, status, what=""):
        lib = library()
        msg = lib.fm_error_string(status).decode()
        if status == -6:
            msg += f" (hip error {lib.fm_last_hip_error()})"
        super().__init__(f"{what}: {msg} [{status}]" if what else f"{msg} [{status}]")
        self.status = status


class _Info(ctypes.Structure):
    _fields_ = [
        ("order", ctypes.c_int * 3), ("axis_class", ctypes.c_int * 3), ("fft_len", ctypes.c_int * 3),
        ("spec_len", ctypes.c_int * 3), ("green_dims", ctypes.c_int * 3),
        ("workspace_bytes", ctypes.c_size_t), ("tiles", ctypes.c_int * 5),
        ("lines_per_tile", ctypes.c_int * 5), ("lds_bytes", ctypes.c_int * 5),
        ("algo_bytes", ctypes.c_double * 5),
    ]


_lib = None


def library():
    """Load libfluxmi.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built: run __graft_entry__.build() first")
    # torch ships its own HIP runtime under the same soname; load it first so that the
    # library binds to the runtime that owns torch's device memory and streams (two
    # runtimes in one process do not share devices, pointers or streams)
    import torch  # noqa: F401
    L = ctypes.CDLL(LIB_PATH)
    vp, ip, dp = ctypes.c_void_p, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_double)
    L.fm_plan_create.argtypes = [ctypes.POINTER(vp), ip, dp, ip, ctypes.c_int, ctypes.c_int,
                                 ctypes.c_int, ctypes.c_int, ctypes.c_int, vp]
    L.fm_plan_create_vector.argtypes = [ctypes.POINTER(vp), ip, dp, ip, ctypes.c_int, ctypes.c_int,
                                        ctypes.c_int, ctypes.c_int, vp]
    L.fm_plan_destroy.argtypes = [vp]
    L.fm_plan_workspace_bytes.argtypes = [vp, ctypes.POINTER(ctypes.c_size_t)]
    L.fm_plan_shape.argtypes = [vp, ip]
    L.fm_solve.argtypes = [vp, vp, vp, vp, vp]
    L.fm_solve_passes.argtypes = [vp, vp, vp, vp, ctypes.c_int, ctypes.c_int, vp]
    L.fm_solve_static.argtypes = [vp, vp, vp, vp]
    L.fm_plan_spectrum_layout.argtypes = [vp, ip, ip, ip, ctypes.POINTER(ctypes.c_size_t)]
    L.fm_fft_forward.argtypes = [vp, vp, vp, vp, vp]
    L.fm_fft_backward.argtypes = [vp, vp, vp, vp, vp]
    L.fm_solve_batched.argtypes = [ctypes.c_int, ctypes.POINTER(vp), ctypes.POINTER(vp),
                                   ctypes.POINTER(vp), vp, ctypes.c_size_t, vp]
    L.fm_batched_workspace_bytes.argtypes = [ctypes.c_int, ctypes.POINTER(vp), ctypes.POINTER(ctypes.c_size_t)]
    L.fm_plan_inspect.argtypes = [ip, dp, ip, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                  ctypes.c_int, ctypes.POINTER(_Info)]
    L.fm_batch_prepare.argtypes = [ctypes.POINTER(vp), ctypes.c_int, ctypes.POINTER(vp), ctypes.POINTER(vp),
                                   ctypes.POINTER(vp), vp, ctypes.c_size_t, vp]
    L.fm_batch_run.argtypes = [vp, vp]
    L.fm_plan_tune.argtypes = [vp, vp, vp]
    L.fm_plan_tiling.argtypes = [vp, ip, ip, ip]
    L.fm_plan_set_tiling.argtypes = [vp, ip, ip, vp]
    L.fm_plan_tuned_from_cache.argtypes = [vp, ip]
    L.fm_plan_device_bytes.argtypes = [vp, ctypes.POINTER(ctypes.c_size_t)]
    L.fm_server_create.argtypes = [ctypes.POINTER(vp), ctypes.c_size_t, ctypes.c_size_t, ctypes.c_int,
                                   ctypes.c_int]
    L.fm_server_submit.argtypes = [vp, ip, dp, ip, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                   ctypes.c_int, vp, vp, vp, ctypes.POINTER(ctypes.c_longlong)]
    L.fm_server_progress.argtypes = [vp, ctypes.POINTER(ctypes.c_longlong), ip, ctypes.c_int,
                                     ctypes.POINTER(ctypes.c_int)]
    L.fm_server_wait_all.argtypes = [vp]
    L.fm_server_get_stats.argtypes = [vp, ctypes.POINTER(ServerStats)]
    L.fm_server_destroy.argtypes = [vp]
    L.fm_batch_destroy.argtypes = [vp]
    L.fm_error_string.argtypes = [ctypes.c_int]
    L.fm_error_string.restype = ctypes.c_char_p
    L.fm_last_hip_error.restype = ctypes.c_int
    _lib = L
    return L


def error_string(status):
    return library().fm_error_string(status).decode()


def _check(status, what):
    if status != 0:
        raise FluxmiError(status, what)


def _args(n, h, bc):
    n3 = (ctypes.c_int * 3)(*[int(v) for v in n])
    h3 = (ctypes.c_double * 3)(*[float(v) for v in h])
    flat = [int(v) for pair in bc for v in pair]
    if len(flat) != 6:
        raise ValueError("bc must be [[xl, xr], [yl, yr], [zl, zr]]")
    b6 = (ctypes.c_int * 6)(*flat)
    return n3, h3, b6


def _stream_ptr(stream):
    if stream is None:
        import torch
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return ctypes.c_void_p(stream)
    return ctypes.c_void_p(stream.cuda_stream)


def plan_inspect(n, h, bc, layout, green=CHAT2, prec=F64, kind=POISSON, ncomp=1):
    """Host-only planning information (no device needed)."""
    n3, h3, b6 = _args(n, h, bc)
    info = _Info()
    _check(library().fm_plan_inspect(n3, h3, b6, layout, green, prec, kind, ncomp, ctypes.byref(info)),
           "fm_plan_inspect")
    return {
        "order": list(info.order), "axis_class": [CLASS_NAMES[c] for c in info.axis_class],
        "fft_len": list(info.fft_len), "spec_len": list(info.spec_len),
        "green_dims": list(info.green_dims), "workspace_bytes": int(info.workspace_bytes),
        "tiles": list(info.tiles), "lines_per_tile": list(info.lines_per_tile),
        "lds_bytes": list(info.lds_bytes), "algo_bytes": list(info.algo_bytes),
    }


class Plan:
    """A solver plan (owns the cached Green's spectrum and twiddles on the device)."""

    def __init__(self, n, h, bc, layout, green=CHAT2, prec=F64, kind=POISSON, ncomp=None, stream=None):
        """bc: [[xl, xr], [yl, yr], [zl, zr]], or for Biot-Savart with conditions per component
        (fm_plan_create_vector) [3][3][2]: per component (x, y, z) such a list."""
        if ncomp is None:
            ncomp = 3 if kind != POISSON else 1
        vector = len(bc) == 3 and all(len(c) == 3 for c in bc)
        self.n, self.h = tuple(int(v) for v in n), tuple(float(v) for v in h)
        self.bc = [[list(f) for f in c] for c in bc] if vector else [list(p) for p in bc]
        self.layout, self.green, self.prec, self.kind, self.ncomp = layout, green, prec, kind, ncomp
        handle = ctypes.c_void_p()
        if vector:
            if ncomp != 3:
                raise ValueError("conditions per component need ncomp = 3")
            n3, h3, _ = _args(n, h, bc[0])
            b18 = (ctypes.c_int * 18)(*[int(v) for c in bc for f in c for v in f])
            _check(library().fm_plan_create_vector(ctypes.byref(handle), n3, h3, b18, layout, green, prec,
                                                   kind, _stream_ptr(stream)), "fm_plan_create_vector")
        else:
            n3, h3, b6 = _args(n, h, bc)
            _check(library().fm_plan_create(ctypes.byref(handle), n3, h3, b6, layout, green, prec, kind, ncomp,
                                            _stream_ptr(stream)), "fm_plan_create")
        self._h = handle
        dims = (ctypes.c_int * 3)()
        _check(library().fm_plan_shape(self._h, dims), "fm_plan_shape")
        self.user_dims = tuple(dims)  # (nx, ny, nz)
        ws = ctypes.c_size_t()
        _check(library().fm_plan_workspace_bytes(self._h, ctypes.byref(ws)), "fm_plan_workspace_bytes")
        self.workspace_bytes = int(ws.value)

    @property
    def shape(self):
        """torch shape of one solve's rhs / out: (ncomp, nz, ny, nx) or (nz, ny, nx)."""
        nx, ny, nz = self.user_dims
        return (self.ncomp, nz, ny, nx) if self.ncomp > 1 else (nz, ny, nx)

    @property
    def dtype(self):
        import torch
        return torch.float64 if self.prec == F64 else torch.float32

    def _check_tensor(self, t, name):
        if not t.is_cuda or t.dtype != self.dtype or not t.is_contiguous():
            raise ValueError(f"{name}: need a contiguous {self.dtype} GPU tensor")
        if t.numel() != self.ncomp * self.user_dims[0] * self.user_dims[1] * self.user_dims[2]:
            raise ValueError(f"{name}: expected {self.shape}, got {tuple(t.shape)}")

    def solve(self, rhs, out=None, workspace=None, stream=None):
        import torch
        self._check_tensor(rhs, "rhs")
        if out is None:
            out = torch.empty_like(rhs)
        self._check_tensor(out, "out")
        ws = ctypes.c_void_p(0)
        if workspace is not None:
            if workspace.numel() * workspace.element_size() < self.workspace_bytes or not workspace.is_cuda:
                raise ValueError("workspace too small")
            ws = ctypes.c_void_p(workspace.data_ptr())
        _check(library().fm_solve(self._h, ctypes.c_void_p(rhs.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                                  ws, _stream_ptr(stream)), "fm_solve")
        return out

    def spectrum_layout(self):
        """(dims slow -> fast, physical axis of each, complex?, bytes) of the spectrum of
        fft_forward (fm_plan_spectrum_layout)."""
        d, a, c, b = (ctypes.c_int * 3)(), (ctypes.c_int * 3)(), ctypes.c_int(), ctypes.c_size_t()
        _check(library().fm_plan_spectrum_layout(self._h, d, a, ctypes.byref(c), ctypes.byref(b)),
               "fm_plan_spectrum_layout")
        return list(d), list(a), bool(c.value), int(b.value)

    def spectrum_empty(self):
        """A torch tensor shaped for the spectrum: (ncomp,) + dims (+ complex dtype)."""
        import torch
        dims, _, cplx, _ = self.spectrum_layout()
        shape = ((self.ncomp,) if self.ncomp > 1 else ()) + tuple(dims)
        if cplx:
            dt = torch.complex128 if self.prec == F64 else torch.complex64
        else:
            dt = self.dtype
        return torch.empty(shape, dtype=dt, device="cuda")

    def _check_spec(self, spec):
        _, _, _, nbytes = self.spectrum_layout()
        if not spec.is_cuda or not spec.is_contiguous() or spec.numel() * spec.element_size() != nbytes:
            raise ValueError("spec: need a contiguous GPU tensor of fm_plan_spectrum_layout's size")

    def fft_forward(self, x, spec=None, workspace=None, stream=None):
        """Forward transforms of every axis, no spectral multiplication (fm_fft_forward)."""
        self._check_tensor(x, "in")
        spec = self.spectrum_empty() if spec is None else spec
        self._check_spec(spec)
        ws = ctypes.c_void_p(0 if workspace is None else workspace.data_ptr())
        _check(library().fm_fft_forward(self._h, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(spec.data_ptr()),
                                        ws, _stream_ptr(stream)), "fm_fft_forward")
        return spec

    def fft_backward(self, spec, out=None, workspace=None, stream=None):
        """Backward transforms with the crop and output conventions (fm_fft_backward)."""
        import torch
        self._check_spec(spec)
        out = torch.empty(self.shape, dtype=self.dtype, device="cuda") if out is None else out
        self._check_tensor(out, "out")
        ws = ctypes.c_void_p(0 if workspace is None else workspace.data_ptr())
        _check(library().fm_fft_backward(self._h, ctypes.c_void_p(spec.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                                         ws, _stream_ptr(stream)), "fm_fft_backward")
        return out

    def solve_static(self, rhs, out, stream=None):
        """fm_solve_static: a solve whose workspace is the library's fixed device array
        (no allocation in the call; calls on one GPU must not overlap)."""
        self._check_tensor(rhs, "rhs")
        self._check_tensor(out, "out")
        _check(library().fm_solve_static(self._h, ctypes.c_void_p(rhs.data_ptr()),
                                         ctypes.c_void_p(out.data_ptr()), _stream_ptr(stream)),
               "fm_solve_static")
        return out

    def solve_passes(self, rhs, out, first, last, workspace=None, stream=None):
        """Run passes first..last (0..4) of a solve; see fm_solve_passes."""
        self._check_tensor(rhs, "rhs")
        self._check_tensor(out, "out")
        ws = ctypes.c_void_p(0 if workspace is None else workspace.data_ptr())
        if workspace is not None and workspace.numel() * workspace.element_size() < self.workspace_bytes:
            raise ValueError("workspace too small")
        _check(library().fm_solve_passes(self._h, ctypes.c_void_p(rhs.data_ptr()),
                                         ctypes.c_void_p(out.data_ptr()), ws, int(first), int(last),
                                         _stream_ptr(stream)), "fm_solve_passes")
        return out

    def tune(self, workspace=None, stream=None):
        """Autotune the tiling of every pass on the device (fm_plan_tune)."""
        ws = ctypes.c_void_p(0 if workspace is None else workspace.data_ptr())
        _check(library().fm_plan_tune(self._h, ws, _stream_ptr(stream)), "fm_plan_tune")
        return self.tiling()

    def tuned_from_cache(self):
        """True when the last tune() applied an entry of the FLUXMI_TUNE_CACHE file."""
        v = ctypes.c_int()
        _check(library().fm_plan_tuned_from_cache(self._h, ctypes.byref(v)), "fm_plan_tuned_from_cache")
        return bool(v.value)

    def tiling(self):
        """(lines per tile, tiles, launch mode) of the five passes; mode 1 = persistent
        grid, 0 = one tile per workgroup with LDS tables, 2 = with global tables, 3 / 4 / 5 =
        the per-wavefront kernels with 16 / 8 / 32 values per lane (5: FP32 Poisson fused
        pass only)."""
        b, t, q = (ctypes.c_int * 5)(), (ctypes.c_int * 5)(), (ctypes.c_int * 5)()
        _check(library().fm_plan_tiling(self._h, b, t, q), "fm_plan_tiling")
        return {"lines_per_tile": list(b), "tiles": list(t), "persistent": list(q)}

    def set_tiling(self, lines_per_tile, persistent, stream=None):
        """Apply a tiling as tiling() reports it (fm_plan_set_tiling)."""
        b = (ctypes.c_int * 5)(*[int(v) for v in lines_per_tile])
        q = (ctypes.c_int * 5)(*[int(v) for v in persistent])
        _check(library().fm_plan_set_tiling(self._h, b, q, _stream_ptr(stream)), "fm_plan_set_tiling")
        return self.tiling()

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            library().fm_plan_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        # at interpreter shutdown the HIP runtime may already be gone: leave the
        # memory to the process teardown
        if sys.is_finalizing():
            return
        try:
            self.close()
        except Exception:
            pass


def batched_workspace_bytes(plans):
    arr = (ctypes.c_void_p * len(plans))(*[p._h.value for p in plans])
    out = ctypes.c_size_t()
    _check(library().fm_batched_workspace_bytes(len(plans), arr, ctypes.byref(out)), "fm_batched_workspace_bytes")
    return int(out.value)


def solve_batched(plans, rhs, outs, workspace, stream=None):
    """One launch per pass for the whole batch (plans may differ; same precision)."""
    n = len(plans)
    if not (len(rhs) == len(outs) == n):
        raise ValueError("plans, rhs and outs must have the same length")
    for p, r, o in zip(plans, rhs, outs):
        p._check_tensor(r, "rhs")
        p._check_tensor(o, "out")
    P = (ctypes.c_void_p * n)(*[p._h.value for p in plans])
    R = (ctypes.c_void_p * n)(*[r.data_ptr() for r in rhs])
    O = (ctypes.c_void_p * n)(*[o.data_ptr() for o in outs])
    nbytes = workspace.numel() * workspace.element_size()
    _check(library().fm_solve_batched(n, P, R, O, ctypes.c_void_p(workspace.data_ptr()), nbytes,
                                      _stream_ptr(stream)), "fm_solve_batched")
    return outs


class Batch:
    """A batch bound to fixed tensors (fm_batch_prepare); run() only enqueues kernels,
    so it can be captured in a HIP graph (torch.cuda.graph) and replayed."""

    def __init__(self, plans, rhs, outs, workspace, stream=None):
        n = len(plans)
        if not (len(rhs) == len(outs) == n) or n == 0:
            raise ValueError("plans, rhs and outs must have the same, nonzero length")
        for p, r, o in zip(plans, rhs, outs):
            p._check_tensor(r, "rhs")
            p._check_tensor(o, "out")
        # keep the plans and buffers alive as long as the batch
        self._keep = (list(plans), list(rhs), list(outs), workspace)
        P = (ctypes.c_void_p * n)(*[p._h.value for p in plans])
        R = (ctypes.c_void_p * n)(*[r.data_ptr() for r in rhs])
        O = (ctypes.c_void_p * n)(*[o.data_ptr() for o in outs])
        handle = ctypes.c_void_p()
        nbytes = workspace.numel() * workspace.element_size()
        _check(library().fm_batch_prepare(ctypes.byref(handle), n, P, R, O, ctypes.c_void_p(workspace.data_ptr()),
                                          nbytes, _stream_ptr(stream)), "fm_batch_prepare")
        self._h = handle

    def run(self, stream=None):
        _check(library().fm_batch_run(self._h, _stream_ptr(stream)), "fm_batch_run")

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            library().fm_batch_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        if sys.is_finalizing():
            return
        try:
            self.close()
        except Exception:
            pass


class Server:
    """Serving loop (fm_server_*): requests are admitted as device streams and workspace
    (within the HBM budget) free up; plans are cached on the device.  One host thread."""

    def __init__(self, workspace_budget_bytes, plan_budget_bytes, slots=8, tune_plans=False):
        handle = ctypes.c_void_p()
        _check(library().fm_server_create(ctypes.byref(handle), int(workspace_budget_bytes),
                                          int(plan_budget_bytes), int(slots), int(bool(tune_plans))),
               "fm_server_create")
        self._h = handle
        self._keep = {}  # ticket -> (rhs, out): alive until finished
        self.failed = {}  # ticket -> status of requests that finished with an error

    def submit(self, n, h, bc, layout, rhs, out, prec=F32, green=CHAT2, kind=POISSON, ncomp=1, stream=None):
        """Enqueue one solve; returns its ticket.  The solve runs after the work enqueued
        so far on `stream` (default: torch's current stream), which produced rhs."""
        import torch
        dt = torch.float64 if prec == F64 else torch.float32
        for t, name in ((rhs, "rhs"), (out, "out")):
            if not t.is_cuda or t.dtype != dt or not t.is_contiguous():
                raise ValueError(f"{name}: need a contiguous {dt} GPU tensor")
        n3, h3, b6 = _args(n, h, bc)
        ticket = ctypes.c_longlong()
        _check(library().fm_server_submit(self._h, n3, h3, b6, layout, green, prec, kind, ncomp,
                                          ctypes.c_void_p(rhs.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                                          _stream_ptr(stream), ctypes.byref(ticket)), "fm_server_submit")
        self._keep[ticket.value] = (rhs, out)
        return ticket.value

    def progress(self, max_finished=4096):
        """Admit and retire; returns the tickets finished since the last call (those that
        finished with an error are also entered in self.failed with their status)."""
        buf = (ctypes.c_longlong * max_finished)()
        st = (ctypes.c_int * max_finished)()
        n = ctypes.c_int()
        _check(library().fm_server_progress(self._h, buf, st, max_finished, ctypes.byref(n)),
               "fm_server_progress")
        done = list(buf[:n.value])
        for t, status in zip(done, st[:n.value]):
            self._keep.pop(t, None)
            if status != 0:
                self.failed[t] = status
        return done

    def wait_all(self):
        _check(library().fm_server_wait_all(self._h), "fm_server_wait_all")

    def stats(self):
        st = ServerStats()
        _check(library().fm_server_get_stats(self._h, ctypes.byref(st)), "fm_server_get_stats")
        return {name: getattr(st, name) for name, _ in ServerStats._fields_}

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            library().fm_server_destroy(self._h)
            self._h = ctypes.c_void_p()
            self._keep.clear()

    def __del__(self):
        if sys.is_finalizing():
            return
        try:
            self.close()
        except Exception:
            pass
