"""Thin Python binding of libtfcb.so (the C-ABI of include/tfcb.h).

Argument marshalling only: torch tensors provide device memory and the
current stream; every step of the reconstruction runs in the library's HIP
kernels.  There is no fallback: if the library is missing or no GPU is
present, the calls raise.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtfcb.so")

F32, F16, BF16 = 0, 1, 2
OK, EINVAL, ENOMEM, EDEVICE, EUNSUPPORTED, ENUMERIC, EBUSY = 0, -1, -2, -3, -4, -5, -6

# every symbol the header declares
EXPORTS = [
    "tfcb_status_str", "tfcb_last_error", "tfcb_version",
    "tfcb_workspace_size", "tfcb_operator_workspace_size", "tfcb_framelet_workspace_size",
    "tfcb_project", "tfcb_backproject", "tfcb_backproject_noalloc", "tfcb_project_siddon",
    "tfcb_backproject_eq3",
    "tfcb_framelet_shrink", "tfcb_rof_workspace_size", "tfcb_rof", "tfcb_cgls",
    "tfcb_fdk_workspace_size", "tfcb_fdk",
    "tfcb_restrict_sino", "tfcb_prolong_vol", "tfcb_reconstruct",
    "tfcb_request_bytes", "tfcb_server_create", "tfcb_server_submit", "tfcb_server_step",
    "tfcb_server_poll", "tfcb_server_cancel", "tfcb_server_destroy",
]
REQ_QUEUED, REQ_RUNNING, REQ_DONE, REQ_FAILED, REQ_CANCELLED = 0, 1, 2, 3, 4


class TfcbError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__("tfcb status %d: %s" % (status, msg))
        self.status = status


class Geometry(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("dx", ctypes.c_double), ("dy", ctypes.c_double), ("dz", ctypes.c_double),
                ("nu", ctypes.c_int32), ("nv", ctypes.c_int32),
                ("du", ctypes.c_double), ("dv", ctypes.c_double),
                ("sad", ctypes.c_double), ("sdd", ctypes.c_double),
                ("n_views", ctypes.c_int32), ("angles", ctypes.POINTER(ctypes.c_double))]


class Options(ctypes.Structure):
    _fields_ = [("lambda_", ctypes.c_double), ("n_grids", ctypes.c_int32),
                ("iters", ctypes.c_int32 * 4), ("cgls_steps", ctypes.c_int32),
                ("framelet_levels", ctypes.c_int32), ("momentum", ctypes.c_int32),
                ("positivity", ctypes.c_int32), ("bin_coarse_detector", ctypes.c_int32),
                ("storage", ctypes.c_int32), ("profile", ctypes.c_int32),
                ("op_pair", ctypes.c_int32), ("regulariser", ctypes.c_int32),
                ("tv_eps", ctypes.c_double), ("tv_tol", ctypes.c_double),
                ("tv_max_steps", ctypes.c_int32)]


class Report(ctypes.Structure):
    _fields_ = [("seconds_total", ctypes.c_double), ("seconds_per_grid", ctypes.c_double * 4),
                ("iters_done", ctypes.c_int32 * 4), ("resid2_last", ctypes.c_double),
                ("cgls_breakdowns", ctypes.c_int32), ("kernel_ms", ctypes.c_double * 4),
                ("kernel_launches", ctypes.c_int32 * 4), ("rof_steps", ctypes.c_int32)]


_lib = None


def load(path: str = LIB_PATH):
    """Load libtfcb.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError("libtfcb.so not found at %s: build it with "
                          "`python paper_1008_2042_amd/csrc/build.py`" % path)
    lib = ctypes.CDLL(path)
    G = ctypes.POINTER(Geometry)
    O = ctypes.POINTER(Options)
    vp, sz, i32, dbl = ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int32, ctypes.c_double
    psz = ctypes.POINTER(ctypes.c_size_t)
    sig = {
        "tfcb_status_str": ([i32], ctypes.c_char_p),
        "tfcb_last_error": ([], ctypes.c_char_p),
        "tfcb_version": ([], ctypes.c_char_p),
        "tfcb_workspace_size": ([G, O, psz], i32),
        "tfcb_operator_workspace_size": ([G, i32, psz], i32),
        "tfcb_framelet_workspace_size": ([i32, i32, i32, i32, i32, psz], i32),
        "tfcb_project": ([G, i32, vp, vp, vp, sz, vp], i32),
        "tfcb_backproject": ([G, i32, vp, vp, vp, sz, vp], i32),
        "tfcb_backproject_noalloc": ([G, i32, vp, vp, vp], i32),
        "tfcb_project_siddon": ([G, i32, vp, vp, vp, sz, vp], i32),
        "tfcb_backproject_eq3": ([G, i32, vp, vp, vp, sz, vp], i32),
        "tfcb_framelet_shrink": ([i32, i32, i32, i32, dbl, i32, i32, vp, vp, vp, sz, vp], i32),
        "tfcb_fdk_workspace_size": ([G, psz], i32),
        "tfcb_fdk": ([G, i32, vp, vp, vp, sz, vp], i32),
        "tfcb_rof_workspace_size": ([i32, i32, i32, psz], i32),
        "tfcb_rof": ([i32, i32, i32, dbl, dbl, dbl, i32, i32, i32, vp, vp, vp, sz, vp,
                      ctypes.POINTER(i32)], i32),
        "tfcb_cgls": ([G, O, vp, vp, vp, sz, vp, ctypes.POINTER(dbl)], i32),
        "tfcb_restrict_sino": ([G, i32, vp, vp, vp], i32),
        "tfcb_prolong_vol": ([G, G, i32, vp, vp, vp], i32),
        "tfcb_reconstruct": ([G, O, vp, vp, vp, sz, vp, ctypes.POINTER(Report)], i32),
        "tfcb_request_bytes": ([G, O, psz], i32),
        "tfcb_server_create": ([vp, sz, i32, ctypes.POINTER(vp)], i32),
        "tfcb_server_submit": ([vp, G, O, vp, vp, vp, ctypes.POINTER(ctypes.c_uint64)], i32),
        "tfcb_server_step": ([vp, ctypes.POINTER(i32), ctypes.POINTER(i32)], i32),
        "tfcb_server_poll": ([vp, ctypes.c_uint64, ctypes.POINTER(i32), ctypes.POINTER(dbl),
                              ctypes.POINTER(i32)], i32),
        "tfcb_server_cancel": ([vp, ctypes.c_uint64], i32),
        "tfcb_server_destroy": ([vp], i32),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    _lib = lib
    return lib


def _check(status: int):
    if status != OK:
        lib = load()
        raise TfcbError(status, lib.tfcb_last_error().decode())


def geometry(g) -> Geometry:
    """Marshal any object with the geometry fields; keeps the angle array alive."""
    s = Geometry(int(g.nx), int(g.ny), int(g.nz), float(g.dx), float(g.dy), float(g.dz),
                 int(g.nu), int(g.nv), float(g.du), float(g.dv), float(g.sad), float(g.sdd),
                 int(g.n_views), None)
    ang = getattr(g, "angles", None)
    if ang is not None:
        a = np.ascontiguousarray(ang, dtype=np.float64)
        s._keep = a
        s.angles = a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    return s


TV_EPS, TV_TOL, TV_MAX_STEPS = 1e-5, 1e-3, 100


def options(lam: float, iters: Sequence[int], cgls_steps: int = 3, framelet_levels: int = 1,
            momentum: bool = True, positivity: bool = True, bin_detector: bool = True,
            storage: int = F32, profile: bool = False, op_pair: int = 0, regulariser: int = 0,
            tv_eps: float = TV_EPS, tv_tol: float = TV_TOL,
            tv_max_steps: int = TV_MAX_STEPS) -> Options:
    """regulariser 0: the tight-frame method (lam = the shrink threshold);
    1: the TV comparison method (lam = mu_TV)."""
    it = list(iters) + [0] * (4 - len(iters))
    return Options(float(lam), len(iters), (ctypes.c_int32 * 4)(*it), int(cgls_steps),
                   int(framelet_levels), int(bool(momentum)), int(bool(positivity)),
                   int(bool(bin_detector)), int(storage), int(bool(profile)), int(op_pair),
                   int(regulariser), float(tv_eps), float(tv_tol), int(tv_max_steps))


# ---------------------------------------------------------------- torch side
def _torch():
    import torch
    return torch


def dtype_code(t) -> int:
    torch = _torch()
    return {torch.float32: F32, torch.float16: F16, torch.bfloat16: BF16}[t]


def torch_dtype(code: int):
    torch = _torch()
    return {F32: torch.float32, F16: torch.float16, BF16: torch.bfloat16}[code]


def _stream(stream=None) -> int:
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return int(s.cuda_stream)


def _ptr(t) -> int:
    assert t.is_cuda and t.is_contiguous(), "device tensors must be contiguous GPU tensors"
    return int(t.data_ptr())


def _workspace(nbytes: int, device):
    torch = _torch()
    # torch allocations are 512-byte aligned
    return torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=device)


def workspace_size(g, opts: Options) -> int:
    n = ctypes.c_size_t(0)
    _check(load().tfcb_workspace_size(ctypes.byref(geometry(g)), ctypes.byref(opts),
                                      ctypes.byref(n)))
    return n.value


def operator_workspace_size(g, dt: int) -> int:
    n = ctypes.c_size_t(0)
    _check(load().tfcb_operator_workspace_size(ctypes.byref(geometry(g)), int(dt),
                                               ctypes.byref(n)))
    return n.value


def project(g, vol, out=None, ws=None, stream=None):
    """proj = P vol (device tensors, dtype float32/float16/bfloat16)."""
    torch = _torch()
    dt = dtype_code(vol.dtype)
    if out is None:
        out = torch.empty((g.n_views, g.nv, g.nu), dtype=vol.dtype, device=vol.device)
    need = operator_workspace_size(g, dt)
    if ws is None:
        ws = _workspace(need, vol.device)
    _check(load().tfcb_project(ctypes.byref(geometry(g)), dt, _ptr(vol), _ptr(out), _ptr(ws),
                               ws.numel() * ws.element_size(), _stream(stream)))
    return out


def backproject(g, proj, out=None, ws=None, stream=None):
    """vol = P^T proj (the exact transpose of project)."""
    torch = _torch()
    dt = dtype_code(proj.dtype)
    if out is None:
        out = torch.empty((g.nz, g.ny, g.nx), dtype=proj.dtype, device=proj.device)
    need = operator_workspace_size(g, dt)
    if ws is None:
        ws = _workspace(need, proj.device)
    _check(load().tfcb_backproject(ctypes.byref(geometry(g)), dt, _ptr(proj), _ptr(out), _ptr(ws),
                                   ws.numel() * ws.element_size(), _stream(stream)))
    return out


NOALLOC_SCRATCH_BYTES = 64 << 20


def backproject_noalloc(g, proj, out=None, stream=None):
    """vol = P^T proj through the entry point that allocates nothing (its
    scratch is the library's static per-GPU array)."""
    torch = _torch()
    dt = dtype_code(proj.dtype)
    if out is None:
        out = torch.empty((g.nz, g.ny, g.nx), dtype=proj.dtype, device=proj.device)
    _check(load().tfcb_backproject_noalloc(ctypes.byref(geometry(g)), dt, _ptr(proj), _ptr(out),
                                           _stream(stream)))
    return out


def project_siddon(g, vol, out=None, ws=None, stream=None):
    """proj = P vol by Siddon's ray tracing (the paper's projector)."""
    torch = _torch()
    dt = dtype_code(vol.dtype)
    if out is None:
        out = torch.empty((g.n_views, g.nv, g.nu), dtype=vol.dtype, device=vol.device)
    if ws is None:
        ws = _workspace(operator_workspace_size(g, dt), vol.device)
    _check(load().tfcb_project_siddon(ctypes.byref(geometry(g)), dt, _ptr(vol), _ptr(out),
                                      _ptr(ws), ws.numel() * ws.element_size(), _stream(stream)))
    return out


def backproject_eq3(g, proj, out=None, ws=None, stream=None):
    """vol = the Eq. (3) closed-form backprojection of proj."""
    torch = _torch()
    dt = dtype_code(proj.dtype)
    if out is None:
        out = torch.empty((g.nz, g.ny, g.nx), dtype=proj.dtype, device=proj.device)
    if ws is None:
        ws = _workspace(operator_workspace_size(g, dt), proj.device)
    _check(load().tfcb_backproject_eq3(ctypes.byref(geometry(g)), dt, _ptr(proj), _ptr(out),
                                       _ptr(ws), ws.numel() * ws.element_size(), _stream(stream)))
    return out


def framelet_shrink(vol, lam: float, levels: int = 1, positivity: bool = True, out=None,
                    stream=None):
    """out = H(W^T T_lambda W vol)."""
    torch = _torch()
    nz, ny, nx = vol.shape
    dt = dtype_code(vol.dtype)
    if out is None:
        out = torch.empty_like(vol)
    n = ctypes.c_size_t(0)
    lib = load()
    _check(lib.tfcb_framelet_workspace_size(nx, ny, nz, int(levels), dt, ctypes.byref(n)))
    ws = _workspace(n.value, vol.device) if n.value else None
    _check(lib.tfcb_framelet_shrink(nx, ny, nz, int(levels), float(lam), int(bool(positivity)),
                                    dt, _ptr(vol), _ptr(out), _ptr(ws) if ws is not None else None,
                                    ws.numel() if ws is not None else 0, _stream(stream)))
    return out


def fdk(g, proj, out=None, stream=None):
    """FDK reconstruction (the comparison baseline) of device projections."""
    torch = _torch()
    dt = dtype_code(proj.dtype)
    if out is None:
        out = torch.empty((g.nz, g.ny, g.nx), dtype=proj.dtype, device=proj.device)
    n = ctypes.c_size_t(0)
    lib = load()
    _check(lib.tfcb_fdk_workspace_size(ctypes.byref(geometry(g)), ctypes.byref(n)))
    ws = _workspace(n.value, proj.device)
    _check(lib.tfcb_fdk(ctypes.byref(geometry(g)), dt, _ptr(proj), _ptr(out), _ptr(ws),
                        ws.numel(), _stream(stream)))
    return out


def rof(x, mu: float, eps: float = TV_EPS, tol: float = TV_TOL, max_steps: int = TV_MAX_STEPS,
        positivity: bool = False, out=None, stream=None):
    """The ROF sub-problem of the TV method by the library's gradient descent
    (synchronises the stream).  Returns (out, accepted steps)."""
    torch = _torch()
    nz, ny, nx = x.shape
    dt = dtype_code(x.dtype)
    if out is None:
        out = torch.empty_like(x)
    n = ctypes.c_size_t(0)
    lib = load()
    _check(lib.tfcb_rof_workspace_size(nx, ny, nz, ctypes.byref(n)))
    ws = _workspace(n.value, x.device)
    steps = ctypes.c_int32(0)
    _check(lib.tfcb_rof(nx, ny, nz, float(mu), float(eps), float(tol), int(max_steps),
                        int(bool(positivity)), dt, _ptr(x), _ptr(out), _ptr(ws), ws.numel(),
                        _stream(stream), ctypes.byref(steps)))
    return out, int(steps.value)


def cgls(g, x, proj, n: int, stream=None, op_pair: int = 0):
    """n CGLS steps from x (updated in place), with the Joseph pair or
    (op_pair 1) the paper's Siddon / Eq. (3) pair.  Returns (x, resid2, broke)."""
    dt = dtype_code(x.dtype)
    opts = options(0.0, [1], cgls_steps=n, storage=dt, op_pair=op_pair)
    need = workspace_size(g, opts)
    ws = _workspace(need, x.device)
    stats = (ctypes.c_double * 2)()
    _check(load().tfcb_cgls(ctypes.byref(geometry(g)), ctypes.byref(opts), _ptr(x), _ptr(proj),
                            _ptr(ws), ws.numel(), _stream(stream), stats))
    return x, stats[0], bool(stats[1])


def restrict_sino(g_fine, proj, stream=None):
    torch = _torch()
    out = torch.empty((g_fine.n_views, (g_fine.nv + 1) // 2, (g_fine.nu + 1) // 2),
                      dtype=proj.dtype, device=proj.device)
    _check(load().tfcb_restrict_sino(ctypes.byref(geometry(g_fine)), dtype_code(proj.dtype),
                                     _ptr(proj), _ptr(out), _stream(stream)))
    return out


def prolong_vol(g_coarse, g_fine, vol, stream=None):
    torch = _torch()
    out = torch.empty((g_fine.nz, g_fine.ny, g_fine.nx), dtype=vol.dtype, device=vol.device)
    _check(load().tfcb_prolong_vol(ctypes.byref(geometry(g_coarse)), ctypes.byref(geometry(g_fine)),
                                   dtype_code(vol.dtype), _ptr(vol), _ptr(out), _stream(stream)))
    return out


def reconstruct(g, proj, lam: float, iters: Sequence[int], cgls_steps: int = 3,
                framelet_levels: int = 1, momentum: bool = True, positivity: bool = True,
                bin_detector: bool = True, storage: int = F32, out=None, ws=None, stream=None,
                check: bool = True, profile: bool = False, op_pair: int = 0,
                regulariser: int = 0, tv_eps: float = TV_EPS, tv_tol: float = TV_TOL,
                tv_max_steps: int = TV_MAX_STEPS):
    """The full method on device FP32 projections; returns (volume, report dict).
    op_pair 1 runs the CGLS with the paper's Siddon / Eq. (3) operators;
    regulariser 1 runs the TV comparison method with lam as mu_TV.
    The call synchronises the stream."""
    torch = _torch()
    opts = options(lam, iters, cgls_steps, framelet_levels, momentum, positivity, bin_detector,
                   storage, profile, op_pair, regulariser, tv_eps, tv_tol, tv_max_steps)
    if out is None:
        out = torch.empty((g.nz, g.ny, g.nx), dtype=torch.float32, device=proj.device)
    need = workspace_size(g, opts)
    if ws is None:
        ws = _workspace(need, proj.device)
    rep = Report()
    st = load().tfcb_reconstruct(ctypes.byref(geometry(g)), ctypes.byref(opts), _ptr(proj),
                                 _ptr(out), _ptr(ws), ws.numel(), _stream(stream),
                                 ctypes.byref(rep))
    if check:
        _check(st)
    report = {"status": st, "seconds_total": rep.seconds_total,
              "seconds_per_grid": list(rep.seconds_per_grid)[:len(iters)],
              "iters_done": list(rep.iters_done)[:len(iters)], "resid2_last": rep.resid2_last,
              "cgls_breakdowns": rep.cgls_breakdowns,
              "kernel_ms": list(rep.kernel_ms), "kernel_launches": list(rep.kernel_launches),
              "rof_steps": rep.rof_steps}
    return out, report


class Server:
    """Continuous-batching reconstruction server over a device arena (see the
    serving section of include/tfcb.h).  Submitted tensors are kept alive by
    this object until their request ends."""

    def __init__(self, arena_bytes: int, max_slots: int = 8, device=None):
        torch = _torch()
        self.device = device or torch.device("cuda:0")
        self.arena = torch.empty(int(arena_bytes), dtype=torch.uint8, device=self.device)
        h = ctypes.c_void_p()
        _check(load().tfcb_server_create(_ptr(self.arena), int(arena_bytes), int(max_slots),
                                         ctypes.byref(h)))
        self._h = h
        self._keep = {}

    @staticmethod
    def request_bytes(g, opts: Options) -> int:
        n = ctypes.c_size_t(0)
        _check(load().tfcb_request_bytes(ctypes.byref(geometry(g)), ctypes.byref(opts),
                                         ctypes.byref(n)))
        return n.value

    def submit(self, g, proj, opts: Options, out=None, stream=None) -> int:
        """Queues a request; its kernels wait for the work already enqueued
        on `stream` (default: torch's current stream), which produced proj."""
        torch = _torch()
        if out is None:
            out = torch.empty((g.nz, g.ny, g.nx), dtype=torch.float32, device=proj.device)
        rid = ctypes.c_uint64(0)
        _check(load().tfcb_server_submit(self._h, ctypes.byref(geometry(g)), ctypes.byref(opts),
                                         _ptr(proj), _ptr(out), _stream(stream),
                                         ctypes.byref(rid)))
        self._keep[rid.value] = (proj, out)
        return rid.value

    def step(self):
        a, q = ctypes.c_int32(0), ctypes.c_int32(0)
        _check(load().tfcb_server_step(self._h, ctypes.byref(a), ctypes.byref(q)))
        return a.value, q.value

    def poll(self, rid: int):
        st, res = ctypes.c_int32(0), ctypes.c_int32(0)
        t = ctypes.c_double(0.0)
        _check(load().tfcb_server_poll(self._h, int(rid), ctypes.byref(st), ctypes.byref(t),
                                       ctypes.byref(res)))
        return st.value, t.value, res.value

    def result(self, rid: int):
        return self._keep[rid][1]

    def release(self, rid: int):
        self._keep.pop(rid, None)

    def cancel(self, rid: int):
        _check(load().tfcb_server_cancel(self._h, int(rid)))

    def close(self):
        if self._h is not None:
            _check(load().tfcb_server_destroy(self._h))
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
