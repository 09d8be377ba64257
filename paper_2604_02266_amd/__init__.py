"""Python binding of libotfs: LMMSE-CG equalisation of Zak-OTFS frames on MI355X.

Argument marshalling only.  Every step of the computation runs in the HIP kernels of
libotfs.so (built in-tree for gfx950); PyTorch provides device memory and the stream.  If
the library is missing, every entry point raises: there is no CPU fallback.

Layout: a batch is one complex64 vector holding the frames back to back, each in the
order q = l*M + k (delay fastest).  Frames are described by objects with the attributes
M, N, tau, nu, h, lam and qam (workloads.FrameSpec is one).
"""
from __future__ import annotations

import ctypes
import os
import re
from typing import List, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# OTFS_LIB selects another build of the same library (e.g. a tuning variant)
LIB_PATH = os.environ.get("OTFS_LIB") or os.path.join(_HERE, "libotfs.so")
HEADER_PATH = os.path.join(os.path.dirname(_HERE), "include", "otfs.h")

# status codes and flags (include/otfs.h)
OK, E_INVAL, E_NOMEM, E_DEVICE, E_BUDGET, E_AGAIN, E_NOTFOUND, E_UNSUPPORTED, E_STATE = range(9)
D_STORED_BF16 = 1 << 0
Y_BF16 = 1 << 1
USE_GRAPH = 1 << 2
TIME_KERNEL = 1 << 3
LDS_GATHER = 1 << 8
AGENT_BARRIER = 1 << 4
NO_LDS_RESIDENT = 1 << 5
SPLIT_DIRECTION = 1 << 6
D_STORED_C64 = 1 << 7
(FRAME_RUNNING, FRAME_CONVERGED, FRAME_CAPPED, FRAME_NONFINITE, FRAME_BREAKDOWN, FRAME_TIMEOUT,
 FRAME_DRYRUN) = range(7)


class OtfsError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"libotfs status {status}: {msg}")
        self.status = status


class FrameDesc(ctypes.Structure):
    _fields_ = [("M", ctypes.c_int32), ("N", ctypes.c_int32), ("P", ctypes.c_int32),
                ("h", ctypes.POINTER(ctypes.c_float)),
                ("delay", ctypes.POINTER(ctypes.c_int32)),
                ("doppler", ctypes.POINTER(ctypes.c_int32)),
                ("noise_var", ctypes.c_float), ("qam", ctypes.c_int32)]


class CgOpts(ctypes.Structure):
    _fields_ = [("max_iters", ctypes.c_int32), ("rel_tol", ctypes.c_float),
                ("refresh_every", ctypes.c_int32), ("flags", ctypes.c_uint32)]


class FrameStats(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("rel_res", ctypes.c_float),
                ("status", ctypes.c_int32), ("tiles", ctypes.c_int32)]


class PlanInfo(ctypes.Structure):
    _fields_ = [("nframes", ctypes.c_int32), ("total_elems", ctypes.c_int64),
                ("grid", ctypes.c_int32), ("block", ctypes.c_int32),
                ("max_paths", ctypes.c_int32), ("tile_elems", ctypes.c_int32),
                ("groups", ctypes.c_int32), ("xcd_local", ctypes.c_int32),
                ("lds_bytes", ctypes.c_int32), ("staged_frames", ctypes.c_int32),
                ("resident_frames", ctypes.c_int32), ("launches", ctypes.c_int32),
                ("fused_direction_frames", ctypes.c_int32)]


class ServerStats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_uint64), ("completed", ctypes.c_uint64),
                ("steps", ctypes.c_uint64), ("queued", ctypes.c_uint64),
                ("active", ctypes.c_uint64), ("pool_bytes_in_use", ctypes.c_uint64),
                ("pool_bytes_peak", ctypes.c_uint64), ("ns_admit", ctypes.c_uint64),
                ("ns_step", ctypes.c_uint64), ("ns_gpu", ctypes.c_uint64),
                ("ns_fetch", ctypes.c_uint64)]


_lib = None
_vp = ctypes.c_void_p


def build_info() -> dict:
    """The loaded library's build stamp {"source_sha", "arch"}, and whether the sources in
    this tree still hash to it ("current")."""
    raw = lib().otfs_build_info().decode()
    info = dict(kv.split("=", 1) for kv in raw.split())
    try:
        from .build_lib import source_sha
        info["current"] = info.get("source_sha") == source_sha()
    except OSError:   # sources not shipped with the library
        info["current"] = None
    return info


def header_functions() -> List[str]:
    """Names of the functions include/otfs.h declares."""
    txt = open(HEADER_PATH).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(otfs_[A-Za-z_0-9]+)\s*\(", txt)))


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built; run paper_2604_02266_amd/build_lib.py first "
                           "(there is no fallback implementation)")
    L = ctypes.CDLL(LIB_PATH)
    st = ctypes.c_int
    sig = {
        "otfs_last_error": (ctypes.c_char_p, []),
        "otfs_build_info": (ctypes.c_char_p, []),
        "otfs_plan": (st, [ctypes.POINTER(FrameDesc), ctypes.c_int32, ctypes.POINTER(CgOpts),
                           ctypes.POINTER(_vp)]),
        "otfs_plan_workspace_bytes": (st, [_vp, ctypes.POINTER(ctypes.c_size_t),
                                           ctypes.POINTER(ctypes.c_int64)]),
        "otfs_plan_bind": (st, [_vp, _vp, ctypes.c_size_t, _vp]),
        "otfs_plan_free": (st, [_vp]),
        "otfs_plan_info": (st, [_vp, ctypes.POINTER(PlanInfo)]),
        "otfs_plan_set_tiling": (st, [_vp, ctypes.c_int32, ctypes.c_int32]),
        "otfs_plan_set_staging": (st, [_vp, ctypes.c_int32]),
        "otfs_plan_set_window": (st, [_vp, ctypes.c_int32, ctypes.c_int32]),
        "otfs_apply_H": (st, [_vp, _vp, _vp, _vp]),
        "otfs_apply_HH": (st, [_vp, _vp, _vp, _vp]),
        "otfs_lmmse_cg": (st, [_vp, _vp, _vp, _vp, _vp, _vp]),
        "otfs_lmmse_cg_plain": (st, [_vp, _vp, _vp, _vp, _vp, _vp]),
        "otfs_lmmse_cg_noalloc": (st, [_vp, _vp, _vp, _vp, _vp, _vp]),
        "otfs_plan_kernel_ms": (st, [_vp, ctypes.POINTER(ctypes.c_float)]),
        "otfs_plan_set_wait_limit": (st, [_vp, ctypes.c_int64]),
        "otfs_plan_paths_from_pilot": (st, [_vp, _vp, ctypes.c_float, _vp, _vp]),
        "otfs_plan_get_paths": (st, [_vp, ctypes.c_int32, ctypes.c_int32,
                                     ctypes.POINTER(ctypes.c_int32), _vp, _vp, _vp, _vp]),
        "otfs_bit_errors": (st, [_vp, _vp, _vp, _vp, _vp]),
        "otfs_dzt": (st, [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, _vp, _vp,
                          ctypes.c_int32, _vp]),
        "otfs_lmmse_cg_trace": (st, [_vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp]),
        "otfs_server_create": (st, [ctypes.c_int, _vp, ctypes.c_size_t, ctypes.POINTER(CgOpts),
                                    ctypes.c_int32, ctypes.POINTER(_vp)]),
        "otfs_submit": (st, [_vp, ctypes.POINTER(FrameDesc), _vp,
                             ctypes.POINTER(ctypes.c_uint64)]),
        "otfs_poll": (st, [_vp, ctypes.c_uint64, _vp, _vp, ctypes.POINTER(FrameStats),
                           ctypes.POINTER(ctypes.c_uint64)]),
        "otfs_submit_many": (st, [_vp, ctypes.POINTER(FrameDesc), ctypes.c_int32,
                                  ctypes.POINTER(_vp), ctypes.POINTER(ctypes.c_uint64)]),
        "otfs_poll_many": (st, [_vp, ctypes.POINTER(ctypes.c_uint64), ctypes.c_int32,
                                ctypes.POINTER(_vp), ctypes.POINTER(_vp),
                                ctypes.POINTER(FrameStats), ctypes.POINTER(ctypes.c_uint64),
                                ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32)]),
        "otfs_server_stats": (st, [_vp, ctypes.POINTER(ServerStats)]),
        "otfs_server_set_tiling": (st, [_vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32]),
        "otfs_server_frame_bytes": (st, [_vp, ctypes.POINTER(FrameDesc),
                                         ctypes.POINTER(ctypes.c_size_t),
                                         ctypes.POINTER(ctypes.c_size_t)]),
        "otfs_server_free": (st, [_vp]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    _lib = L
    return L


def last_error() -> str:
    return lib().otfs_last_error().decode()


def _check(status: int):
    if status != OK:
        raise OtfsError(status, last_error())


def _torch():
    import torch
    return torch


def _stream_ptr(stream=None) -> int:
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return int(s.cuda_stream)


def _ptr(t) -> Optional[int]:
    return None if t is None else int(t.data_ptr())


class _Descs:
    """ctypes frame descriptors plus the numpy arrays they point into."""

    def __init__(self, frames: Sequence):
        self.keep = []
        self.arr = (FrameDesc * max(len(frames), 1))()
        for i, f in enumerate(frames):
            h = np.ascontiguousarray(np.stack([np.real(f.h), np.imag(f.h)], axis=1)
                                     .astype(np.float32).reshape(-1))
            tau = np.ascontiguousarray(np.asarray(f.tau, dtype=np.int32))
            nu = np.ascontiguousarray(np.asarray(f.nu, dtype=np.int32))
            self.keep += [h, tau, nu]
            d = self.arr[i]
            d.M, d.N, d.P = int(f.M), int(f.N), int(tau.shape[0])
            d.h = h.ctypes.data_as(ctypes.POINTER(ctypes.c_float))
            d.delay = tau.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
            d.doppler = nu.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
            d.noise_var = float(f.lam)
            d.qam = int(getattr(f, "qam", 0) or 0)


def make_opts(max_iters=50, rel_tol=1e-6, refresh_every=0, flags=0) -> CgOpts:
    return CgOpts(int(max_iters), float(rel_tol), int(refresh_every), int(flags))


class Plan:
    """A bound batch of frames: otfs_plan + a torch-owned workspace + otfs_plan_bind."""

    def __init__(self, frames: Sequence, max_iters: int = 50, rel_tol: float = 1e-6,
                 refresh_every: int = 0, flags: int = 0, tile_elems: int = 0,
                 max_grid: int = 0, stage_bytes: Optional[int] = None,
                 window: Optional[Sequence[int]] = None, bind: bool = True,
                 tune: bool = True):
        self._lib = lib()
        self.frames = list(frames)
        # launch shape stored by the autotuner for this batch signature, unless the caller
        # chose one
        self.tuned = None
        if tune and not tile_elems and stage_bytes is None and window is None and self.frames:
            from . import autotune
            self.tuned = autotune.lookup(self.frames, refresh_every, flags)
            if self.tuned is not None:
                tile_elems = int(self.tuned["tile_elems"])
                stage_bytes = int(self.tuned["stage_bytes"]) or None
                if self.tuned["split_direction"]:
                    flags |= SPLIT_DIRECTION
                if self.tuned.get("lds_gather"):
                    flags |= LDS_GATHER
        self.opts = make_opts(max_iters, rel_tol, refresh_every, flags)
        descs = _Descs(self.frames)
        h = _vp()
        _check(self._lib.otfs_plan(descs.arr, len(self.frames), ctypes.byref(self.opts),
                                   ctypes.byref(h)))
        self._h = h
        self.ws = None
        if tile_elems or max_grid:
            _check(self._lib.otfs_plan_set_tiling(self._h, int(tile_elems), int(max_grid)))
        if stage_bytes is not None:
            _check(self._lib.otfs_plan_set_staging(self._h, int(stage_bytes)))
        if window is not None:
            _check(self._lib.otfs_plan_set_window(self._h, int(window[0]), int(window[1])))
        if bind:
            self.bind()

    # ---- lifetime ----
    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            self._lib.otfs_plan_free(self._h)
            self._h = _vp()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---- plan queries ----
    def workspace_bytes(self):
        nb = ctypes.c_size_t()
        ne = ctypes.c_int64()
        _check(self._lib.otfs_plan_workspace_bytes(self._h, ctypes.byref(nb), ctypes.byref(ne)))
        return int(nb.value), int(ne.value)

    @property
    def total_elems(self) -> int:
        return self.workspace_bytes()[1]

    @property
    def nframes(self) -> int:
        return len(self.frames)

    def info(self) -> PlanInfo:
        inf = PlanInfo()
        _check(self._lib.otfs_plan_info(self._h, ctypes.byref(inf)))
        return inf

    def set_tiling(self, tile_elems: int = 0, max_grid: int = 0, rebind: bool = True):
        _check(self._lib.otfs_plan_set_tiling(self._h, int(tile_elems), int(max_grid)))
        if rebind:
            self.bind()

    def bind(self, stream=None):
        torch = _torch()
        nbytes, _ = self.workspace_bytes()
        raw = torch.empty(nbytes + 256, dtype=torch.uint8, device="cuda")
        base = raw.data_ptr()
        pad = (-base) % 256
        self.ws = raw
        _check(self._lib.otfs_plan_bind(self._h, _vp(base + pad), nbytes,
                                        _vp(_stream_ptr(stream))))

    # ---- buffers ----
    def _vec(self, t, name, dtype=None):
        torch = _torch()
        dtype = dtype or torch.complex64
        n = self.total_elems
        if t is None:
            return torch.empty(n, dtype=dtype, device="cuda")
        if t.dtype != dtype or not t.is_cuda or not t.is_contiguous() or t.numel() != n:
            raise ValueError(f"{name}: need a contiguous cuda {dtype} tensor of {n} elements")
        return t

    def _y(self, y):
        torch = _torch()
        if self.opts.flags & Y_BF16:
            if (y.dtype != torch.bfloat16 or not y.is_cuda or not y.is_contiguous()
                    or y.numel() != 2 * self.total_elems):
                raise ValueError("y: with Y_BF16 need a contiguous cuda bfloat16 tensor of "
                                 "2 * total_elems values (re, im)")
            return y
        return self._vec(y, "y")

    def new_stats(self):
        torch = _torch()
        return torch.zeros((max(self.nframes, 1), 4), dtype=torch.int32, device="cuda")

    # ---- operator ----
    def apply_H(self, x, y=None, stream=None):
        x = self._vec(x, "x")
        y = self._vec(y, "y")
        _check(self._lib.otfs_apply_H(self._h, _vp(_ptr(x)), _vp(_ptr(y)), _vp(_stream_ptr(stream))))
        return y

    def apply_HH(self, y, x=None, stream=None):
        y = self._vec(y, "y")
        x = self._vec(x, "x")
        _check(self._lib.otfs_apply_HH(self._h, _vp(_ptr(y)), _vp(_ptr(x)), _vp(_stream_ptr(stream))))
        return x

    # ---- solver ----
    def _solve(self, fn, y, xhat, sym, stats, stream):
        torch = _torch()
        y = self._y(y)
        xhat = self._vec(xhat, "xhat")
        if sym is not None:
            sym = self._vec(sym, "sym", torch.uint8)
        if stats is not None and (stats.dtype != torch.int32 or stats.numel() < 4 * self.nframes
                                  or not stats.is_contiguous() or not stats.is_cuda):
            raise ValueError("stats: need a contiguous cuda int32 tensor of shape (nframes, 4)")
        _check(fn(self._h, _vp(_ptr(y)), _vp(_ptr(xhat)), _vp(_ptr(sym)), _vp(_ptr(stats)),
                  _vp(_stream_ptr(stream))))
        return xhat

    def lmmse_cg(self, y, xhat=None, sym=None, stats=None, stream=None):
        return self._solve(self._lib.otfs_lmmse_cg, y, xhat, sym, stats, stream)

    def lmmse_cg_plain(self, y, xhat=None, sym=None, stats=None, stream=None):
        return self._solve(self._lib.otfs_lmmse_cg_plain, y, xhat, sym, stats, stream)

    def lmmse_cg_noalloc(self, y, xhat=None, sym=None, stats=None, stream=None):
        """otfs_lmmse_cg_noalloc: the plan is rebound to the library's static scratch."""
        return self._solve(self._lib.otfs_lmmse_cg_noalloc, y, xhat, sym, stats, stream)

    def paths_from_pilot(self, ypilot, theta: float = 0.08, npaths=None, stream=None):
        """otfs_plan_paths_from_pilot: the frames' paths from their received pilot frames
        (complex64, batch layout).  Returns the int32 tensor of per-frame counts above
        theta."""
        torch = _torch()
        ypilot = self._vec(ypilot, "ypilot")
        if npaths is None:
            npaths = torch.zeros(max(self.nframes, 1), dtype=torch.int32, device="cuda")
        _check(self._lib.otfs_plan_paths_from_pilot(self._h, _vp(_ptr(ypilot)), float(theta),
                                                    _vp(_ptr(npaths)), _vp(_stream_ptr(stream))))
        return npaths

    def bit_errors(self, sym, sym_tx, errs=None, stream=None):
        """otfs_bit_errors: per-frame bit errors (Gray map) of decisions vs transmitted."""
        torch = _torch()
        sym = self._vec(sym, "sym", torch.uint8)
        sym_tx = self._vec(sym_tx, "sym_tx", torch.uint8)
        if errs is None:
            errs = torch.zeros(max(self.nframes, 1), dtype=torch.int64, device="cuda")
        _check(self._lib.otfs_bit_errors(self._h, _vp(_ptr(sym)), _vp(_ptr(sym_tx)),
                                         _vp(_ptr(errs)), _vp(_stream_ptr(stream))))
        return errs

    def lmmse_cg_trace(self, y, sym_tx, xhat=None, sym=None, stats=None, stream=None):
        """otfs_lmmse_cg_trace: returns (xhat, sym, errs) with errs of shape
        (max_iters, nframes): bit errors after each iteration."""
        torch = _torch()
        y = self._y(y)
        xhat = self._vec(xhat, "xhat")
        sym = self._vec(sym, "sym", torch.uint8)
        sym_tx = self._vec(sym_tx, "sym_tx", torch.uint8)
        errs = torch.zeros((self.opts.max_iters, max(self.nframes, 1)), dtype=torch.int64,
                           device="cuda")
        _check(self._lib.otfs_lmmse_cg_trace(self._h, _vp(_ptr(y)), _vp(_ptr(xhat)),
                                             _vp(_ptr(sym)), _vp(_ptr(stats)),
                                             _vp(_ptr(sym_tx)), _vp(_ptr(errs)),
                                             _vp(_stream_ptr(stream))))
        return xhat, sym, errs

    def get_paths(self, frame: int, stream=None):
        """otfs_plan_get_paths: (delay, doppler, h) of a frame's paths on the device."""
        cap = max(int(getattr(self.frames[frame], "P", 0) or
                      np.asarray(self.frames[frame].tau).shape[0]), 64)
        P = ctypes.c_int32()
        tau = np.zeros(cap, dtype=np.int32)
        nu = np.zeros(cap, dtype=np.int32)
        h = np.zeros(2 * cap, dtype=np.float32)
        _check(self._lib.otfs_plan_get_paths(self._h, int(frame), cap, ctypes.byref(P),
                                             _vp(tau.ctypes.data), _vp(nu.ctypes.data),
                                             _vp(h.ctypes.data), _vp(_stream_ptr(stream))))
        n = min(int(P.value), cap)
        return tau[:n].copy(), nu[:n].copy(), (h[0:2 * n:2] + 1j * h[1:2 * n:2]).astype(np.complex64)

    def set_wait_limit(self, wait_us: int):
        _check(self._lib.otfs_plan_set_wait_limit(self._h, int(wait_us)))

    def kernel_ms(self) -> float:
        ms = ctypes.c_float()
        _check(self._lib.otfs_plan_kernel_ms(self._h, ctypes.byref(ms)))
        return float(ms.value)


class Server:
    """Continuous-batching server: otfs_server_create over a torch-owned pool.

    device=-1 gives a dry run (scheduling only, no device work, no torch needed).
    """

    def __init__(self, pool_bytes: int, max_iters: int = 50, rel_tol: float = 1e-6,
                 refresh_every: int = 0, flags: int = 0, step_iters: int = 10,
                 device: Optional[int] = None, tune: bool = True):
        self._lib = lib()
        self.opts = make_opts(max_iters, rel_tol, refresh_every, flags)
        self.pool = None
        ptr = 0
        if device is None:
            device = _torch().cuda.current_device()
        if device >= 0:
            torch = _torch()
            raw = torch.empty(int(pool_bytes) + 256, dtype=torch.uint8,
                              device=f"cuda:{device}")
            ptr = raw.data_ptr() + (-raw.data_ptr()) % 256
            self.pool = raw
        h = _vp()
        _check(self._lib.otfs_server_create(int(device), _vp(ptr), int(pool_bytes),
                                            ctypes.byref(self.opts), int(step_iters),
                                            ctypes.byref(h)))
        self._h = h
        self.device = device
        if tune:   # per-shape tiles stored by the autotuner
            from . import autotune
            for shape, te in autotune.serving_tiles().items():
                M, N = (int(v) for v in shape.split("x"))
                self.set_tiling(M, N, te)

    def set_tiling(self, M: int, N: int, tile_elems: int):
        _check(self._lib.otfs_server_set_tiling(self._h, int(M), int(N), int(tile_elems)))

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            self._lib.otfs_server_free(self._h)
            self._h = _vp()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    @staticmethod
    def prepare(frame) -> "_Descs":
        """The frame's descriptor built once, for repeated submits of the same channel."""
        return frame if isinstance(frame, _Descs) else _Descs([frame])

    def submit(self, frame, y) -> int:
        """Queue one frame (a frame spec, or its prepare() result); y: host complex64 array
        of M*N values (copied)."""
        descs = self.prepare(frame)
        E = int(descs.arr[0].M) * int(descs.arr[0].N)
        if not (isinstance(y, np.ndarray) and y.dtype == np.complex64 and y.flags.c_contiguous):
            y = np.ascontiguousarray(np.asarray(y, dtype=np.complex64))
        if y.size != E:
            raise ValueError(f"y: need {E} values, got {y.size}")
        t = ctypes.c_uint64()
        _check(self._lib.otfs_submit(self._h, descs.arr, _vp(y.ctypes.data), ctypes.byref(t)))
        return int(t.value)

    def poll(self, ticket: int, frame, out=None):
        """None while running; else (xhat, sym or None, FrameStats, latency_s).  out: an
        optional (xhat, sym) pair of arrays (complex64 and uint8, M*N each; sym may be None)
        to receive the results instead of new arrays."""
        if isinstance(frame, _Descs):
            E, qam = int(frame.arr[0].M) * int(frame.arr[0].N), int(frame.arr[0].qam)
        else:
            E, qam = int(frame.M) * int(frame.N), int(getattr(frame, "qam", 0) or 0)
        if out is not None:
            x, sym = out
            if x.dtype != np.complex64 or x.size != E or not x.flags.c_contiguous or (
                    sym is not None and (sym.dtype != np.uint8 or sym.size != E)):
                raise ValueError("out: need complex64 and uint8 arrays of M*N values")
            if qam <= 0:
                sym = None
        else:
            x = np.empty(E, dtype=np.complex64)
            sym = np.empty(E, dtype=np.uint8) if qam > 0 else None
        st = FrameStats()
        lat = ctypes.c_uint64()
        status = self._lib.otfs_poll(self._h, ctypes.c_uint64(ticket), _vp(x.ctypes.data),
                                     _vp(sym.ctypes.data) if sym is not None else None,
                                     ctypes.byref(st), ctypes.byref(lat))
        if status == E_AGAIN:
            return None
        _check(status)
        return x, sym, st, lat.value * 1e-9

    def submit_many(self, frames, ys) -> List[int]:
        """Queue frames[i] (specs or prepare() results) with received frames ys[i] (host
        complex64 arrays, copied) in one call; returns their tickets."""
        n = len(frames)
        if n != len(ys):
            raise ValueError("need one y per frame")
        arr = (FrameDesc * max(n, 1))()
        keep = []
        ptrs = (_vp * max(n, 1))()
        for i, (f, y) in enumerate(zip(frames, ys)):
            d = self.prepare(f)
            keep.append(d)
            arr[i] = d.arr[0]
            E = int(d.arr[0].M) * int(d.arr[0].N)
            if not (isinstance(y, np.ndarray) and y.dtype == np.complex64 and y.flags.c_contiguous):
                y = np.ascontiguousarray(np.asarray(y, dtype=np.complex64))
            if y.size != E:
                raise ValueError(f"ys[{i}]: need {E} values, got {y.size}")
            keep.append(y)
            ptrs[i] = y.ctypes.data
        t = (ctypes.c_uint64 * max(n, 1))()
        _check(self._lib.otfs_submit_many(self._h, arr, n, ptrs, t))
        return [int(t[i]) for i in range(n)]

    def poll_many(self, tickets, outs):
        """Poll tickets[i] into outs[i] = (xhat, sym or None) arrays (complex64 / uint8, M*N
        each).  Returns a list with (FrameStats, latency_s) for the finished tickets and None
        for those still running."""
        n = len(tickets)
        tk = (ctypes.c_uint64 * max(n, 1))(*tickets)
        xp = (_vp * max(n, 1))()
        sp = (_vp * max(n, 1))()
        for i, (x, sym) in enumerate(outs):
            if x.dtype != np.complex64 or not x.flags.c_contiguous:
                raise ValueError("outs: xhat must be a contiguous complex64 array")
            xp[i] = x.ctypes.data
            sp[i] = sym.ctypes.data if sym is not None else None
        stats = (FrameStats * max(n, 1))()
        lat = (ctypes.c_uint64 * max(n, 1))()
        status = (ctypes.c_int32 * max(n, 1))()
        nd = ctypes.c_int32()
        _check(self._lib.otfs_poll_many(self._h, tk, n, xp, sp, stats, lat, status,
                                        ctypes.byref(nd)))
        res = []
        for i in range(n):
            if status[i] == 0:
                res.append((stats[i], lat[i] * 1e-9))
            elif status[i] == E_AGAIN:
                res.append(None)
            else:
                raise OtfsError(int(status[i]), f"ticket {tickets[i]}: status {status[i]}")
        return res

    def wait(self, ticket: int, frame, timeout: float = 60.0, sleep: float = 1e-4, out=None):
        import time
        t_end = time.monotonic() + timeout
        while True:
            r = self.poll(ticket, frame, out=out)
            if r is not None:
                return r
            if time.monotonic() > t_end:
                raise TimeoutError(f"ticket {ticket} not done after {timeout} s")
            time.sleep(sleep)

    def frame_bytes(self, frame):
        """(pool bytes one admitted frame of this shape holds, control region bytes)."""
        fb = ctypes.c_size_t()
        cb = ctypes.c_size_t()
        descs = _Descs([frame])
        _check(self._lib.otfs_server_frame_bytes(self._h, descs.arr, ctypes.byref(fb),
                                                 ctypes.byref(cb)))
        return int(fb.value), int(cb.value)

    def stats(self) -> ServerStats:
        out = ServerStats()
        _check(self._lib.otfs_server_stats(self._h, ctypes.byref(out)))
        return out


def dzt(x, M: int, N: int, inverse: bool = False, out=None, stream=None):
    """otfs_dzt: DZT (Eq. zak) or its inverse (Eq. iZak) of a contiguous complex64 tensor
    holding nframes frames of M*N samples; returns the output tensor."""
    torch = _torch()
    if x.dtype != torch.complex64 or not x.is_cuda or not x.is_contiguous() or x.numel() % (M * N):
        raise ValueError("x: need a contiguous cuda complex64 tensor of nframes * M * N values")
    out = torch.empty_like(x) if out is None else out
    _check(lib().otfs_dzt(int(M), int(N), x.numel() // (M * N), _vp(_ptr(x)), _vp(_ptr(out)),
                          int(bool(inverse)), _vp(_stream_ptr(stream))))
    return out


def stats_numpy(stats) -> np.ndarray:
    """(nframes, 4) int32 device tensor -> structured array (iters, rel_res, status, tiles)."""
    a = stats.detach().cpu().numpy().astype(np.int32)
    out = np.zeros(a.shape[0], dtype=[("iters", np.int32), ("rel_res", np.float32),
                                      ("status", np.int32), ("tiles", np.int32)])
    out["iters"] = a[:, 0]
    out["rel_res"] = a[:, 1].view(np.float32)
    out["status"] = a[:, 2]
    out["tiles"] = a[:, 3]
    return out


def frame_offsets(frames: Sequence) -> np.ndarray:
    sizes = np.array([int(f.M) * int(f.N) for f in frames], dtype=np.int64)
    return np.concatenate([[0], np.cumsum(sizes)])
