"""ctypes binding of the raybornhf C ABI (include/raybornhf.h).

Argument marshalling only: tensors are allocated with torch on the GPU and their device
pointers are handed to the library; every step of the computation runs in the HIP kernels.
There is no fallback: without the built library or a GPU, calls raise.
"""
from __future__ import annotations

import ctypes
import dataclasses
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libraybornhf.so")

RB_OK, RB_EINVAL, RB_ENOMEM, RB_EDEVICE, RB_ENONFINITE, RB_EUNSUPPORTED = 0, -1, -2, -3, -4, -5
RB_F32, RB_BF16, RB_F16, RB_F16X = 1, 2, 3, 4
RB_RAY_BORN, RB_RAY_ONLY = 0, 1
RB_GREEN_RAY, RB_GREEN_WATER = 0, 1

SYMBOLS = (
    "rb_create", "rb_destroy", "rb_last_error", "rb_mask_count", "rb_refractive_index",
    "rb_trace_rays", "rb_build_green", "rb_born_forward", "rb_born_adjoint", "rb_residual",
    "rb_backproject", "rb_frequency_step", "rb_profile_enable", "rb_profile_read",
    "rb_stage_name", "rb_trace_lost_nodes", "rb_trace_samples", "rb_frequency_sweep",
    "rb_frequency_step_batch", "rb_step_bytes", "rb_set_sample_budget", "rb_autotune",
    "rb_set_tuning", "rb_get_tuning", "rb_set_receiver_linking", "rb_workspace_bytes",
    "rb_reserve", "rb_backproject_noalloc", "rb_gauss_newton_step", "rb_lossy_maps",
    "rb_trace_rays_lossy", "rb_backproject_lossy", "rb_frequency_step_lossy",
)
RB_TILE_256x128, RB_TILE_128x128 = 0, 1
GROUP_MAX = 16  # scans per rb_frequency_step_batch call
N_STAGES = 12


class Ring(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("radius", ctypes.c_double), ("psi0", ctypes.c_double)]


class Grid(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("dx", ctypes.c_double),
                ("x0", ctypes.c_double), ("y0", ctypes.c_double),
                ("mask_radius", ctypes.c_double)]


class TraceParams(ctypes.Structure):
    _fields_ = [("n_rays", ctypes.c_int32), ("max_steps", ctypes.c_int32),
                ("ds", ctypes.c_double), ("c0", ctypes.c_double)]


class _Tables(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("n_mask", ctypes.c_int32),
                ("T", ctypes.c_void_p), ("A", ctypes.c_void_p), ("ux", ctypes.c_void_p),
                ("uy", ctypes.c_void_p), ("flags", ctypes.c_void_p), ("rx_T", ctypes.c_void_p),
                ("rx_A", ctypes.c_void_p), ("rx_flags", ctypes.c_void_p)]


class _Absorption(ctypes.Structure):
    _fields_ = [("alpha0", ctypes.c_void_p), ("y", ctypes.c_double)]


class _Green(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("n_mask", ctypes.c_int32), ("prec", ctypes.c_int),
                ("G", ctypes.c_void_p), ("H", ctypes.c_void_p), ("scales", ctypes.c_void_p)]


class Report(ctypes.Structure):
    """rb_report (lives in device memory; this host mirror decodes a copy of it)."""
    _fields_ = [("status", ctypes.c_int32), ("flags", ctypes.c_int32),
                ("lost_nodes", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("ray_samples", ctypes.c_int64)]


REPORT_BYTES = ctypes.sizeof(Report)


def decode_report(t: torch.Tensor) -> Report:
    """A device rb_report (uint8 tensor of REPORT_BYTES) read back into a Report."""
    raw = bytes(t.detach().cpu().numpy().tobytes())
    return Report.from_buffer_copy(raw)


class _ScanStep(ctypes.Structure):
    _fields_ = [("ctx", ctypes.c_void_p), ("grid", ctypes.POINTER(Grid)),
                ("ring", ctypes.POINTER(Ring)), ("tp", ctypes.POINTER(TraceParams)),
                ("c", ctypes.c_void_p), ("smooth_w", ctypes.c_int32),
                ("n_omega", ctypes.c_int32), ("omega", ctypes.POINTER(ctypes.c_double)),
                ("d_omega", ctypes.POINTER(ctypes.c_double)), ("data", ctypes.c_void_p),
                ("tau", ctypes.c_double), ("mode", ctypes.c_int),
                ("residual_norm", ctypes.c_void_p)]


class Tuning(ctypes.Structure):
    """rb_tuning: forward launch configuration of one shape."""
    _fields_ = [("n", ctypes.c_int32), ("n_mask", ctypes.c_int32), ("prec", ctypes.c_int),
                ("fwd_tile", ctypes.c_int), ("fwd_splitk", ctypes.c_int32),
                ("fwd_ms", ctypes.c_float)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class RayBornError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"raybornhf status {status}: {msg}")
        self.status = status


_lib = None


def load(path: str = LIB_PATH):
    """Load the shared library (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with paper_2211_00316_amd/build.py")
    lib = ctypes.CDLL(path)
    P, I32, D = ctypes.c_void_p, ctypes.c_int32, ctypes.c_double
    sig = {
        "rb_create": ([ctypes.POINTER(P), ctypes.c_int, P], ctypes.c_int),
        "rb_destroy": ([P], None),
        "rb_last_error": ([P], ctypes.c_char_p),
        "rb_mask_count": ([ctypes.POINTER(Grid)], ctypes.c_int64),
        "rb_refractive_index": ([P, ctypes.POINTER(Grid), P, D, I32, P], ctypes.c_int),
        "rb_trace_rays": ([P, ctypes.POINTER(Grid), ctypes.POINTER(Ring),
                           ctypes.POINTER(TraceParams), P, ctypes.POINTER(_Tables)], ctypes.c_int),
        "rb_build_green": ([P, ctypes.POINTER(_Tables), D, D, ctypes.POINTER(_Green)],
                           ctypes.c_int),
        "rb_born_forward": ([P, ctypes.POINTER(_Green), P, P, P], ctypes.c_int),
        "rb_born_adjoint": ([P, ctypes.POINTER(_Green), P, P, P], ctypes.c_int),
        "rb_residual": ([P, ctypes.POINTER(_Tables), D, D, P, P, P], ctypes.c_int),
        "rb_backproject": ([P, ctypes.POINTER(_Green), P, P, D, D, P, I32], ctypes.c_int),
        "rb_backproject_noalloc": ([P, ctypes.POINTER(_Green), P, P, D, D, P, I32],
                                   ctypes.c_int),
        "rb_frequency_step": ([P, ctypes.POINTER(Grid), ctypes.POINTER(Ring),
                               ctypes.POINTER(TraceParams), P, I32, I32,
                               ctypes.POINTER(D), ctypes.POINTER(D), P, D, ctypes.c_int,
                               ctypes.c_int, P, P], ctypes.c_int),
        "rb_frequency_sweep": ([P, ctypes.POINTER(Grid), ctypes.POINTER(Ring),
                                ctypes.POINTER(TraceParams), P, I32, ctypes.POINTER(I32),
                                ctypes.POINTER(I32), ctypes.POINTER(D), ctypes.POINTER(D), P, D,
                                ctypes.c_int, ctypes.c_int, I32, P], ctypes.c_int),
        "rb_profile_enable": ([P, I32], ctypes.c_int),
        "rb_profile_read": ([P, ctypes.POINTER(D), ctypes.POINTER(ctypes.c_int64)], ctypes.c_int),
        "rb_stage_name": ([I32], ctypes.c_char_p),
        "rb_trace_lost_nodes": ([P], ctypes.c_int64),
        "rb_trace_samples": ([P], ctypes.c_int64),
        "rb_frequency_step_batch": ([ctypes.POINTER(_ScanStep), I32, ctypes.c_int,
                                     ctypes.POINTER(ctypes.c_int)], ctypes.c_int),
        "rb_step_bytes": ([ctypes.POINTER(Grid), ctypes.POINTER(Ring),
                           ctypes.POINTER(TraceParams), ctypes.c_int, ctypes.c_size_t],
                          ctypes.c_size_t),
        "rb_set_sample_budget": ([P, ctypes.c_size_t], ctypes.c_int),
        "rb_autotune": ([P, ctypes.POINTER(Grid), ctypes.POINTER(Ring), ctypes.c_int,
                         ctypes.POINTER(Tuning)], ctypes.c_int),
        "rb_set_tuning": ([P, ctypes.POINTER(Tuning)], ctypes.c_int),
        "rb_get_tuning": ([P, ctypes.POINTER(Tuning)], ctypes.c_int),
        "rb_set_receiver_linking": ([P, I32, D], ctypes.c_int),
        "rb_workspace_bytes": ([ctypes.POINTER(Grid), ctypes.POINTER(Ring),
                                ctypes.POINTER(TraceParams), ctypes.c_int, ctypes.c_size_t],
                               ctypes.c_size_t),
        "rb_reserve": ([P, ctypes.POINTER(Grid), ctypes.POINTER(Ring),
                        ctypes.POINTER(TraceParams), ctypes.c_int], ctypes.c_int),
        "rb_lossy_maps": ([P, ctypes.POINTER(Grid), P, ctypes.POINTER(_Absorption), D, D, I32,
                           P, P], ctypes.c_int),
        "rb_trace_rays_lossy": ([P, ctypes.POINTER(Grid), ctypes.POINTER(Ring),
                                 ctypes.POINTER(TraceParams), P, P, ctypes.POINTER(_Tables)],
                                ctypes.c_int),
        "rb_backproject_lossy": ([P, ctypes.POINTER(_Green), P, P, P, D, D, D, P, I32],
                                 ctypes.c_int),
        "rb_frequency_step_lossy": ([P, ctypes.POINTER(Grid), ctypes.POINTER(Ring),
                                     ctypes.POINTER(TraceParams), P, ctypes.POINTER(_Absorption),
                                     I32, I32, ctypes.POINTER(D), ctypes.POINTER(D), P, D,
                                     ctypes.c_int, ctypes.c_int, P, P], ctypes.c_int),
        "rb_gauss_newton_step": ([P, ctypes.POINTER(Grid), ctypes.POINTER(Ring),
                                  ctypes.POINTER(TraceParams), P, I32, I32, ctypes.POINTER(D),
                                  P, D, I32, ctypes.c_int, ctypes.c_int, P, P, P],
                                 ctypes.c_int),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    _lib = lib
    return lib


def mask_count(grid: Grid) -> int:
    return int(load().rb_mask_count(ctypes.byref(grid)))


def step_bytes(grid: Grid, ring: Ring, tp: TraceParams, prec: int, sample_budget: int) -> int:
    """Peak device bytes of a context stepping this geometry (rb_step_bytes)."""
    return int(load().rb_step_bytes(ctypes.byref(grid), ctypes.byref(ring), ctypes.byref(tp),
                                    int(prec), int(sample_budget)))


def workspace_bytes(grid: Grid, ring: Ring, tp: TraceParams, prec: int,
                    sample_budget: int) -> int:
    """Device bytes rb_reserve takes for this geometry (rb_workspace_bytes)."""
    return int(load().rb_workspace_bytes(ctypes.byref(grid), ctypes.byref(ring),
                                         ctypes.byref(tp), int(prec), int(sample_budget)))


@dataclasses.dataclass
class ScanStep:
    """Arguments of one scan's step in a batch (rb_scan_step)."""

    ctx: "Context"
    grid: Grid
    ring: Ring
    tp: TraceParams
    c: torch.Tensor
    smooth_w: int
    omegas: list
    d_omegas: list
    data: torch.Tensor
    tau: float
    mode: int = RB_RAY_BORN
    residual_norm: torch.Tensor | None = None


def frequency_step_batch(steps, prec: int = RB_BF16):
    """One frequency step of each scan (rb_frequency_step_batch); returns each scan's status
    (RB_OK, or RB_ENONFINITE for a scan whose step was rejected and left its model as it
    was). Raises if the batch could not be launched."""
    lib = load()
    n = len(steps)
    if not 1 <= n <= GROUP_MAX:
        raise ValueError(f"a batch holds 1..{GROUP_MAX} scans, got {n}")
    arr = (_ScanStep * n)()
    keep = []
    for i, s in enumerate(steps):
        _dev(s.c, torch.float64)
        _dev(s.data, torch.complex64)
        if s.residual_norm is not None:
            _dev(s.residual_norm, torch.float64)
        if len(s.omegas) != len(s.d_omegas) or s.data.shape[0] < len(s.omegas):
            raise ValueError(f"scan {i}: one spacing and one data slice per frequency")
        om = (ctypes.c_double * len(s.omegas))(*[float(o) for o in s.omegas])
        dom = (ctypes.c_double * len(s.d_omegas))(*[float(o) for o in s.d_omegas])
        keep += [om, dom]
        arr[i] = _ScanStep(s.ctx._h, ctypes.pointer(s.grid), ctypes.pointer(s.ring),
                           ctypes.pointer(s.tp), s.c.data_ptr(), int(s.smooth_w),
                           len(s.omegas), om, dom, s.data.data_ptr(), float(s.tau), int(s.mode),
                           s.residual_norm.data_ptr() if s.residual_norm is not None else None)
    status = (ctypes.c_int * n)()
    st = lib.rb_frequency_step_batch(arr, n, int(prec), status)
    out = [int(v) for v in status]
    if st != RB_OK and all(v == RB_OK for v in out):
        bad = next((s.ctx for s in steps if lib.rb_last_error(s.ctx._h)), steps[0].ctx)
        raise RayBornError(st, lib.rb_last_error(bad._h).decode())
    return out


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def _dev(t, dtype):
    if not t.is_cuda or t.dtype != dtype or not t.is_contiguous():
        raise TypeError(f"expected a contiguous {dtype} GPU tensor, got {t.dtype} on {t.device}")
    return t


@dataclasses.dataclass
class Tables:
    """Device tensors of rb_tables (grid tables [n][n_mask], receiver tables [n][n])."""

    T: torch.Tensor
    A: torch.Tensor
    ux: torch.Tensor
    uy: torch.Tensor
    flags: torch.Tensor
    rx_T: torch.Tensor
    rx_A: torch.Tensor
    rx_flags: torch.Tensor

    @classmethod
    def empty(cls, n, n_mask, device):
        f = dict(device=device)
        return cls(torch.empty(n, n_mask, dtype=torch.float64, **f),
                   torch.empty(n, n_mask, dtype=torch.float32, **f),
                   torch.empty(n, n_mask, dtype=torch.float32, **f),
                   torch.empty(n, n_mask, dtype=torch.float32, **f),
                   torch.empty(n, n_mask, dtype=torch.uint8, **f),
                   torch.empty(n, n, dtype=torch.float64, **f),
                   torch.empty(n, n, dtype=torch.float32, **f),
                   torch.empty(n, n, dtype=torch.uint8, **f))

    def struct(self):
        n, nm = self.T.shape
        return _Tables(n, nm, *(t.data_ptr() for t in (self.T, self.A, self.ux, self.uy,
                                                       self.flags, self.rx_T, self.rx_A,
                                                       self.rx_flags)))


_LP_DTYPE = {RB_BF16: torch.bfloat16, RB_F16: torch.float16, RB_F16X: torch.float16}


@dataclasses.dataclass
class Green:
    """Device tensors of rb_green.

    RB_F32: G complex64 [n][n_mask], H complex64 [3][n][n_mask].
    RB_BF16 / RB_F16: G planar [2][n][m_pad], H planar node-major [3][2][n_mask][n_pad]
    (pads: rounded up to 32), scales float32 [2][n] (per-row powers of two of G and H; the
    stored operands carry them). RB_F16X: as RB_F16 with H [2 (hi, lo)][3][2][n_mask][n_pad]."""

    G: torch.Tensor
    H: torch.Tensor
    prec: int = RB_F32
    scales: torch.Tensor | None = None

    @classmethod
    def empty(cls, n, n_mask, device, prec=RB_F32):
        if prec == RB_F32:
            return cls(torch.empty(n, n_mask, dtype=torch.complex64, device=device),
                       torch.empty(3, n, n_mask, dtype=torch.complex64, device=device), prec)
        dt = _LP_DTYPE[prec]
        n_pad = (n + 31) // 32 * 32
        m_pad = (n_mask + 31) // 32 * 32
        hshape = (3, 2, n_mask, n_pad) if prec != RB_F16X else (2, 3, 2, n_mask, n_pad)
        return cls(torch.empty(2, n, m_pad, dtype=dt, device=device),
                   torch.empty(*hshape, dtype=dt, device=device), prec,
                   torch.ones(2, n, dtype=torch.float32, device=device))

    @property
    def n(self):
        return self.G.shape[-2]

    @property
    def n_mask(self):
        return self.G.shape[-1] if self.prec == RB_F32 else self.H.shape[-2]

    def complex_G(self):
        """G as complex [n][n_mask] (float32 parts, row scales divided out), for checks."""
        if self.prec == RB_F32:
            return self.G
        m = self.n_mask
        s = self.scales[0][:, None]
        return torch.complex(self.G[0, :, :m].float() / s, self.G[1, :, :m].float() / s)

    def complex_H(self):
        """H, H u_x, H u_y as complex [3][n][n_mask] (row scales divided out), for checks."""
        if self.prec == RB_F32:
            return self.H
        n = self.n
        t = self.scales[1][None, :, None]
        H = self.H.float()
        if self.prec == RB_F16X:
            H = H[0] + H[1]   # high and low parts
        return torch.complex(H[:, 0, :, :n], H[:, 1, :, :n]).transpose(1, 2) / t

    def struct(self):
        return _Green(self.n, self.n_mask, self.prec, self.G.data_ptr(), self.H.data_ptr(),
                      self.scales.data_ptr() if self.scales is not None else None)


class Context:
    """One rb_ctx bound to a torch device and a stream (default: the current one)."""

    def __init__(self, device=None, stream: torch.cuda.Stream | None = None):
        if not torch.cuda.is_available():
            raise RuntimeError("raybornhf needs a GPU (torch.cuda.is_available() is False)")
        self.lib = load()
        self.device = torch.device(device if device is not None else "cuda:0")
        idx = self.device.index or 0
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        h = ctypes.c_void_p()
        st = self.lib.rb_create(ctypes.byref(h), idx, ctypes.c_void_p(self.stream.cuda_stream))
        if st != RB_OK:
            raise RayBornError(st, "rb_create failed")
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            self.lib.rb_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, st):
        if st != RB_OK:
            raise RayBornError(st, self.lib.rb_last_error(self._h).decode())

    def set_receiver_linking(self, max_iter: int, tol: float = 1e-8):
        """Receiver tables by secant ray linking (max_iter > 0) or fan interpolation (0)."""
        self._check(self.lib.rb_set_receiver_linking(self._h, int(max_iter), float(tol)))

    def reserve(self, grid: Grid, ring: Ring, tp: TraceParams, prec: int):
        """Allocate every workspace of this geometry now; later calls allocate nothing."""
        self._check(self.lib.rb_reserve(self._h, ctypes.byref(grid), ctypes.byref(ring),
                                        ctypes.byref(tp), int(prec)))

    def set_sample_budget(self, nbytes: int):
        """Bytes of ray samples one tracer launch may hold (rb_set_sample_budget)."""
        self._check(self.lib.rb_set_sample_budget(self._h, int(nbytes)))

    def autotune(self, grid: Grid, ring: Ring, prec: int) -> Tuning:
        """Time the forward's configurations for this shape and keep the fastest."""
        t = Tuning()
        self._check(self.lib.rb_autotune(self._h, ctypes.byref(grid), ctypes.byref(ring),
                                         int(prec), ctypes.byref(t)))
        return t

    def set_tuning(self, t: Tuning | dict | None):
        if isinstance(t, dict):
            t = Tuning(**{k: t[k] for k, _ in Tuning._fields_ if k in t})
        self._check(self.lib.rb_set_tuning(self._h, ctypes.byref(t) if t is not None else None))

    def get_tuning(self, n: int, n_mask: int, prec: int) -> Tuning | None:
        t = Tuning(n, n_mask, prec)
        return t if self.lib.rb_get_tuning(self._h, ctypes.byref(t)) == RB_OK else None

    def lost_nodes(self) -> int:
        """Mask nodes the last binning could not place (diagnostic; 0 normally)."""
        return int(self.lib.rb_trace_lost_nodes(self._h))

    def trace_samples(self) -> int:
        """Ray samples written by the last trace (the tracer's unit of work)."""
        return int(self.lib.rb_trace_samples(self._h))

    # measurement ------------------------------------------------------------------------
    def profile_enable(self, on: bool = True):
        self._check(self.lib.rb_profile_enable(self._h, int(on)))

    def profile_read(self):
        """{stage name: (total ms, launches)} since the last read (synchronizes)."""
        ms = (ctypes.c_double * N_STAGES)()
        cnt = (ctypes.c_int64 * N_STAGES)()
        self._check(self.lib.rb_profile_read(self._h, ms, cnt))
        return {self.lib.rb_stage_name(i).decode(): (ms[i], cnt[i]) for i in range(N_STAGES)}

    # entry points (same names as the C ABI) ---------------------------------------------
    def refractive_index(self, grid: Grid, c: torch.Tensor, c0: float, w: int) -> torch.Tensor:
        _dev(c, torch.float64)
        out = torch.empty(grid.ny, grid.nx, dtype=torch.float32, device=self.device)
        self._check(self.lib.rb_refractive_index(self._h, ctypes.byref(grid), _ptr(c), c0, w,
                                                 _ptr(out)))
        return out

    def lossy_maps(self, grid: Grid, c: torch.Tensor, alpha0: torch.Tensor, y: float,
                   c0: float, omega: float, w: int):
        """rb_lossy_maps: (n_w, a_w), float32 [ny][nx] each, of an absorbing medium at omega
        (alpha0: float64 [ny][nx] in Np (rad/s)^-y m^-1)."""
        _dev(c, torch.float64)
        _dev(alpha0, torch.float64)
        n_w = torch.empty(grid.ny, grid.nx, dtype=torch.float32, device=self.device)
        a_w = torch.empty_like(n_w)
        ab = _Absorption(_ptr(alpha0), float(y))
        self._check(self.lib.rb_lossy_maps(self._h, ctypes.byref(grid), _ptr(c), ctypes.byref(ab),
                                           c0, omega, w, _ptr(n_w), _ptr(a_w)))
        return n_w, a_w

    def trace_rays_lossy(self, grid: Grid, ring: Ring, tp: TraceParams, n_w: torch.Tensor,
                         a_w: torch.Tensor) -> Tables:
        _dev(n_w, torch.float32)
        _dev(a_w, torch.float32)
        tb = Tables.empty(ring.n, mask_count(grid), self.device)
        s = tb.struct()
        self._check(self.lib.rb_trace_rays_lossy(self._h, ctypes.byref(grid), ctypes.byref(ring),
                                                 ctypes.byref(tp), _ptr(n_w), _ptr(a_w),
                                                 ctypes.byref(s)))
        return tb

    def trace_rays(self, grid: Grid, ring: Ring, tp: TraceParams, n_s: torch.Tensor) -> Tables:
        _dev(n_s, torch.float32)
        tb = Tables.empty(ring.n, mask_count(grid), self.device)
        s = tb.struct()
        self._check(self.lib.rb_trace_rays(self._h, ctypes.byref(grid), ctypes.byref(ring),
                                           ctypes.byref(tp), _ptr(n_s), ctypes.byref(s)))
        return tb

    def build_green(self, tb: Tables, omega: float, c0: float, out: Green | None = None,
                    prec: int = RB_F32) -> Green:
        n, nm = tb.T.shape
        gr = out if out is not None else Green.empty(n, nm, self.device, prec)
        s, g = tb.struct(), gr.struct()
        self._check(self.lib.rb_build_green(self._h, ctypes.byref(s), omega, c0, ctypes.byref(g)))
        return gr

    def born_forward(self, gr: Green, w: torch.Tensor | None, delta: torch.Tensor | None,
                     out: torch.Tensor | None = None) -> torch.Tensor:
        """w = delta = None: the operands already carry sqrt(w delta)."""
        if w is not None or delta is not None:
            _dev(w, torch.complex64)
            _dev(delta, torch.float32)
        n = gr.n
        d = out if out is not None else torch.empty(n, n, dtype=torch.complex64, device=self.device)
        g = gr.struct()
        self._check(self.lib.rb_born_forward(self._h, ctypes.byref(g), _ptr(w), _ptr(delta),
                                             _ptr(d)))
        return d

    def born_adjoint(self, gr: Green, w: torch.Tensor, R: torch.Tensor) -> torch.Tensor:
        _dev(w, torch.complex64)
        _dev(R, torch.complex64)
        out = torch.empty(gr.n_mask, dtype=torch.float32, device=self.device)
        g = gr.struct()
        self._check(self.lib.rb_born_adjoint(self._h, ctypes.byref(g), _ptr(w), _ptr(R),
                                             _ptr(out)))
        return out

    def residual(self, tb: Tables, omega: float, c0: float, data: torch.Tensor,
                 d_born: torch.Tensor | None = None) -> torch.Tensor:
        _dev(data, torch.complex64)
        if d_born is not None:
            _dev(d_born, torch.complex64)
        R = torch.empty_like(data)
        s = tb.struct()
        self._check(self.lib.rb_residual(self._h, ctypes.byref(s), omega, c0, _ptr(d_born),
                                         _ptr(data), _ptr(R)))
        return R

    def backproject(self, gr: Green, R: torch.Tensor, c_mask: torch.Tensor, omega: float,
                    d_omega: float, out: torch.Tensor | None = None,
                    accumulate: bool = False) -> torch.Tensor:
        _dev(R, torch.complex64)
        _dev(c_mask, torch.float64)
        dm = out if out is not None else torch.empty(gr.n_mask, dtype=torch.float32,
                                                     device=self.device)
        g = gr.struct()
        self._check(self.lib.rb_backproject(self._h, ctypes.byref(g), _ptr(R), _ptr(c_mask),
                                            omega, d_omega, _ptr(dm), int(accumulate)))
        return dm

    def backproject_lossy(self, gr: Green, R: torch.Tensor, c_mask: torch.Tensor,
                          alpha0_mask: torch.Tensor, y: float, omega: float, d_omega: float,
                          out: torch.Tensor | None = None,
                          accumulate: bool = False) -> torch.Tensor:
        _dev(R, torch.complex64)
        _dev(c_mask, torch.float64)
        _dev(alpha0_mask, torch.float64)
        dm = out if out is not None else torch.empty(gr.n_mask, dtype=torch.float32,
                                                     device=self.device)
        g = gr.struct()
        self._check(self.lib.rb_backproject_lossy(self._h, ctypes.byref(g), _ptr(R),
                                                  _ptr(c_mask), _ptr(alpha0_mask), float(y),
                                                  omega, d_omega, _ptr(dm), int(accumulate)))
        return dm

    def backproject_noalloc(self, gr: Green, R: torch.Tensor, c_mask: torch.Tensor,
                            omega: float, d_omega: float, out: torch.Tensor,
                            accumulate: bool = False) -> torch.Tensor:
        """rb_backproject_noalloc: the back-projection into the caller's `out`, with the
        library's fixed scratch (no device allocation by the library)."""
        _dev(R, torch.complex64)
        _dev(c_mask, torch.float64)
        _dev(out, torch.float32)
        g = gr.struct()
        self._check(self.lib.rb_backproject_noalloc(self._h, ctypes.byref(g), _ptr(R),
                                                    _ptr(c_mask), omega, d_omega, _ptr(out),
                                                    int(accumulate)))
        return out

    def frequency_step(self, grid: Grid, ring: Ring, tp: TraceParams, c: torch.Tensor,
                       smooth_w: int, omegas, d_omegas, data: torch.Tensor, tau: float,
                       mode: int = RB_RAY_BORN, residual_norm: torch.Tensor | None = None,
                       prec: int = RB_F32, report: torch.Tensor | None = None):
        """Updates c (float64 [ny][nx], on the GPU) in place. report (uint8 GPU tensor of
        REPORT_BYTES, optional): the step's status goes there and nothing waits for the
        stream (decode it with decode_report)."""
        _dev(c, torch.float64)
        _dev(data, torch.complex64)
        if report is not None:
            _dev(report, torch.uint8)
            if report.numel() < REPORT_BYTES or report.data_ptr() % 8:
                raise ValueError("report needs REPORT_BYTES bytes, 8-byte aligned")
        k = len(omegas)
        om = (ctypes.c_double * k)(*omegas)
        dom = (ctypes.c_double * k)(*d_omegas)
        self._check(self.lib.rb_frequency_step(
            self._h, ctypes.byref(grid), ctypes.byref(ring), ctypes.byref(tp), _ptr(c),
            int(smooth_w), k, om, dom, _ptr(data), float(tau), int(mode), int(prec),
            _ptr(residual_norm), _ptr(report)))
        return c

    def frequency_step_lossy(self, grid: Grid, ring: Ring, tp: TraceParams, c: torch.Tensor,
                             alpha0: torch.Tensor, y: float, smooth_w: int, omegas, d_omegas,
                             data: torch.Tensor, tau: float, mode: int = RB_RAY_BORN,
                             residual_norm: torch.Tensor | None = None, prec: int = RB_F32,
                             report: torch.Tensor | None = None):
        """rb_frequency_step_lossy: frequency_step in an absorbing, dispersive medium
        (alpha0: float64 [ny][nx], Np (rad/s)^-y m^-1; y: power-law exponent)."""
        _dev(c, torch.float64)
        _dev(alpha0, torch.float64)
        _dev(data, torch.complex64)
        if report is not None:
            _dev(report, torch.uint8)
            if report.numel() < REPORT_BYTES or report.data_ptr() % 8:
                raise ValueError("report needs REPORT_BYTES bytes, 8-byte aligned")
        k = len(omegas)
        om = (ctypes.c_double * k)(*omegas)
        dom = (ctypes.c_double * k)(*d_omegas)
        ab = _Absorption(_ptr(alpha0), float(y))
        self._check(self.lib.rb_frequency_step_lossy(
            self._h, ctypes.byref(grid), ctypes.byref(ring), ctypes.byref(tp), _ptr(c),
            ctypes.byref(ab), int(smooth_w), k, om, dom, _ptr(data), float(tau), int(mode),
            int(prec), _ptr(residual_norm), _ptr(report)))
        return c

    def gauss_newton_step(self, grid: Grid, ring: Ring, tp: TraceParams, c: torch.Tensor,
                          smooth_w: int, omegas, data: torch.Tensor, tau: float, n_inner: int,
                          model: int = RB_GREEN_RAY, prec: int = RB_F32,
                          residual_norm: torch.Tensor | None = None,
                          cg_norms: torch.Tensor | None = None,
                          report: torch.Tensor | None = None):
        """rb_gauss_newton_step: one Gauss-Newton update of c (float64 [ny][nx], on the GPU)
        in place; model RB_GREEN_RAY (Hessian-based ray-Born) or RB_GREEN_WATER (prototype
        Born). cg_norms: float64 [n_inner + 1] receiving |r_k| of the CG iterates."""
        _dev(c, torch.float64)
        _dev(data, torch.complex64)
        for t in (residual_norm, cg_norms):
            if t is not None:
                _dev(t, torch.float64)
        if cg_norms is not None and cg_norms.numel() < n_inner + 1:
            raise ValueError("cg_norms needs n_inner + 1 entries")
        if report is not None:
            _dev(report, torch.uint8)
        k = len(omegas)
        om = (ctypes.c_double * k)(*[float(o) for o in omegas])
        self._check(self.lib.rb_gauss_newton_step(
            self._h, ctypes.byref(grid), ctypes.byref(ring), ctypes.byref(tp), _ptr(c),
            int(smooth_w), k, om, _ptr(data), float(tau), int(n_inner), int(model), int(prec),
            _ptr(residual_norm), _ptr(cg_norms), _ptr(report)))
        return c

    def frequency_sweep(self, grid: Grid, ring: Ring, tp: TraceParams, c: torch.Tensor,
                        smooth_ws, omega_sets, d_omega_sets, data: torch.Tensor, tau: float,
                        mode: int = RB_RAY_BORN, prec: int = RB_F32, use_graph: bool = False,
                        residual_norms: torch.Tensor | None = None):
        """Steps k = 0.. of the frequency continuation in one call (no host synchronisation
        between steps; one graph launch with use_graph). omega_sets[k], d_omega_sets[k]: the
        frequencies of step k; data: complex64 [total frequencies][n][n] in the same order.
        Updates c (float64 [ny][nx], on the GPU) in place."""
        _dev(c, torch.float64)
        _dev(data, torch.complex64)
        n = len(omega_sets)
        if len(smooth_ws) != n or len(d_omega_sets) != n:
            raise ValueError("one window, frequency set and spacing set per step")
        flat = [float(o) for s in omega_sets for o in s]
        dflat = [float(o) for s in d_omega_sets for o in s]
        if data.shape[0] != len(flat):
            raise ValueError(f"data holds {data.shape[0]} frequencies, the steps use {len(flat)}")
        if residual_norms is not None:
            _dev(residual_norms, torch.float64)
        sw = (ctypes.c_int32 * n)(*[int(w) for w in smooth_ws])
        no = (ctypes.c_int32 * n)(*[len(s) for s in omega_sets])
        om = (ctypes.c_double * len(flat))(*flat)
        dom = (ctypes.c_double * len(dflat))(*dflat)
        self._check(self.lib.rb_frequency_sweep(
            self._h, ctypes.byref(grid), ctypes.byref(ring), ctypes.byref(tp), _ptr(c), n, sw,
            no, om, dom, _ptr(data), float(tau), int(mode), int(prec), int(bool(use_graph)),
            _ptr(residual_norms)))
        return c
