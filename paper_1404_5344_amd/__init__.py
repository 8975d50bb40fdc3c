"""Python binding of the MI355X FoE + iPiano despeckling library (C ABI in include/foe.h).

Argument marshalling only: every step of the method runs in the HIP library
``_lib/libfoe.so``.  PyTorch supplies device memory and the HIP stream.  There
is no CPU fallback: if the library is missing, importing the binding raises.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "_lib", "libfoe.so")
ABI_VERSION = 2   # FOE_ABI_VERSION of include/foe.h that the structures below mirror

OK, EINVAL, ENOMEM, EDEVICE, ELINESEARCH, ENONFINITE, EINPUT = 0, 1, 2, 3, 4, 5, 6
COMBINED, LOG, IDIV = 0, 1, 2
SYMMETRIC, ZERO, PERIODIC = 0, 1, 2
BACKTRACK, FIXED = 0, 1
FP32, BF16 = 0, 1
ENGINE_AUTO, ENGINE_VALU, ENGINE_MFMA, ENGINE_MFMA_SPLIT = 0, 1, 2, 3
STATS_COLS = 8
STATS_NAMES = ("F", "G", "L", "alpha", "trials", "s1", "s2", "m")


class FoeError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{status_str(status)}: {msg}")
        self.status = status


class Params(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int32) for n in (
        "height", "width", "num_filters", "ksize", "model", "boundary", "precision", "step_mode", "looks",
        "max_iters", "max_backtracks", "newton_iters", "engine", "fusion", "prox_method")] + \
        [(n, ctypes.c_double) for n in ("lambda1", "lambda2", "beta", "alpha_fixed", "L0", "eta_up", "eta_down")]


class Summary(ctypes.Structure):
    _fields_ = [("iters_done", ctypes.c_int32), ("total_trials", ctypes.c_int32), ("H", ctypes.c_double),
                ("F", ctypes.c_double), ("G", ctypes.c_double), ("L", ctypes.c_double), ("alpha", ctypes.c_double)]

    def as_dict(self) -> dict:
        return {n: getattr(self, n) for n, _ in self._fields_}


_VP = ctypes.c_void_p
_DP = ctypes.POINTER(ctypes.c_double)


def _load():
    # torch ships its own HIP runtime under the same soname (libamdhip64.so.7).  Loading torch
    # first makes the library bind to that runtime, so device pointers and streams of torch and
    # of the library belong to one HIP runtime in the process.
    import torch  # noqa: F401
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"HIP library not built: {LIB_PATH} (run paper_1404_5344_amd/build.py)")
    L = ctypes.CDLL(LIB_PATH)
    L.foe_default_params.argtypes = [ctypes.POINTER(Params)]
    L.foe_default_params.restype = None
    L.foe_create.argtypes = [ctypes.POINTER(Params), _VP, _VP, _VP, ctypes.POINTER(_VP)]
    L.foe_destroy.argtypes = [_VP]
    L.foe_solve.argtypes = [_VP, _VP, _VP, _VP, ctypes.POINTER(Summary), _DP]
    L.foe_solve_from.argtypes = [_VP, _VP, _VP, _VP, _DP, ctypes.c_int32, ctypes.POINTER(Summary), _DP]
    L.foe_eval_gradient.argtypes = [_VP, _VP, _VP]
    L.foe_eval_energy.argtypes = [_VP, _VP, _VP, _DP, _DP]
    L.foe_eval_prox.argtypes = [_VP, _VP, _VP, ctypes.c_double, _VP]
    L.foe_step.argtypes = [_VP, _VP, _VP, _VP, ctypes.c_double, _VP, _DP]
    L.foe_last_timing.argtypes = [_VP, _DP, ctypes.POINTER(ctypes.c_int32)]
    L.foe_batch_latency.argtypes = [_VP, _DP]
    L.foe_real_sar_params.argtypes = [ctypes.POINTER(Params)]
    L.foe_profile_trial.argtypes = [_VP, ctypes.c_int32, _DP]
    _IP = ctypes.POINTER(ctypes.c_int32)
    L.foe_batch_create.argtypes = [ctypes.POINTER(Params), ctypes.c_int32, _IP, _IP, _DP, _DP, _IP, _VP, _VP, _VP,
                                   ctypes.POINTER(_VP)]
    L.foe_batch_layout.argtypes = [_VP, _IP, ctypes.POINTER(ctypes.c_int64)]
    L.foe_batch_solve.argtypes = [_VP, _VP, _VP, _VP, ctypes.POINTER(Summary), _DP]
    L.foe_autotune.argtypes = [_VP, _VP, ctypes.c_int32, _IP]
    L.foe_set_tile_config.argtypes = [_VP, ctypes.c_int32]
    L.foe_solve_noalloc.argtypes = [ctypes.POINTER(Params), _VP, _VP, _VP, _VP, _VP, _VP, ctypes.POINTER(Summary), _DP]
    L.foe_cnn_num_params.restype = ctypes.c_int64
    L.foe_cnn_create.argtypes = [_VP, _VP, ctypes.POINTER(_VP)]
    L.foe_cnn_destroy.argtypes = [_VP]
    L.foe_cnn_get_params.argtypes = [_VP, _VP, _VP]
    L.foe_cnn_infer.argtypes = [_VP, _VP, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, _VP]
    L.foe_cnn_loss_grad.argtypes = [_VP, _VP, _VP, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, _DP, _VP]
    L.foe_cnn_train_step.argtypes = [_VP, _VP, _VP, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_double,
                                     _DP]
    L.foe_ssim.argtypes = [_VP, _VP, ctypes.c_int32, ctypes.c_int32, ctypes.c_double, _VP, _DP]
    L.foe_ssim.restype = ctypes.c_int
    L.foe_status_str.argtypes = [ctypes.c_int]
    L.foe_status_str.restype = ctypes.c_char_p
    L.foe_last_error.argtypes = []
    L.foe_last_error.restype = ctypes.c_char_p
    L.foe_abi_version.restype = ctypes.c_int32
    for name in ("foe_create", "foe_destroy", "foe_solve", "foe_solve_from", "foe_eval_gradient", "foe_eval_energy",
                 "foe_eval_prox", "foe_step", "foe_last_timing", "foe_profile_trial", "foe_batch_create",
                 "foe_batch_layout", "foe_batch_solve", "foe_autotune", "foe_solve_noalloc", "foe_set_tile_config", "foe_cnn_create",
                 "foe_cnn_destroy", "foe_cnn_get_params", "foe_cnn_infer", "foe_cnn_loss_grad", "foe_cnn_train_step",
                 "foe_batch_latency", "foe_real_sar_params"):
        getattr(L, name).restype = ctypes.c_int
    if L.foe_abi_version() != ABI_VERSION:
        raise ImportError(f"{LIB_PATH} has ABI version {L.foe_abi_version()}, this binding expects {ABI_VERSION}")
    return L


lib = _load()


def status_str(st: int) -> str:
    return lib.foe_status_str(int(st)).decode()


def _check(st: int, allow=(OK,)):
    if st not in allow:
        raise FoeError(st, lib.foe_last_error().decode())
    return st


def real_sar_params(height: int, width: int, **kw) -> Params:
    """The parameters of the real-SAR experiment (Sec. III-C: L = 5, lambda = (50, 0.15)), see foe_real_sar_params."""
    p = Params()
    _check(lib.foe_real_sar_params(ctypes.byref(p)))
    p.height, p.width = int(height), int(width)
    for k, v in kw.items():
        if not hasattr(p, k):
            raise KeyError(k)
        setattr(p, k, v)
    return p


def default_params(height: int, width: int, **kw) -> Params:
    p = Params()
    lib.foe_default_params(ctypes.byref(p))
    p.height, p.width = int(height), int(width)
    for k, v in kw.items():
        if not hasattr(p, k):
            raise KeyError(k)
        setattr(p, k, v)
    return p


def _torch():
    import torch
    return torch


def _dev_ptr(t, shape=None, name="tensor"):
    torch = _torch()
    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != torch.float32 or not t.is_contiguous():
        raise TypeError(f"{name} must be a contiguous float32 CUDA tensor")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
    return _VP(t.data_ptr())


@dataclass
class SolveResult:
    u: object            # torch tensor [H, W]
    summary: dict
    stats: np.ndarray    # [iters_done, 8]
    status: int


class Solver:
    """One image size and filter bank; owns device scratch.  All tensors are float32 CUDA [H, W]."""

    def __init__(self, params: Params, filters, weights, stream=None):
        torch = _torch()
        self.params = params
        self.shape = (params.height, params.width)
        k = np.ascontiguousarray(np.asarray(filters, dtype=np.float32).reshape(-1, 7, 7))
        th = np.ascontiguousarray(np.asarray(weights, dtype=np.float32).reshape(-1))
        if k.shape[0] != params.num_filters or th.shape[0] != params.num_filters:
            raise ValueError("filters/weights do not match num_filters")
        self._k, self._th = k, th
        if stream is None:
            stream = torch.cuda.current_stream()
        self.stream = stream
        h = _VP()
        _check(lib.foe_create(ctypes.byref(params), k.ctypes.data_as(_VP), th.ctypes.data_as(_VP),
                              _VP(stream.cuda_stream), ctypes.byref(h)))
        self._h = h

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            lib.foe_destroy(self._h)
            self._h = _VP()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def _sync_in(self):
        # inputs produced on torch's current stream must be complete before the solver stream reads them
        torch = _torch()
        if self.stream != torch.cuda.current_stream():
            self.stream.wait_stream(torch.cuda.current_stream())

    def solve(self, f, init=None, out=None, allow_failure=False) -> SolveResult:
        torch = _torch()
        self._sync_in()
        if out is None:
            out = torch.empty(self.shape, dtype=torch.float32, device=f.device)
        s = Summary()
        stats = np.zeros((max(self.params.max_iters, 1), STATS_COLS))
        st = lib.foe_solve(self._h, _dev_ptr(f, self.shape, "f"),
                           _dev_ptr(init, self.shape, "init") if init is not None else None,
                           _dev_ptr(out, self.shape, "out"), ctypes.byref(s), stats.ctypes.data_as(_DP))
        _check(st, (OK, ELINESEARCH, ENONFINITE) if allow_failure else (OK,))
        return SolveResult(out, s.as_dict(), stats[:s.iters_done].copy(), st)

    def solve_from(self, f, x_cur, x_prev, L: float, iters: int, allow_failure=False):
        """Advance the state (x_cur, x_prev, L) in place by `iters` iterations; returns (L, summary, stats)."""
        self._sync_in()
        Lc = ctypes.c_double(L)
        s = Summary()
        stats = np.zeros((max(iters, 1), STATS_COLS))
        st = lib.foe_solve_from(self._h, _dev_ptr(f, self.shape, "f"), _dev_ptr(x_cur, self.shape, "x_cur"),
                                _dev_ptr(x_prev, self.shape, "x_prev"), ctypes.byref(Lc), int(iters), ctypes.byref(s),
                                stats.ctypes.data_as(_DP))
        _check(st, (OK, ELINESEARCH, ENONFINITE) if allow_failure else (OK,))
        return Lc.value, s.as_dict(), stats[:s.iters_done].copy()

    def eval_gradient(self, x):
        torch = _torch()
        self._sync_in()
        g = torch.empty(self.shape, dtype=torch.float32, device=x.device)
        _check(lib.foe_eval_gradient(self._h, _dev_ptr(x, self.shape, "x"), _dev_ptr(g)))
        return g

    def eval_energy(self, x, f):
        self._sync_in()
        F, G = ctypes.c_double(), ctypes.c_double()
        _check(lib.foe_eval_energy(self._h, _dev_ptr(x, self.shape, "x"), _dev_ptr(f, self.shape, "f"),
                                   ctypes.byref(F), ctypes.byref(G)))
        return F.value, G.value

    def eval_prox(self, xhat, f, tau: float):
        torch = _torch()
        self._sync_in()
        out = torch.empty(self.shape, dtype=torch.float32, device=xhat.device)
        _check(lib.foe_eval_prox(self._h, _dev_ptr(xhat, self.shape, "xhat"), _dev_ptr(f, self.shape, "f"),
                                 float(tau), _dev_ptr(out)))
        return out

    def step(self, f, x, xprev, L: float):
        torch = _torch()
        self._sync_in()
        out = torch.empty(self.shape, dtype=torch.float32, device=x.device)
        info = np.zeros(4)
        _check(lib.foe_step(self._h, _dev_ptr(f, self.shape, "f"), _dev_ptr(x, self.shape, "x"),
                            _dev_ptr(xprev, self.shape, "xprev"), float(L), _dev_ptr(out), info.ctypes.data_as(_DP)))
        return out, dict(F=info[0], G=info[1], s1=info[2], s2=info[3])

    def profile_trial(self, reps: int = 20) -> float:
        """Mean duration (ms) of one fused trial launch, from per-launch HIP event pairs."""
        ms = ctypes.c_double()
        _check(lib.foe_profile_trial(self._h, int(reps), ctypes.byref(ms)))
        return ms.value

    def autotune(self, f, reps: int = 3) -> int:
        """Pick the fastest tile configuration for this solver's images (see foe_autotune)."""
        self._sync_in()
        c = ctypes.c_int32(-1)
        _check(lib.foe_autotune(self._h, _dev_ptr(f, None, "f"), int(reps), ctypes.byref(c)))
        return c.value

    def set_tile_config(self, cfg: int):
        _check(lib.foe_set_tile_config(self._h, int(cfg)))

    def last_timing(self):
        ms = ctypes.c_double()
        n = ctypes.c_int32()
        _check(lib.foe_last_timing(self._h, ctypes.byref(ms), ctypes.byref(n)))
        return ms.value, n.value

    def latency(self) -> np.ndarray:
        """Per-image latency (ms) of the last solve from device timestamps (see foe_batch_latency)."""
        out = np.zeros(getattr(self, "n_images", 1))
        _check(lib.foe_batch_latency(self._h, out.ctypes.data_as(_DP)))
        return out


def solve_noalloc(params: Params, filters, weights, f, init=None, out=None, stream=None,
                  allow_failure=False) -> SolveResult:
    """One solve through the allocation-free entry point (see foe_solve_noalloc): no solver handle, the
    library's static device workspace in place of per-solver buffers.  out (optional) receives u."""
    torch = _torch()
    shape = (params.height, params.width)
    k = np.ascontiguousarray(np.asarray(filters, dtype=np.float32).reshape(-1, 7, 7))
    th = np.ascontiguousarray(np.asarray(weights, dtype=np.float32).reshape(-1))
    if k.shape[0] != params.num_filters or th.shape[0] != params.num_filters:
        raise ValueError("filters/weights do not match num_filters")
    if stream is None:
        stream = torch.cuda.current_stream()
    elif stream != torch.cuda.current_stream():
        stream.wait_stream(torch.cuda.current_stream())
    if out is None:
        out = torch.empty(shape, dtype=torch.float32, device=f.device)
    s = Summary()
    stats = np.zeros((max(params.max_iters, 1), STATS_COLS))
    st = lib.foe_solve_noalloc(ctypes.byref(params), k.ctypes.data_as(_VP), th.ctypes.data_as(_VP),
                               _VP(stream.cuda_stream), _dev_ptr(f, shape, "f"),
                               _dev_ptr(init, shape, "init") if init is not None else None,
                               _dev_ptr(out, shape, "out"), ctypes.byref(s), stats.ctypes.data_as(_DP))
    _check(st, (OK, ELINESEARCH, ENONFINITE) if allow_failure else (OK,))
    return SolveResult(out, s.as_dict(), stats[:s.iters_done].copy(), st)


class BatchSolver(Solver):
    """Many images of uneven sizes solved together; images are packed planes (see foe.h)."""

    def __init__(self, params: Params, sizes, looks, filters, weights, lambda1=None, lambda2=None, stream=None):
        torch = _torch()
        self.params = params
        n = len(sizes)
        self.sizes = [(int(h), int(w)) for h, w in sizes]
        k = np.ascontiguousarray(np.asarray(filters, dtype=np.float32).reshape(-1, 7, 7))
        th = np.ascontiguousarray(np.asarray(weights, dtype=np.float32).reshape(-1))
        self._k, self._th = k, th
        Hs = (ctypes.c_int32 * n)(*[h for h, _ in self.sizes])
        Ws = (ctypes.c_int32 * n)(*[w for _, w in self.sizes])
        Ls = (ctypes.c_int32 * n)(*[int(x) for x in looks])
        l1 = (ctypes.c_double * n)(*lambda1) if lambda1 is not None else None
        l2 = (ctypes.c_double * n)(*lambda2) if lambda2 is not None else None
        if stream is None:
            stream = torch.cuda.current_stream()
        self.stream = stream
        h = _VP()
        _check(lib.foe_batch_create(ctypes.byref(params), n, Hs, Ws, l1, l2, Ls, k.ctypes.data_as(_VP),
                                    th.ctypes.data_as(_VP), _VP(stream.cuda_stream), ctypes.byref(h)))
        self._h = h
        self.n_images = n
        offs = (ctypes.c_int64 * (n + 1))()
        _check(lib.foe_batch_layout(self._h, None, offs))
        self.offsets = [int(o) for o in offs]
        self.shape = (self.offsets[-1],)

    def solve_from(self, f_packed, x_cur, x_prev, L, iters: int, allow_failure=False):
        """Advance every image's state (packed x_cur, x_prev; per-image L list) in place by `iters`
        iterations; returns (L list, summaries, status)."""
        self._sync_in()
        n = self.n_images
        Lc = (ctypes.c_double * n)(*[float(v) for v in L])
        sums = (Summary * n)()
        st = lib.foe_solve_from(self._h, _dev_ptr(f_packed, self.shape, "f"), _dev_ptr(x_cur, self.shape, "x_cur"),
                                _dev_ptr(x_prev, self.shape, "x_prev"), Lc, int(iters), sums, None)
        _check(st, (OK, ELINESEARCH, ENONFINITE) if allow_failure else (OK,))
        return [Lc[i] for i in range(n)], [sums[i].as_dict() for i in range(n)], st

    def pack(self, images):
        torch = _torch()
        return torch.cat([torch.as_tensor(im, dtype=torch.float32).reshape(-1) for im in images]).contiguous()

    def unpack(self, packed):
        return [packed[self.offsets[i]:self.offsets[i + 1]].reshape(self.sizes[i]) for i in range(self.n_images)]

    def solve(self, f_packed, init=None, out=None, allow_failure=False):
        torch = _torch()
        self._sync_in()
        if out is None:
            out = torch.empty_like(f_packed)
        n = self.n_images
        sums = (Summary * n)()
        rows = max(self.params.max_iters, 1)
        stats = np.zeros((n, rows, STATS_COLS))
        st = lib.foe_batch_solve(self._h, _dev_ptr(f_packed, self.shape, "f"),
                                 _dev_ptr(init, self.shape, "init") if init is not None else None,
                                 _dev_ptr(out, self.shape, "out"), sums, stats.ctypes.data_as(_DP))
        _check(st, (OK, ELINESEARCH, ENONFINITE) if allow_failure else (OK,))
        summaries = [sums[i].as_dict() for i in range(n)]
        return out, summaries, [stats[i, :summaries[i]["iters_done"]].copy() for i in range(n)], st


CNN_LAYERS = [(1, 32), (32, 32), (32, 32), (32, 32), (32, 32), (32, 1)]   # (in, out) channels, 3x3 taps


def cnn_num_params() -> int:
    return int(lib.foe_cnn_num_params())


def cnn_init_params(seed: int) -> np.ndarray:
    """He-normal weights (std sqrt(2 / (9 c_in))), zero biases; the last layer is scaled by 0.1
    so that the untrained network starts near w0 = log f."""
    rng = np.random.Generator(np.random.PCG64(seed))
    parts = []
    for l, (ci, co) in enumerate(CNN_LAYERS):
        std = np.sqrt(2.0 / (9 * ci)) * (0.1 if l == len(CNN_LAYERS) - 1 else 1.0)
        parts += [rng.standard_normal(co * ci * 9) * std, np.zeros(co)]
    return np.concatenate(parts).astype(np.float32)


class WarmStartNet:
    """The warm-start network on the GPU.  Batches are float32 CUDA tensors [n, H, W]."""

    def __init__(self, params, stream=None):
        torch = _torch()
        p = np.ascontiguousarray(np.asarray(params, dtype=np.float32).reshape(-1))
        if p.size != cnn_num_params():
            raise ValueError(f"expected {cnn_num_params()} parameters, got {p.size}")
        if stream is None:
            stream = torch.cuda.current_stream()
        self.stream = stream
        h = _VP()
        _check(lib.foe_cnn_create(p.ctypes.data_as(_VP), _VP(stream.cuda_stream), ctypes.byref(h)))
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            lib.foe_cnn_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _sync_in(self):
        torch = _torch()
        if self.stream != torch.cuda.current_stream():
            self.stream.wait_stream(torch.cuda.current_stream())

    def params(self):
        """(FP32 master parameters, their BF16 rounding) as NumPy float32 arrays."""
        m = np.zeros(cnn_num_params(), np.float32)
        q = np.zeros(cnn_num_params(), np.float32)
        _check(lib.foe_cnn_get_params(self._h, m.ctypes.data_as(_VP), q.ctypes.data_as(_VP)))
        return m, q

    def infer(self, f, out=None):
        torch = _torch()
        self._sync_in()
        n, H, W = f.shape
        if out is None:
            out = torch.empty_like(f)
        _check(lib.foe_cnn_infer(self._h, _dev_ptr(f, None, "f"), n, H, W, _dev_ptr(out, f.shape, "out")))
        return out

    def loss_grad(self, f, u_target):
        self._sync_in()
        n, H, W = f.shape
        loss = ctypes.c_double()
        g = np.zeros(cnn_num_params(), np.float32)
        _check(lib.foe_cnn_loss_grad(self._h, _dev_ptr(f, None, "f"), _dev_ptr(u_target, f.shape, "u_target"), n, H,
                                     W, ctypes.byref(loss), g.ctypes.data_as(_VP)))
        return loss.value, g

    def train_step(self, f, u_target, lr):
        self._sync_in()
        n, H, W = f.shape
        loss = ctypes.c_double()
        _check(lib.foe_cnn_train_step(self._h, _dev_ptr(f, None, "f"), _dev_ptr(u_target, f.shape, "u_target"), n,
                                      H, W, float(lr), ctypes.byref(loss)))
        return loss.value


def ssim(u, ref, peak: float = 255.0, stream=None) -> float:
    """Mean SSIM of u against ref (float32 CUDA tensors [H, W]) on the GPU (see foe_ssim)."""
    torch = _torch()
    if stream is None:
        stream = torch.cuda.current_stream()
    H, W = u.shape
    out = ctypes.c_double()
    _check(lib.foe_ssim(_dev_ptr(u, None, "u"), _dev_ptr(ref, (H, W), "ref"), H, W, float(peak),
                        _VP(stream.cuda_stream), ctypes.byref(out)))
    return out.value
