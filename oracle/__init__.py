"""FP64 CPU oracle of the FoE + iPiano despeckling model -- TEST INFRASTRUCTURE.

Only ``tests/``, ``__graft_entry__.smoke()`` and the benchmark's CPU-baseline
leg may import this package.  It shares no code with the HIP library: the C
file ``foe_oracle.c`` is compiled here with gcc, and ``dense.py`` is an
independent NumPy brute force built from explicit N x N matrices.

Every function takes float64 NumPy arrays (inputs that the GPU received as
float32 are promoted before the call) and returns float64.

Models (Sec. II-B, II-C and III-A of the paper):
  COMBINED  eq. (newmodel):  F(w) = E_FoE(e^w),
            G(w) = lam1/2 (2w + f^2 e^{-2w}) + lam2/2 (e^{2w} - 2 f^2 w), summed over pixels
  LOG       eq. (original):  COMBINED with lam2 = 0
  IDIV      eq. (variant):   F(u) = E_FoE(u), G(u) = lam/2 <u^2 - 2 f^2 log u, 1>, lam = lam1
Boundary maps: SYMMETRIC (half-sample), ZERO, PERIODIC (the paper is silent).
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

from . import build as _build

COMBINED, LOG, IDIV = 0, 1, 2
SYMMETRIC, ZERO, PERIODIC = 0, 1, 2
BACKTRACK, FIXED = 0, 1
OK, EINVAL, ENOMEM, ELINESEARCH, ENONFINITE, EINPUT = 0, 1, 2, 4, 5, 6

_lib = None


class _Params(ctypes.Structure):
    _fields_ = [("model", ctypes.c_int32), ("boundary", ctypes.c_int32), ("step_mode", ctypes.c_int32),
                ("max_backtracks", ctypes.c_int32), ("lam1", ctypes.c_double), ("lam2", ctypes.c_double),
                ("beta", ctypes.c_double), ("alpha_fixed", ctypes.c_double), ("eta_up", ctypes.c_double),
                ("eta_down", ctypes.c_double)]


@dataclass
class Params:
    model: int = COMBINED
    boundary: int = SYMMETRIC
    lam1: float = 160.0
    lam2: float = 0.004
    beta: float = 0.8
    step_mode: int = BACKTRACK
    alpha_fixed: float = 0.0
    eta_up: float = 2.0
    eta_down: float = 1.0
    max_backtracks: int = 40

    def c(self) -> _Params:
        return _Params(self.model, self.boundary, self.step_mode, self.max_backtracks, self.lam1, self.lam2,
                       self.beta, self.alpha_fixed, self.eta_up, self.eta_down)


_D = ctypes.POINTER(ctypes.c_double)
_I = ctypes.c_int
_L = ctypes.c_long


def lib():
    global _lib
    if _lib is None:
        path = _build.LIB
        if not os.path.exists(path):
            _build.build()
        L = ctypes.CDLL(path)
        L.ora_forward.argtypes = [_D, _I, _I, _D, _I, _D]
        L.ora_adjoint.argtypes = [_D, _I, _I, _D, _I, _D]
        L.ora_adjoint.restype = _I
        L.ora_energy_F.argtypes = [_D, _I, _I, _D, _D, _I, _I, _I]
        L.ora_energy_F.restype = ctypes.c_double
        L.ora_energy_G.argtypes = [_D, _D, _I, _I, _I, ctypes.c_double, ctypes.c_double]
        L.ora_energy_G.restype = ctypes.c_double
        L.ora_grad_F.argtypes = [_D, _I, _I, _D, _D, _I, _I, _I, _D]
        L.ora_grad_F.restype = _I
        L.ora_prox.argtypes = [_D, _D, _L, _I, ctypes.c_double, ctypes.c_double, ctypes.c_double, _D,
                               ctypes.POINTER(ctypes.c_int)]
        L.ora_prox.restype = _I
        L.ora_step.argtypes = [ctypes.POINTER(_Params), _D, _D, _D, _I, _I, _I, _D, _D, ctypes.c_double, _D, _D]
        L.ora_step.restype = _I
        L.ora_ipiano.argtypes = [ctypes.POINTER(_Params), _D, _D, _D, _I, _I, _I, _D, _D, _D, _I, _D]
        L.ora_ipiano.restype = _I
        L.ora_set_threads.argtypes = [_I]
        L.ora_get_threads.restype = _I
        _lib = L
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(_D)


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def set_threads(n: int) -> None:
    lib().ora_set_threads(int(n))


def get_threads() -> int:
    return int(lib().ora_get_threads())


def forward(x, k, bc=SYMMETRIC) -> np.ndarray:
    """K x for one 7x7 filter (true convolution of the boundary-extended image)."""
    x = _f64(x); k = _f64(k)
    H, W = x.shape
    y = np.empty_like(x)
    lib().ora_forward(_p(x), H, W, _p(k), bc, _p(y))
    return y


def adjoint(v, k, bc=SYMMETRIC) -> np.ndarray:
    """K^T v = P^T C^T v for one 7x7 filter."""
    v = _f64(v); k = _f64(k)
    H, W = v.shape
    out = np.empty_like(v)
    assert lib().ora_adjoint(_p(v), H, W, _p(k), bc, _p(out)) == OK
    return out


def energy_F(x, bank, theta, model=COMBINED, bc=SYMMETRIC) -> float:
    x = _f64(x); bank = _f64(bank); theta = _f64(theta)
    H, W = x.shape
    return float(lib().ora_energy_F(_p(x), H, W, _p(bank), _p(theta), len(theta), model, bc))


def energy_G(x, f, model=COMBINED, lam1=160.0, lam2=0.004) -> float:
    x = _f64(x); f = _f64(f)
    H, W = x.shape
    return float(lib().ora_energy_G(_p(x), _p(f), H, W, model, lam1, lam2))


def grad_F(x, bank, theta, model=COMBINED, bc=SYMMETRIC) -> np.ndarray:
    x = _f64(x); bank = _f64(bank); theta = _f64(theta)
    H, W = x.shape
    g = np.empty_like(x)
    assert lib().ora_grad_F(_p(x), H, W, _p(bank), _p(theta), len(theta), model, bc, _p(g)) == OK
    return g


def prox(xhat, f, tau, model=COMBINED, lam1=160.0, lam2=0.004, return_iters=False):
    """prox_{tau G}(xhat), pixelwise."""
    xhat = _f64(xhat); f = _f64(f)
    out = np.empty_like(xhat)
    it = ctypes.c_int(0)
    lib().ora_prox(_p(xhat), _p(f), xhat.size, model, tau, lam1, lam2, _p(out), ctypes.byref(it))
    return (out, it.value) if return_iters else out


def init_state(f, model=COMBINED):
    """x^0 = x^{-1} = log f (log models) or f (I-divergence model)."""
    f = _f64(f)
    x0 = np.log(f) if model in (COMBINED, LOG) else f.copy()
    return x0.copy(), x0.copy()


def step(params: Params, f, bank, theta, x, xprev, L):
    """One trial at a forced L: returns (x+, {F, G, s1, s2})."""
    f = _f64(f); bank = _f64(bank); theta = _f64(theta); x = _f64(x); xprev = _f64(xprev)
    H, W = x.shape
    xn = np.empty_like(x)
    info = np.zeros(4)
    pc = params.c()
    st = lib().ora_step(ctypes.byref(pc), _p(f), _p(bank), _p(theta), len(theta), H, W, _p(x), _p(xprev), L,
                        _p(xn), _p(info))
    assert st == OK
    return xn, dict(F=info[0], G=info[1], s1=info[2], s2=info[3])


@dataclass
class Result:
    x: np.ndarray          # x^N
    x_prev: np.ndarray     # x^{N-1}
    L: float
    stats: np.ndarray      # [iters, 8]: F, G, L, alpha, trials, s1, s2, |x - x_prev|^2
    status: int

    def u(self, model=COMBINED) -> np.ndarray:
        return np.exp(self.x) if model in (COMBINED, LOG) else self.x.copy()


def ipiano(params: Params, f, bank, theta, iters: int, L0: float = 1.0, x_cur=None, x_prev=None) -> Result:
    f = _f64(f); bank = _f64(bank); theta = _f64(theta)
    H, W = f.shape
    if x_cur is None:
        x_cur, x_prev = init_state(f, params.model)
    x_cur = _f64(x_cur).copy(); x_prev = _f64(x_prev).copy()
    Lc = ctypes.c_double(L0)
    stats = np.zeros((iters, 8))
    pc = params.c()
    st = lib().ora_ipiano(ctypes.byref(pc), _p(f), _p(bank), _p(theta), len(theta), H, W, _p(x_cur), _p(x_prev),
                          ctypes.byref(Lc), iters, _p(stats))
    return Result(x_cur, x_prev, Lc.value, stats, st)


# ---------------------------------------------------------------- warm-start network (cnn_oracle.c)
def _cnn_lib():
    L = lib()
    if not getattr(L, "_cnn_ready", False):
        L.ora_cnn_num_params.restype = ctypes.c_long
        L.ora_cnn_loss_grad.argtypes = [_D, _D, _D, _I, _I, _I, _D]
        L.ora_cnn_loss_grad.restype = ctypes.c_double
        L.ora_cnn_forward.argtypes = [_D, _D, _I, _I, _D]
        L._cnn_ready = True
    return L


CNN_LAYERS = [(1, 32), (32, 32), (32, 32), (32, 32), (32, 32), (32, 1)]   # (in, out) channels
CNN_SHIFT = 4.5


def cnn_num_params() -> int:
    return int(_cnn_lib().ora_cnn_num_params())


def cnn_loss_grad(params, f, u_target, with_grad=True):
    """Mean squared error of w0 = log f + net(log f - 4.5) against log u_target over a batch
    [n, H, W], and its gradient with respect to the parameters (layout of cnn_oracle.c)."""
    params = _f64(params); f = _f64(f); ut = _f64(u_target)
    n, H, W = f.shape
    g = np.zeros(params.size) if with_grad else None
    loss = _cnn_lib().ora_cnn_loss_grad(_p(params), _p(f), _p(ut), n, H, W, _p(g) if with_grad else None)
    return float(loss), g


def cnn_forward(params, f):
    params = _f64(params); f = _f64(f)
    H, W = f.shape
    w0 = np.empty_like(f)
    _cnn_lib().ora_cnn_forward(_p(params), _p(f), H, W, _p(w0))
    return w0


def cnn_relu_margin(params, f) -> float:
    """Smallest |pre-activation| of the ReLUs over a batch [n, H, W]."""
    params = _f64(params); f = _f64(f)
    n, H, W = f.shape
    L = _cnn_lib()
    L.ora_cnn_relu_margin.argtypes = [_D, _D, _I, _I, _I]
    L.ora_cnn_relu_margin.restype = ctypes.c_double
    return float(L.ora_cnn_relu_margin(_p(params), _p(f), n, H, W))


from .quality import ssim, ssim_map  # noqa: E402,F401  (FP64 SSIM, quality reporting)
