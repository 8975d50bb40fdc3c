"""Shared set-up of the GPU parity tests: problems, solvers and the oracle side."""
from __future__ import annotations

import numpy as np

import oracle
import synth


def torch_dev():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm GPU"
    return torch, torch.device("cuda:0")


def bank_and_theta(kind: str, nf: int = 48, seed: int = 1):
    if kind == "dct":
        bank = synth.dct_bank()[:nf]
    else:
        bank = synth.random_bank(seed, nf)
    return bank, synth.theta_weights(seed, nf)


def make_solver(H, W, bank, theta, **kw):
    import paper_1404_5344_amd as foe
    p = foe.default_params(H, W, num_filters=len(theta), **kw)
    return foe.Solver(p, bank, theta)


def oracle_params(model, bc, lam1, lam2, beta=0.8, step_mode=oracle.BACKTRACK, alpha_fixed=0.0, max_backtracks=40):
    return oracle.Params(model=model, boundary=bc, lam1=lam1, lam2=lam2 if model == oracle.COMBINED else 0.0,
                         beta=beta, step_mode=step_mode, alpha_fixed=alpha_fixed, max_backtracks=max_backtracks)


def state_for(model, f):
    """A realistic iterate: log f (log models) or f, plus a small seeded perturbation."""
    r = np.random.default_rng(123)
    f = np.asarray(f, np.float64)
    if model != oracle.IDIV:
        return (np.log(f) + 0.05 * r.standard_normal(f.shape)).astype(np.float32)
    return (f * np.exp(0.05 * r.standard_normal(f.shape))).astype(np.float32)   # stays > 0


def speckled(H, W, looks=4, seed=0):
    clean = synth.shapes_cosine_image(77, seed, H, W)
    return clean, synth.speckle(clean, looks, 77, seed)


def rel_inf(a, b):
    a = np.asarray(a, np.float64); b = np.asarray(b, np.float64)
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


# ---- rounding bounds of the FP32 path, derived from the arithmetic (standard model, unit roundoff 2^-24)
U32 = 2.0 ** -24


def gamma(n: int) -> float:
    """Bound on the relative error of an n-term FP32 sum of products (n u / (1 - n u))."""
    return n * U32 / (1.0 - n * U32)


def fp32_bounds(x, bank, theta, bc, model=oracle.COMBINED, operand_rel=0.0, adjoint_rel=0.0):
    """Pointwise bound on |g_gpu - g_ora| and bound on |F_gpu - F_ora| for the FP32 path at x.

    Forward: y_i = K_i u carries |dy_i| <= (gamma(49) + 2 operand_rel) (|K_i| |u|), operand_rel being the
    relative rounding of each forward operand (0 for FP32 operands, 2^-22 for the FP16 head + tail split).
    Nonlinearity: z = y / (1 + y^2) has |dz/dy| <= 1 and adds two roundings, |dz| <= |dy| + 2^-22 |z|.
    Adjoint: each term 2 theta_i k_i[t] z_i carries adjoint_rel (0 in FP32, 2^-8 + 2^-18 for BF16 operands) and
    the sum of 48 x 49 terms gamma(2400) of sum |terms|; the chain rule by u one more rounding.
    F: theta_i (|rho'(y)| |dy| + rounding of 1 + y^2 (2^-24, absolute) and of the hardware log (2^-22 rel.)).
    Returns (g_bound [H, W], F_bound)."""
    x = np.asarray(x, np.float64)
    u = np.exp(x) if model != oracle.IDIV else x
    acc = np.zeros_like(u)
    Fb = 0.0
    for i in range(len(theta)):
        k = np.asarray(bank[i], np.float64)
        y = oracle.forward(u, k, bc)
        ay = oracle.forward(np.abs(u), np.abs(k), bc)
        dy = (gamma(49) + 2.0 * operand_rel) * ay
        z = y / (1.0 + y * y)
        dz = dy + 2.0 ** -22 * np.abs(z)
        acc += 2.0 * float(theta[i]) * (oracle.adjoint(dz, np.abs(k), bc) +
                                        (gamma(2400) + adjoint_rel) * oracle.adjoint(np.abs(z), np.abs(k), bc))
        Fb += float(theta[i]) * float(np.sum(2.0 * np.abs(z) * dy + 2.0 ** -22 * np.log1p(y * y) + 2.0 ** -23))
    w = u if model != oracle.IDIV else 1.0
    g_ora = oracle.grad_F(x, bank, theta, model, bc)
    return w * acc + 2.0 ** -23 * np.abs(g_ora), Fb
