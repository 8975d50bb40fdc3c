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
