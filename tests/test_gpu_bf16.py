"""BF16 precision against the FP64 oracle.  The BF16 engine runs the forward bank of the split-FP16
engine (FP32-level y, so the energies of the line search keep FP32 accuracy) and the adjoint bank
sum_i K_i^T (2 theta_i z_i) (Sec. II-C) as a Toeplitz GEMM on v_mfma_f32_16x16x32_bf16: every z_i and every
adjoint tap 2 theta_i k_i[t] is rounded once to BF16, products and sums are FP32; the prox is FP32, the
energies and reductions FP64.

Bars, from the arithmetic.  BF16 round-to-nearest has unit roundoff 2^-9, so each adjoint product
(2 theta_i k_i[t]) z_i(q) carries a relative error of at most 2^-8 + 2^-18.  Summed over filters and taps
(including the mirror terms of the boundary map) the gradient error at pixel p is bounded by
  |g(p) - g_ora(p)| <= (2^-8 + 2^-18) w(p) sum_i 2 theta_i (|K_i|^T |z_i|)(p)  +  1e-5 |g_ora|_inf,
w = u for the log models; the last term is FP32 room (the FP32 bank meets 1e-6).  A wrong tap, sign, layout
or lane breaks this pointwise bound.  Through the nonexpansive prox a trial step inherits alpha times that
bound, and F(x+) the change that bound allows.  F comes from the FP32-level forward and keeps the FP32 bar
(2e-6) at a given x.  Full runs: PSNR within 0.05 dB
of the oracle (the BF16 target) and the final energy within 1e-4; the 2048 x 2048 SAR-like tiles state the
largest absolute error on the stored sample of output pixels.
"""
import json
import os

import numpy as np
import pytest

import oracle
import synth
from gpu_helpers import bank_and_theta, make_solver, oracle_params, rel_inf, speckled, state_for, torch_dev

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
BF16 = dict(precision=1)
U_PROD = 2.0 ** -8 + 2.0 ** -18


def _gpu(a, dev):
    torch, _ = torch_dev()
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(dev)


def gradient_bound(x, bank, theta, bc, model=oracle.COMBINED):
    """The pointwise BF16 bound on |g - g_ora| (module docstring), from the oracle's operators."""
    u = np.exp(np.asarray(x, np.float64)) if model != oracle.IDIV else np.asarray(x, np.float64)
    acc = np.zeros_like(u)
    for i in range(len(theta)):
        y = oracle.forward(u, bank[i], bc)
        z = y / (1.0 + y * y)
        acc += 2.0 * float(theta[i]) * oracle.adjoint(np.abs(z), np.abs(np.asarray(bank[i], np.float64)), bc)
    return U_PROD * (u if model != oracle.IDIV else 1.0) * acc


@pytest.mark.parametrize("bc", [oracle.SYMMETRIC, oracle.ZERO, oracle.PERIODIC])
@pytest.mark.parametrize("shape", [(8, 8), (37, 64), (100, 131), (33, 257), (66, 34)])
def test_bf16_gradient_and_energy(shape, bc):
    torch, dev = torch_dev()
    H, W = shape
    clean, f = speckled(H, W, seed=H * 1000 + W)
    bank, theta = bank_and_theta("random" if (H + W + bc) % 2 else "dct", seed=H + W)
    x = state_for(oracle.COMBINED, f)
    s = make_solver(H, W, bank, theta, boundary=bc, lambda1=358.0, lambda2=0.0104, **BF16)
    g = s.eval_gradient(_gpu(x, dev)).cpu().numpy().astype(np.float64)
    g_ora = oracle.grad_F(x, bank, theta, oracle.COMBINED, bc)
    bound = gradient_bound(x, bank, theta, bc) + 1e-5 * np.abs(g_ora).max()
    ratio = float(np.max(np.abs(g - g_ora) / bound))
    F, G = s.eval_energy(_gpu(x, dev), _gpu(f, dev))
    F_ora = oracle.energy_F(x, bank, theta, oracle.COMBINED, bc)
    print(f"bf16 {shape} bc {bc}: gradient rel err {rel_inf(g, g_ora):.2e}, error / bound {ratio:.3f}, "
          f"F rel err {abs(F - F_ora) / abs(F_ora):.2e}")
    assert ratio <= 1.0
    assert abs(F - F_ora) <= 2e-6 * abs(F_ora)
    s.close()


@pytest.mark.parametrize("bc", [oracle.SYMMETRIC, oracle.ZERO])
def test_bf16_step_teacher_forced(bc):
    torch, dev = torch_dev()
    H, W = 70, 45
    clean, f = speckled(H, W, looks=4, seed=11)
    bank, theta = bank_and_theta("dct")
    po = oracle_params(oracle.COMBINED, bc, 358.0, 0.0104)
    res = oracle.ipiano(po, f, bank, theta, 6, L0=1.0)
    x, xp, L = res.x.astype(np.float32), res.x_prev.astype(np.float32), float(res.L)
    s = make_solver(H, W, bank, theta, boundary=bc, lambda1=358.0, lambda2=0.0104, **BF16)
    xn, info = s.step(_gpu(f, dev), _gpu(x, dev), _gpu(xp, dev), L)
    xn_ora, info_ora = oracle.step(po, f, bank, theta, x, xp, L)
    alpha = 1.9 * (1.0 - 0.8) / L
    g_ora = oracle.grad_F(x, bank, theta, oracle.COMBINED, bc)
    bound = alpha * (gradient_bound(x, bank, theta, bc) + 1e-5 * np.abs(g_ora).max()) + 1e-5 * np.abs(xn_ora).max()
    err = np.abs(xn.cpu().numpy().astype(np.float64) - xn_ora)
    print(f"bf16 step bc {bc}: x+ rel err {rel_inf(xn.cpu().numpy(), xn_ora):.2e}, error / bound "
          f"{float(np.max(err / bound)):.3f}, F rel err {abs(info['F'] - info_ora['F']) / abs(info_ora['F']):.2e}")
    assert np.all(err <= bound)
    # F(x+) moves with x+: |F(x+) - F(x+_ora)| <= sum_p |grad F(x+_ora)| (x+ error bound), plus the FP32 bar
    dF = float(np.sum(np.abs(oracle.grad_F(xn_ora, bank, theta, oracle.COMBINED, bc)) * bound))
    assert abs(info["F"] - info_ora["F"]) <= 2e-6 * abs(info_ora["F"]) + dF
    s.close()


def test_bf16_config1_runs():
    """Config 1 image, fixed step (100 iterations) and backtracking (100 iterations)."""
    torch, dev = torch_dev()
    pr = synth.config1()
    bank, theta = synth.dct_bank(), synth.theta_weights(1)
    po_bt = oracle_params(oracle.COMBINED, oracle.SYMMETRIC, pr.lam1, pr.lam2)
    ref_bt = oracle.ipiano(po_bt, pr.f, bank, theta, 100, L0=1.0)
    alpha = 1.9 * 0.2 / (2.0 * ref_bt.stats[:, 2].max())
    po_fx = oracle_params(oracle.COMBINED, oracle.SYMMETRIC, pr.lam1, pr.lam2, step_mode=oracle.FIXED,
                          alpha_fixed=alpha)
    ref_fx = oracle.ipiano(po_fx, pr.f, bank, theta, 100)
    for name, ref, kw in (("fixed", ref_fx, dict(step_mode=1, alpha_fixed=alpha)), ("backtracking", ref_bt, {})):
        s = make_solver(64, 64, bank, theta, lambda1=pr.lam1, lambda2=pr.lam2, max_iters=100, **kw, **BF16)
        out = s.solve(_gpu(pr.f, dev))
        d = abs(synth.psnr(out.u.cpu().numpy(), pr.clean) - synth.psnr(ref.u(), pr.clean))
        H = out.stats[-1, 0] + out.stats[-1, 1]
        H_ora = ref.stats[-1, 0] + ref.stats[-1, 1]
        print(f"bf16 config1 {name}: PSNR diff {d:.4f} dB, final energy rel diff {abs(H - H_ora) / H_ora:.2e}")
        assert d <= 0.05
        assert abs(H - H_ora) <= 1e-4 * H_ora
        s.close()


@pytest.mark.parametrize("tile", [0, 1, 2, 3])
def test_config4_tile_against_stored_oracle(tile):
    """2048 x 2048 SAR-like tile, 300 backtracking iterations, BF16 and FP32 filter banks."""
    path = os.path.join(GOLDEN, f"config4_tile{tile}_oracle.json")
    if not os.path.exists(path):
        pytest.skip(f"no stored oracle run for tile {tile} (tests/golden/make_golden.py config4_{tile})")
    ref = json.load(open(path))
    torch, dev = torch_dev()
    pr = synth.config4(tile)
    bank, theta = synth.dct_bank(), synth.theta_weights(4)
    idx = np.array(ref["u_sample_idx"])
    u_ref = np.array(ref["u_sample"])
    H_ora = ref["F"][-1] + ref["G"][-1]
    for name, kw in (("bf16", BF16), ("fp32", {})):
        s = make_solver(2048, 2048, bank, theta, lambda1=pr.lam1, lambda2=pr.lam2, max_iters=300, **kw)
        out = s.solve(_gpu(pr.f, dev))
        u = out.u.cpu().numpy()
        d = abs(synth.psnr(u, pr.clean, pr.peak) - ref["psnr_final"])
        H = out.stats[-1, 0] + out.stats[-1, 1]
        err = np.abs(u.ravel()[idx].astype(np.float64) - u_ref)
        print(f"config4 tile {tile} {name}: PSNR {synth.psnr(u, pr.clean, pr.peak):.4f} vs oracle "
              f"{ref['psnr_final']:.4f} (diff {d:.4f} dB), energy rel diff {abs(H - H_ora) / H_ora:.2e}, max abs "
              f"err on {len(idx)} sampled pixels {err.max():.3e} (max rel {np.max(err / u_ref):.2e})")
        assert d <= 0.05, (name, d)
        assert abs(H - H_ora) <= 1e-4 * H_ora
        s.close()
