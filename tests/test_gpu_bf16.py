"""BF16 filter bank (forward contraction on v_mfma_f32_16x16x32_bf16, FP32 accumulation) against the
FP64 oracle; the prox, the adjoint, the energies and the line search stay FP32 / FP64.

Bars.  Each forward product is formed from a two-term BF16 split of both operands (the image
differences and the taps) with the lo x lo term dropped: the per-product relative error is at most
about 3 * 2^-16 = 4.6e-5 of |k| |delta u|, against 2^-24 for FP32.  Hence:
  * gradient probe: |g - g_ora|_inf / |g_ora|_inf <= 1e-3.  The per-product error reaches the
    gradient through rho' (slope up to 2) and the sums over 49 taps and up to 64 filters, against a
    gradient that cancels across filters; measured 1.2e-4 .. 4.1e-4 on these cases, against
    about 1e-6 for the FP32 bank.  The bar catches a wrong tap, sign or layout (errors of order 1);
    the accuracy that matters is that of full runs, bounded below;
  * energy F: relative 2e-5;
  * one teacher-forced trial step: |x+ - x+_ora|_inf / |x+_ora|_inf <= 1e-5 (the step moves x by
    far less than |x|, so the FP32 bar still holds);
  * full runs: PSNR within 0.05 dB of the oracle (the BF16 target), energies within 1e-4 relative;
  * the 2048 x 2048 SAR-like tile: PSNR of the BF16 and of the FP32 solve against the stored oracle
    run, and the largest absolute error on the stored sample of output pixels (stated, not bounded
    beyond the PSNR bar).
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
BF16 = dict(precision=1, engine=2)


def _gpu(a, dev):
    torch, _ = torch_dev()
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(dev)


@pytest.mark.parametrize("bc", [oracle.SYMMETRIC, oracle.ZERO, oracle.PERIODIC])
@pytest.mark.parametrize("shape", [(8, 8), (37, 64), (100, 131), (33, 257), (66, 34)])
def test_bf16_gradient_and_energy(shape, bc):
    torch, dev = torch_dev()
    H, W = shape
    clean, f = speckled(H, W, seed=H * 1000 + W)
    bank, theta = bank_and_theta("random" if (H + W + bc) % 2 else "dct", seed=H + W)
    x = state_for(oracle.COMBINED, f)
    s = make_solver(H, W, bank, theta, boundary=bc, lambda1=358.0, lambda2=0.0104, **BF16)
    g = s.eval_gradient(_gpu(x, dev)).cpu().numpy()
    g_ora = oracle.grad_F(x, bank, theta, oracle.COMBINED, bc)
    err = rel_inf(g, g_ora)
    F, G = s.eval_energy(_gpu(x, dev), _gpu(f, dev))
    F_ora = oracle.energy_F(x, bank, theta, oracle.COMBINED, bc)
    print(f"bf16 {shape} bc {bc}: gradient rel err {err:.2e}, F rel err {abs(F - F_ora) / abs(F_ora):.2e}")
    assert err <= 1e-3
    assert abs(F - F_ora) <= 2e-5 * abs(F_ora)
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
    err = rel_inf(xn.cpu().numpy(), xn_ora)
    print(f"bf16 step bc {bc}: x+ rel err {err:.2e}")
    assert err <= 1e-5
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


def test_config4_tile_against_stored_oracle():
    """2048 x 2048 SAR-like tile, 300 backtracking iterations, BF16 and FP32 filter banks."""
    path = os.path.join(GOLDEN, "config4_tile0_oracle.json")
    ref = json.load(open(path))
    torch, dev = torch_dev()
    pr = synth.config4(0)
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
        print(f"config4 {name}: PSNR {synth.psnr(u, pr.clean, pr.peak):.4f} vs oracle {ref['psnr_final']:.4f} "
              f"(diff {d:.4f} dB), energy rel diff {abs(H - H_ora) / H_ora:.2e}, max abs err on "
              f"{len(idx)} sampled pixels {err.max():.3e} (max rel {np.max(err / u_ref):.2e})")
        assert d <= 0.05, (name, d)
        assert abs(H - H_ora) <= 1e-4 * H_ora
        s.close()
