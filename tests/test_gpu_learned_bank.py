"""Filter banks of the learned kind (Sec. II-A: filters of varied norm and weight, not zero-sum) on every
engine, against the FP64 oracle.

The seeded banks (synth.learned_style_bank) keep a random mean per filter, norms from 0.2 to 5 and weights up to
5: the responses K_i u of an 8-bit image then reach |y| >> 1, where rho' saturates.  A bank scaled by 2^-18 (taps
of order 1e-6) checks that no engine loses accuracy on small taps.

Bars.  The fixed relative bars of test_gpu_parity.py (gradient 1e-4, F 2e-6) were set for unit-norm zero-sum
banks; with these banks FP32 arithmetic itself -- the VALU direct convolution included -- exceeds them: the
forward sums cancel (|K u| << |K| |u|) and, for tiny taps, 1 + y^2 rounds to 1 in FP32.  Every engine is held
instead to the pointwise rounding bound of its own arithmetic (gpu_helpers.fp32_bounds: FP32 operands, the
2^-22 split operands of the FP16 head + tail engine, the BF16 adjoint), and a trial step to alpha times the
gradient bound plus FP32 step rounding (the prox is nonexpansive).  A wrong tap, index or layout misses these
bounds by orders of magnitude; the printed ratio error / bound shows the margin.
"""
import numpy as np
import pytest

import oracle
import synth
from gpu_helpers import fp32_bounds, make_solver, oracle_params, rel_inf, speckled, torch_dev

pytestmark = pytest.mark.gpu

ENGINES = {"valu": dict(engine=1), "mfma_fp32": dict(engine=2), "mfma_split": dict(engine=3), "bf16": dict(precision=1)}
# (operand_rel, adjoint_rel) of each engine's arithmetic (gpu_helpers.fp32_bounds)
ROUNDING = {"valu": (0.0, 0.0), "mfma_fp32": (0.0, 0.0), "mfma_split": (2.0 ** -22, 0.0),
            "bf16": (2.0 ** -22, 2.0 ** -8 + 2.0 ** -18)}
LAM = (358.0, 0.0104)


def _gpu(t, dev):
    torch, _ = torch_dev()
    return torch.from_numpy(np.ascontiguousarray(t, dtype=np.float32)).to(dev)


def _bank(kind, seed):
    bank, theta = synth.learned_style_bank(seed)
    if kind == "tiny":
        bank = (bank.astype(np.float64) * 2.0 ** -18).astype(np.float32)
    return bank, theta


@pytest.mark.parametrize("kind", ["learned", "tiny"])
@pytest.mark.parametrize("engine", list(ENGINES))
@pytest.mark.parametrize("bc", [oracle.SYMMETRIC, oracle.PERIODIC])
@pytest.mark.parametrize("shape", [(37, 64), (70, 45), (100, 131)])
def test_gradient_and_energy(shape, bc, engine, kind):
    torch, dev = torch_dev()
    H, W = shape
    clean, f = speckled(H, W, seed=H + 7 * W)
    bank, theta = _bank(kind, H + W)
    x = (np.log(f) + 0.05 * np.random.default_rng(3).standard_normal(f.shape)).astype(np.float32)
    s = make_solver(H, W, bank, theta, boundary=bc, lambda1=LAM[0], lambda2=LAM[1], **ENGINES[engine])
    g = s.eval_gradient(_gpu(x, dev)).cpu().numpy().astype(np.float64)
    g_ora = oracle.grad_F(x, bank, theta, oracle.COMBINED, bc)
    F, G = s.eval_energy(_gpu(x, dev), _gpu(f, dev))
    F_ora = oracle.energy_F(x, bank, theta, oracle.COMBINED, bc)
    gb, Fb = fp32_bounds(x, bank, theta, bc, operand_rel=ROUNDING[engine][0], adjoint_rel=ROUNDING[engine][1])
    ratio = float(np.max(np.abs(g - g_ora) / gb))
    print(f"{kind} {engine} {shape} bc {bc}: gradient rel err {rel_inf(g, g_ora):.2e} (error / bound {ratio:.3f}), "
          f"F rel err {abs(F - F_ora) / abs(F_ora):.2e} (error / bound {abs(F - F_ora) / Fb:.3f})")
    assert ratio <= 1.0
    assert abs(F - F_ora) <= Fb
    s.close()


@pytest.mark.parametrize("kind", ["learned", "tiny"])
@pytest.mark.parametrize("engine", list(ENGINES))
def test_step_teacher_forced(engine, kind):
    torch, dev = torch_dev()
    H, W = 70, 45
    clean, f = speckled(H, W, looks=4, seed=21)
    bank, theta = _bank(kind, 5)
    po = oracle_params(oracle.COMBINED, oracle.SYMMETRIC, *LAM)
    res = oracle.ipiano(po, f, bank, theta, 6, L0=1.0)
    assert res.status == oracle.OK
    x, xp, L = res.x.astype(np.float32), res.x_prev.astype(np.float32), float(res.L)
    s = make_solver(H, W, bank, theta, lambda1=LAM[0], lambda2=LAM[1], **ENGINES[engine])
    xn, info = s.step(_gpu(f, dev), _gpu(x, dev), _gpu(xp, dev), L)
    xn = xn.cpu().numpy().astype(np.float64)
    xn_ora, info_ora = oracle.step(po, f, bank, theta, x, xp, L)
    alpha = 1.9 * (1.0 - 0.8) / L
    gb, _ = fp32_bounds(x, bank, theta, oracle.SYMMETRIC, operand_rel=ROUNDING[engine][0],
                        adjoint_rel=ROUNDING[engine][1])
    # x_hat = x - alpha g + beta (x - x_prev) in FP32 (three roundings of terms up to |x|), the prox's Newton
    # tolerance 4e-7 max(1, |w|), and the gradient's share alpha |dg| (the prox is nonexpansive)
    bound = alpha * gb + (4.0 * 2.0 ** -24 + 4e-7) * np.maximum(1.0, np.abs(x).astype(np.float64)) + \
        2.0 ** -24 * np.abs(xn_ora)
    ratio = float(np.max(np.abs(xn - xn_ora) / bound))
    print(f"{kind} {engine} step: x+ rel err {rel_inf(xn, xn_ora):.2e}, error / bound {ratio:.3f}, L {L:.3g}")
    assert ratio <= 1.0
    s.close()
