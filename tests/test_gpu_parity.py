"""GPU parity of the HIP path against the FP64 oracle (through the C ABI).

Bars (all float32 on the GPU against float64 on the CPU, same float32 inputs):
  * gradient probe:  |g_gpu - g_ora|_inf / |g_ora|_inf <= 1e-4
  * energies:        relative 2e-6 (F), 1e-6 (G)
  * prox probe:      |x_gpu - x_ora| <= 1e-5 max(1, |x_ora|) elementwise
  * one trial step at a forced L (teacher-forced): |x+_gpu - x+_ora|_inf / |x+_ora|_inf <= 1e-5
Sizes span one to many 32x32 tiles with ragged tails; the three models and three boundary maps.
"""
import numpy as np
import pytest

import oracle
import synth
from gpu_helpers import bank_and_theta, make_solver, oracle_params, rel_inf, speckled, state_for, torch_dev

pytestmark = pytest.mark.gpu

MODELS = [oracle.COMBINED, oracle.LOG, oracle.IDIV]
BCS = [oracle.SYMMETRIC, oracle.ZERO, oracle.PERIODIC]
# ragged tails of every length mod 32, including tails of 1 and 2 (mirror samples past the next tile)
SIZES = [(8, 8), (13, 21), (37, 64), (70, 45), (100, 131), (33, 257), (66, 34)]
LAMS = {oracle.COMBINED: (358.0, 0.0104), oracle.LOG: (358.0, 0.0), oracle.IDIV: (10.0, 0.0)}


def _gpu(t, dev):
    torch, _ = torch_dev()
    return torch.from_numpy(np.ascontiguousarray(t, dtype=np.float32)).to(dev)


ENGINES = [1, 2, 3]   # FOE_ENGINE_VALU, FOE_ENGINE_MFMA, FOE_ENGINE_MFMA_SPLIT (forward bank on matrix cores)


@pytest.mark.parametrize("engine", ENGINES)
@pytest.mark.parametrize("model", MODELS)
@pytest.mark.parametrize("bc", BCS)
@pytest.mark.parametrize("shape", SIZES)
def test_gradient_and_energy(model, bc, shape, engine):
    torch, dev = torch_dev()
    H, W = shape
    clean, f = speckled(H, W, seed=H * 1000 + W)
    bank, theta = bank_and_theta("random" if (H + W + bc) % 2 else "dct", seed=H + W)
    x = state_for(model, f)
    l1, l2 = LAMS[model]
    s = make_solver(H, W, bank, theta, model=model, boundary=bc, lambda1=l1, lambda2=l2, engine=engine)
    g = s.eval_gradient(_gpu(x, dev)).cpu().numpy()
    g_ora = oracle.grad_F(x, bank, theta, model, bc)
    assert rel_inf(g, g_ora) <= 1e-4, (model, bc, shape, rel_inf(g, g_ora))
    F, G = s.eval_energy(_gpu(x, dev), _gpu(f, dev))
    F_ora = oracle.energy_F(x, bank, theta, model, bc)
    G_ora = oracle.energy_G(x, f, model, l1, l2)
    assert abs(F - F_ora) <= 2e-6 * abs(F_ora), (F, F_ora)
    assert abs(G - G_ora) <= 1e-6 * abs(G_ora) + 1e-6, (G, G_ora)
    s.close()


@pytest.mark.parametrize("model", MODELS)
def test_prox(model):
    torch, dev = torch_dev()
    H, W = 64, 96
    clean, f = speckled(H, W, looks=1, seed=5)
    r = np.random.default_rng(0)
    l1, l2 = LAMS[model]
    bank, theta = bank_and_theta("dct")
    s = make_solver(H, W, bank, theta, model=model, lambda1=l1, lambda2=l2)
    for tau in (1e-6, 3e-5, 1e-3, 0.05):
        if model == oracle.IDIV:
            xh = (f + r.uniform(-100, 100, f.shape)).astype(np.float32)
        else:
            xh = (np.log(f) + r.uniform(-3, 3, f.shape)).astype(np.float32)
        out = s.eval_prox(_gpu(xh, dev), _gpu(f, dev), tau).cpu().numpy()
        ref = oracle.prox(xh, f, float(np.float32(tau)), model, l1, l2)
        err = np.abs(out - ref) / np.maximum(1.0, np.abs(ref))
        assert err.max() <= 1e-5, (tau, err.max())
    s.close()


@pytest.mark.parametrize("engine", ENGINES)
@pytest.mark.parametrize("model", MODELS)
@pytest.mark.parametrize("bc", BCS)
def test_step_teacher_forced(model, bc, engine):
    torch, dev = torch_dev()
    H, W = 70, 45
    clean, f = speckled(H, W, looks=4, seed=11)
    bank, theta = bank_and_theta("dct")
    l1, l2 = LAMS[model]
    po = oracle_params(model, bc, l1, l2)
    # reach a mid-run state with the oracle, then compare one step at the oracle's accepted L
    res = oracle.ipiano(po, f, bank, theta, 6, L0=1.0)
    assert res.status == oracle.OK
    x = res.x.astype(np.float32)
    xp = res.x_prev.astype(np.float32)
    L = float(res.L)
    s = make_solver(H, W, bank, theta, model=model, boundary=bc, lambda1=l1, lambda2=l2, engine=engine)
    xn, info = s.step(_gpu(f, dev), _gpu(x, dev), _gpu(xp, dev), L)
    xn = xn.cpu().numpy()
    xn_ora, info_ora = oracle.step(po, f, bank, theta, x, xp, L)
    assert rel_inf(xn, xn_ora) <= 1e-5, rel_inf(xn, xn_ora)
    d_gpu = xn - x
    d_ora = xn_ora - x
    # increment error, reported separately; float32 storage of x+ bounds it below by a few ulp of x
    inc_err = float(np.max(np.abs(d_gpu - d_ora)))
    print(f"step model {model} bc {bc}: |x+ err| rel {rel_inf(xn, xn_ora):.2e}, |d err| {inc_err:.2e} "
          f"vs |d| {np.max(np.abs(d_ora)):.2e}")
    assert inc_err <= 2e-3 * np.max(np.abs(d_ora)) + 8 * np.finfo(np.float32).eps * np.max(np.abs(x))
    assert abs(info["F"] - info_ora["F"]) <= 2e-6 * abs(info_ora["F"])
    # |d|^2: the device reduction equals the sum over the returned float32 x+, and matches the oracle
    # up to the float32 storage of x+ (sqrt(N) ulp of x)
    assert abs(info["s2"] - float(np.sum(d_gpu.astype(np.float64) ** 2))) <= 1e-6 * info["s2"]
    q = np.sqrt(d_gpu.size) * 8 * np.finfo(np.float32).eps * np.max(np.abs(x))
    assert abs(np.sqrt(info["s2"]) - np.sqrt(info_ora["s2"])) <= 2e-3 * np.sqrt(info_ora["s2"]) + q
    s.close()


@pytest.mark.parametrize("engine", ENGINES)
@pytest.mark.parametrize("nf", [13, 48, 64])
def test_random_filters_and_filter_counts(nf, engine):
    """Nothing may rely on the DCT bank: random non-separable filters; 13 filters (ragged chunk), 64 (maximum)."""
    torch, dev = torch_dev()
    H, W = 45, 77
    clean, f = speckled(H, W, seed=3)
    bank, theta = bank_and_theta("random", nf=nf, seed=7)
    x = state_for(oracle.COMBINED, f)
    s = make_solver(H, W, bank, theta, engine=engine)
    g = s.eval_gradient(_gpu(x, dev)).cpu().numpy()
    assert rel_inf(g, oracle.grad_F(x, bank, theta)) <= 1e-4
    s.close()


@pytest.mark.parametrize("cfg", [0, 1, 2, 3])
@pytest.mark.parametrize("bc", BCS)
@pytest.mark.parametrize("shape", [(37, 64), (70, 45), (100, 131), (33, 257), (66, 98), (17, 18)])
def test_gradient_tile_configs(shape, bc, cfg):
    """Every tile configuration (32x32, 32x16 and 32x8 output tiles) against the oracle."""
    torch, dev = torch_dev()
    H, W = shape
    clean, f = speckled(H, W, seed=H * 7 + W)
    bank, theta = bank_and_theta("random", seed=H)
    x = state_for(oracle.COMBINED, f)
    s = make_solver(H, W, bank, theta, boundary=bc)
    s.set_tile_config(cfg)
    g = s.eval_gradient(_gpu(x, dev)).cpu().numpy()
    g_ora = oracle.grad_F(x, bank, theta, oracle.COMBINED, bc)
    F, G = s.eval_energy(_gpu(x, dev), _gpu(f, dev))
    assert rel_inf(g, g_ora) <= 1e-4, (shape, bc, cfg, rel_inf(g, g_ora))
    assert abs(F - oracle.energy_F(x, bank, theta, oracle.COMBINED, bc)) <= 2e-6 * abs(F)
    s.close()


@pytest.mark.parametrize("scale", [1e-5, 1e2, "targets"])
@pytest.mark.parametrize("model", MODELS)
def test_split_engine_tile_scaling(model, scale):
    """Intensities outside [2^-4, 2^14), where the split-FP16 engine scales u per tile by a power of two
    before splitting it: its gradient and F are as close to the oracle as those of the FP32-operand engine
    (within 2x, or within the FP32 bars).  At large intensities FP32 itself loses the fine scale of y (the
    zero-mean filters cancel to |y| ~ 1 against u ~ 1e5), so both engines are held to each other there;
    "targets" scales 6 pixels by 200 (bright point targets), so that only their tiles are rescaled.  F
    also gets the absolute error of FP32 log(1 + y^2): 1 + y^2 is rounded to FP32 (relative error <= 2^-24),
    so each term theta_i log(1 + y^2) may be off by theta_i 2^-24, which dominates when every y is tiny."""
    torch, dev = torch_dev()
    H, W = 70, 45
    clean, f = speckled(H, W, seed=5)
    f = f.astype(np.float64)
    if scale == "targets":
        idx = np.random.default_rng(9).choice(H * W, 6, replace=False)
        f.reshape(-1)[idx] *= 200.0
    else:
        f = f * scale
    f = f.astype(np.float32)
    bank, theta = bank_and_theta("dct", seed=3)
    x = state_for(model, f)
    l1, l2 = LAMS[model]
    g_ora = oracle.grad_F(x, bank, theta, model, oracle.SYMMETRIC)
    F_ora = oracle.energy_F(x, bank, theta, model, oracle.SYMMETRIC)
    tol_F = 2e-6 * abs(F_ora) + 2.0 ** -24 * float(np.sum(theta)) * H * W
    err_g, err_F = {}, {}
    for engine in (2, 3):
        s = make_solver(H, W, bank, theta, model=model, boundary=oracle.SYMMETRIC, lambda1=l1, lambda2=l2,
                        engine=engine)
        err_g[engine] = rel_inf(s.eval_gradient(_gpu(x, dev)).cpu().numpy(), g_ora)
        F, G = s.eval_energy(_gpu(x, dev), _gpu(f, dev))
        err_F[engine] = abs(F - F_ora)
        s.close()
    print(f"model {model} scale {scale}: grad err fp32 {err_g[2]:.2e} split {err_g[3]:.2e}; "
          f"F err fp32 {err_F[2]:.2e} split {err_F[3]:.2e} (bar {tol_F:.2e})")
    assert err_g[3] <= max(1e-4, 2.0 * err_g[2]), err_g
    assert err_F[3] <= max(tol_F, 2.0 * err_F[2]), (err_F, tol_F)


def test_auto_engine_falls_back_for_large_taps():
    """AUTO takes the split-FP16 engine only when every abs(tap) < 2^14; a bank beyond that runs on the
    FP32-operand engine: bitwise the same gradient and energies as asking for that engine."""
    torch, dev = torch_dev()
    H, W = 37, 64
    clean, f = speckled(H, W, seed=11)
    f = (f.astype(np.float64) * 1e-4).astype(np.float32)       # keeps y = K u of order 1
    bank, theta = bank_and_theta("dct", seed=2)
    bank = (np.asarray(bank, np.float64) * 6e4).astype(np.float32)
    assert np.abs(bank).max() >= 2.0 ** 14
    x = state_for(oracle.COMBINED, f)
    out = {}
    for engine in (0, 2):   # AUTO, FP32 operands
        s = make_solver(H, W, bank, theta, engine=engine)
        g = s.eval_gradient(_gpu(x, dev)).cpu().numpy()
        out[engine] = (g, s.eval_energy(_gpu(x, dev), _gpu(f, dev)))
        s.close()
    assert np.array_equal(out[0][0], out[2][0])
    assert out[0][1] == out[2][1]


def test_auto_engine_is_the_split_engine():
    """With every abs(tap) < 2^14 AUTO runs the split-FP16 engine: bitwise its gradient and energies."""
    torch, dev = torch_dev()
    H, W = 37, 64
    clean, f = speckled(H, W, seed=12)
    bank, theta = bank_and_theta("random", seed=4)
    x = state_for(oracle.COMBINED, f)
    out = {}
    for engine in (0, 3):   # AUTO, split FP16
        s = make_solver(H, W, bank, theta, engine=engine)
        out[engine] = (s.eval_gradient(_gpu(x, dev)).cpu().numpy(), s.eval_energy(_gpu(x, dev), _gpu(f, dev)))
        s.close()
    assert np.array_equal(out[0][0], out[3][0]) and out[0][1] == out[3][1]


def test_auto_engine_falls_back_for_tiny_filters():
    """The split carries a tap to an absolute 2^-36, so AUTO runs a bank with a nonzero filter whose
    largest abs(tap) is below 2^-10 on the FP32-operand engine: bitwise that engine's gradient and
    energies, and the gradient within the FP32 bar of the oracle on a bank scaled by 2^-18 (theta scaled
    by 2^36 to keep the gradient of order one)."""
    torch, dev = torch_dev()
    H, W = 37, 64
    clean, f = speckled(H, W, seed=13)
    bank, theta = bank_and_theta("random", seed=5)
    bank = (np.asarray(bank, np.float64) * 2.0 ** -18).astype(np.float32)
    theta = (np.asarray(theta, np.float64) * 2.0 ** 36).astype(np.float32)
    assert 0.0 < np.abs(bank).max() < 2.0 ** -10
    x = state_for(oracle.COMBINED, f)
    g_ora = oracle.grad_F(x, bank, theta, oracle.COMBINED, oracle.SYMMETRIC)
    out = {}
    for engine in (0, 2, 3):   # AUTO, FP32 operands, split FP16
        s = make_solver(H, W, bank, theta, engine=engine)
        out[engine] = (s.eval_gradient(_gpu(x, dev)).cpu().numpy(), s.eval_energy(_gpu(x, dev), _gpu(f, dev)))
        s.close()
    print("gradient rel err: FP32 engine %.3e, split engine %.3e" % (rel_inf(out[2][0], g_ora), rel_inf(out[3][0], g_ora)))
    assert np.array_equal(out[0][0], out[2][0]) and out[0][1] == out[2][1]
    assert rel_inf(out[0][0], g_ora) <= 1e-4
