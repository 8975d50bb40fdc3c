"""Unfused gradient path (forward launch writes the 48 z planes to HBM, adjoint launch reads them)
against the FP64 oracle, at the bars of the fused path, and against the fused path itself."""
import numpy as np
import pytest

import oracle
import synth
from gpu_helpers import bank_and_theta, make_solver, oracle_params, rel_inf, speckled, state_for, torch_dev

pytestmark = pytest.mark.gpu

LAMS = {oracle.COMBINED: (358.0, 0.0104), oracle.LOG: (358.0, 0.0), oracle.IDIV: (10.0, 0.0)}


def _gpu(a, dev):
    torch, _ = torch_dev()
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(dev)


@pytest.mark.parametrize("engine", [1, 2, 3])
@pytest.mark.parametrize("model", [oracle.COMBINED, oracle.LOG, oracle.IDIV])
@pytest.mark.parametrize("bc", [oracle.SYMMETRIC, oracle.ZERO, oracle.PERIODIC])
@pytest.mark.parametrize("shape", [(8, 8), (37, 64), (66, 34), (100, 131), (33, 257)])
def test_unfused_gradient_and_energy(shape, bc, model, engine):
    torch, dev = torch_dev()
    H, W = shape
    clean, f = speckled(H, W, seed=H * 1000 + W)
    bank, theta = bank_and_theta("random" if (H + W + bc) % 2 else "dct", seed=H + W)
    x = state_for(model, f)
    l1, l2 = LAMS[model]
    s = make_solver(H, W, bank, theta, model=model, boundary=bc, lambda1=l1, lambda2=l2, engine=engine, fusion=1)
    g = s.eval_gradient(_gpu(x, dev)).cpu().numpy()
    g_ora = oracle.grad_F(x, bank, theta, model, bc)
    assert rel_inf(g, g_ora) <= 1e-4, rel_inf(g, g_ora)
    F, G = s.eval_energy(_gpu(x, dev), _gpu(f, dev))
    assert abs(F - oracle.energy_F(x, bank, theta, model, bc)) <= 2e-6 * abs(F)
    assert abs(G - oracle.energy_G(x, f, model, l1, l2)) <= 1e-6 * abs(G) + 1e-6
    s.close()


@pytest.mark.parametrize("bc", [oracle.SYMMETRIC, oracle.PERIODIC])
def test_unfused_step_teacher_forced(bc):
    torch, dev = torch_dev()
    H, W = 70, 45
    clean, f = speckled(H, W, looks=4, seed=11)
    bank, theta = bank_and_theta("dct")
    l1, l2 = LAMS[oracle.COMBINED]
    po = oracle_params(oracle.COMBINED, bc, l1, l2)
    res = oracle.ipiano(po, f, bank, theta, 6, L0=1.0)
    x, xp, L = res.x.astype(np.float32), res.x_prev.astype(np.float32), float(res.L)
    s = make_solver(H, W, bank, theta, boundary=bc, lambda1=l1, lambda2=l2, fusion=1)
    xn, info = s.step(_gpu(f, dev), _gpu(x, dev), _gpu(xp, dev), L)
    xn_ora, info_ora = oracle.step(po, f, bank, theta, x, xp, L)
    assert rel_inf(xn.cpu().numpy(), xn_ora) <= 1e-5
    assert abs(info["F"] - info_ora["F"]) <= 2e-6 * abs(info_ora["F"])
    s.close()


def test_unfused_solve_matches_fused():
    """Config 1, fixed step, 100 iterations: the two paths differ only in the order of the
    floating-point sums, and the unfused run meets the oracle bar."""
    torch, dev = torch_dev()
    pr = synth.config1()
    bank, theta = synth.dct_bank(), synth.theta_weights(1)
    kw = dict(lambda1=pr.lam1, lambda2=pr.lam2, step_mode=1, alpha_fixed=2e-6, max_iters=100)
    out = {}
    for fusion in (0, 1):
        s = make_solver(64, 64, bank, theta, fusion=fusion, **kw)
        r = s.solve(_gpu(pr.f, dev))
        out[fusion] = (r.u.cpu().numpy(), r.stats)
        s.close()
    assert np.max(np.abs(out[0][0] - out[1][0]) / out[0][0]) <= 1e-5
    po = oracle_params(oracle.COMBINED, oracle.SYMMETRIC, pr.lam1, pr.lam2, step_mode=oracle.FIXED, alpha_fixed=2e-6)
    ref = oracle.ipiano(po, pr.f, bank, theta, 100)
    assert abs(synth.psnr(out[1][0], pr.clean) - synth.psnr(ref.u(), pr.clean)) <= 0.01


def test_unfused_batch_equals_single():
    import paper_1404_5344_amd as foe
    torch, dev = torch_dev()
    sizes, looks = [(64, 96), (70, 45), (33, 257)], [1, 4, 2]
    probs = [synth.config3_image(i, H, W, L) for i, ((H, W), L) in enumerate(zip(sizes, looks))]
    bank, theta = synth.dct_bank(), synth.theta_weights(3)
    p = foe.default_params(0, 0, max_iters=20, fusion=1)
    b = foe.BatchSolver(p, sizes, looks, bank, theta)
    out, sums, stats, st = b.solve(b.pack([torch.from_numpy(pr.f) for pr in probs]).to(dev))
    outs = b.unpack(out)
    for i, pr in enumerate(probs):
        s = make_solver(pr.f.shape[0], pr.f.shape[1], bank, theta, max_iters=20, looks=pr.looks, fusion=1)
        r = s.solve(_gpu(pr.f, dev))
        assert torch.equal(r.u, outs[i]), i
        s.close()
    b.close()
