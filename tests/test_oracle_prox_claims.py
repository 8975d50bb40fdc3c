"""Oracle pins that tie the data term to its prox (Sec. II-C, eq. (subproblem)) and the paper's statement that
the Newton solve of the prox needs fewer than 10 iterations.

* G against the prox: w* = prox_{tau G}(w_hat) minimises |w - w_hat|^2 / 2 + tau G(w), so at w* the derivative of
  G at each pixel equals (w_hat - w*) / tau.  The test takes central differences of the oracle's G (one pixel at a
  time) at w* from the oracle's prox and compares them with (w_hat - w*) / tau: a dropped term, a wrong sign or a
  wrong factor in either function fails it.  The prox itself is pinned elsewhere (closed forms through Lambert's W,
  scalar minimisation, the printed IDIV formula), so this pins G outright, for COMBINED, LOG and IDIV.
* Newton count: on iterates of seeded runs of the configurations' workloads (step x_hat = x - alpha grad F(x) +
  beta (x - x_prev) at the accepted L), Newton's method from w_hat reaches the root of phi to FP64 precision in
  fewer than 10 iterations at every pixel.
"""
import numpy as np
import pytest

import oracle
import synth

CASES = [(oracle.COMBINED, 358.0, 0.0104), (oracle.COMBINED, 160.0, 0.004), (oracle.LOG, 550.0, 0.0),
         (oracle.IDIV, 10.0, 0.0)]


@pytest.mark.parametrize("model,lam1,lam2", CASES)
def test_G_derivative_equals_prox_optimality(model, lam1, lam2):
    rng = np.random.default_rng(11)
    H, W = 6, 7
    f = rng.uniform(10.0, 255.0, (H, W))
    if model == oracle.IDIV:
        xh = f * np.exp(rng.normal(0.0, 0.3, (H, W)))
        tau = 0.02
    else:
        xh = np.log(f) + rng.normal(0.0, 0.5, (H, W))
        tau = 1e-3
    ws = oracle.prox(xh, f, tau, model, lam1, lam2)
    want = (xh - ws) / tau
    G = lambda w: oracle.energy_G(w, f, model, lam1, lam2)
    for p in range(H * W):
        e = np.zeros(H * W)
        h = 1e-4 * max(1.0, abs(ws.ravel()[p]))
        e[p] = h
        e = e.reshape(H, W)
        # fourth-order central difference
        d = (-G(ws + 2 * e) + 8 * G(ws + e) - 8 * G(ws - e) + G(ws - 2 * e)) / (12 * h)
        scale = max(abs(want.ravel()[p]), lam1 * 1e-3)
        assert abs(d - want.ravel()[p]) <= 1e-6 * scale, (p, d, want.ravel()[p])


def _steps(pr, bank, theta, iters, model=oracle.COMBINED):
    """(x_hat, f, alpha) of every accepted step of a seeded backtracking run."""
    p = oracle.Params(model=model, lam1=pr.lam1, lam2=pr.lam2 if model == oracle.COMBINED else 0.0)
    x, xp = oracle.init_state(pr.f, model)
    L = 1.0
    out = []
    for _ in range(iters):
        r = oracle.ipiano(p, pr.f, bank, theta, 1, L0=L, x_cur=x, x_prev=xp)
        L = float(r.L)
        alpha = 1.9 * (1.0 - 0.8) / L
        g = oracle.grad_F(x, bank, theta, model)
        out.append((x - alpha * g + 0.8 * (x - xp), alpha))
        x, xp = r.x, r.x_prev
    return out


@pytest.mark.parametrize("which", ["config1", "config2_crop", "config4_crop"])
def test_newton_fewer_than_ten_iterations(which):
    bank = synth.dct_bank()
    if which == "config1":
        pr, theta = synth.config1(), synth.theta_weights(1)
    elif which == "config2_crop":
        pr, theta = synth.config2(0, 64, 64), synth.theta_weights(2)
    else:
        pr, theta = synth.config4(0, 64, 64), synth.theta_weights(4)
    worst = 0
    for xh, alpha in _steps(pr, bank, theta, 6):
        _, it = oracle.prox(xh, pr.f, alpha, oracle.COMBINED, pr.lam1, pr.lam2, return_iters=True)
        worst = max(worst, it)
    print(f"{which}: at most {worst} Newton iterations per pixel")
    assert worst < 10
