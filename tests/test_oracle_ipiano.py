"""Pins of the oracle's iPiano loop (CPU only).

iPiano's update (Sec. II-C, eq. (fplusg)): x+ = prox_{aG}(x - a grad F(x) + b (x - x_prev)).
  * Special cases: G = 0 reduces it to the heavy-ball method, b = 0 to the
    proximal gradient method; both are run here as textbook loops on the dense
    brute-force gradient.
  * Every accepted backtracking step satisfies the descent-lemma test and L
    never decreases when eta_down = 1.
  * Lyapunov decrease: with d = x+ - x, m = x - x_prev, delta = b/(2a) and
    gamma = (1-b)/a - L/2 > 0, convexity of G (Sec. II-B: the data terms are
    convex in w, eq. (newmodel) stays convex) and the descent inequality give
    H(x+) + delta |d|^2 <= H(x) + delta |m|^2 - gamma |d|^2.
  * Stationarity: the prox-gradient residual goes to zero.
  * Convex regime (I-divergence model with lam > lam_max(sum theta K^T K)/4,
    since rho'' >= -1/4): the limit is the unique minimiser, found here by L-BFGS-B.
"""
import numpy as np
import pytest
import scipy.optimize as so

import oracle
import synth
from oracle import dense


def _small_problem(H=32, W=32, looks=4, seed=0):
    clean = synth.shapes_image(90, seed, H, W)
    f = synth.speckle(clean, looks, 90, seed)
    return clean, f.astype(np.float64)


def test_heavy_ball_special_case():
    H, W = 8, 8
    bank = synth.random_bank(21)[:8]
    theta = np.linspace(0.05, 0.5, 8)
    f = np.random.default_rng(0).uniform(30, 200, (H, W))
    Ks = dense.k_matrices(H, W, bank, oracle.SYMMETRIC)
    p = oracle.Params(model=oracle.LOG, lam1=0.0, lam2=0.0, beta=0.6, step_mode=oracle.FIXED, alpha_fixed=1e-4)
    res = oracle.ipiano(p, f, bank, theta, 25)
    x = np.log(f); xp = x.copy()
    for _ in range(25):
        xn = x - p.alpha_fixed * dense.grad_F(x, Ks, theta, oracle.LOG) + p.beta * (x - xp)
        xp, x = x, xn
    assert np.max(np.abs(res.x - x)) <= 1e-12 * np.max(np.abs(x))
    assert np.max(np.abs(res.x_prev - xp)) <= 1e-12 * np.max(np.abs(x))


def test_proximal_gradient_special_case():
    H, W = 8, 8
    bank = synth.dct_bank()
    theta = synth.theta_weights(3)
    f = np.random.default_rng(1).uniform(30, 200, (H, W))
    Ks = dense.k_matrices(H, W, bank, oracle.SYMMETRIC)
    p = oracle.Params(model=oracle.IDIV, lam1=2.0, lam2=0.0, beta=0.0, step_mode=oracle.FIXED, alpha_fixed=0.01)
    res = oracle.ipiano(p, f, bank, theta, 10)
    u = f.copy()
    a, lam = p.alpha_fixed, p.lam1
    for _ in range(10):
        uh = u - a * dense.grad_F(u, Ks, theta, oracle.IDIV)
        # closed-form prox printed in Sec. II-C (uhat > 0 throughout this run)
        assert np.all(uh > 0)
        u = (uh + np.sqrt(uh * uh + 4 * (1 + a * lam) * a * lam * f * f)) / (2 * (1 + a * lam))
    assert np.max(np.abs(res.x - u)) <= 1e-12 * np.max(np.abs(u))


@pytest.fixture(scope="module")
def backtracking_run():
    clean, f = _small_problem()
    bank = synth.dct_bank()
    theta = synth.theta_weights(1)
    l1, l2 = synth.default_lambdas(4)
    p = oracle.Params(model=oracle.COMBINED, lam1=l1, lam2=l2, beta=0.8)
    x0, _ = oracle.init_state(f)
    H0 = oracle.energy_F(x0, bank, theta) + oracle.energy_G(x0, f, oracle.COMBINED, l1, l2)
    res = oracle.ipiano(p, f, bank, theta, 80, L0=1.0)
    return p, res, H0, clean, f


def test_line_search_invariants(backtracking_run):
    p, res, H0, clean, f = backtracking_run
    assert res.status == oracle.OK
    st = res.stats
    F = st[:, 0]; L = st[:, 2]; s1 = st[:, 5]; s2 = st[:, 6]
    Fprev = np.concatenate([[H0 - oracle.energy_G(np.log(f), f, oracle.COMBINED, p.lam1, p.lam2)], F[:-1]])
    assert np.all(F <= Fprev + s1 + 0.5 * L * s2)
    assert np.all(np.diff(L) >= 0)
    assert np.all(st[:, 4] >= 1)
    assert np.allclose(st[:, 3], 1.9 * (1 - p.beta) / L, rtol=1e-15)


def test_lyapunov_decrease(backtracking_run):
    p, res, H0, clean, f = backtracking_run
    st = res.stats
    H = st[:, 0] + st[:, 1]
    Hprev = np.concatenate([[H0], H[:-1]])
    alpha, L, s2, m = st[:, 3], st[:, 2], st[:, 6], st[:, 7]
    delta = p.beta / (2 * alpha)
    gamma = (1 - p.beta) / alpha - L / 2
    assert np.all(gamma > 0)
    lhs = H + delta * s2
    rhs = Hprev + delta * m - gamma * s2
    assert np.all(lhs <= rhs + 1e-12 * np.abs(Hprev))
    assert H[-1] < H0
    # the despeckled output is closer to the clean image than the observation is
    assert synth.psnr(res.u(), clean) > synth.psnr(f, clean) + 3.0


def test_fixed_step_lyapunov_chain_idiv():
    """FIXED mode, I-divergence model, a < 2(1-b)/L_hat with L_hat a global Lipschitz bound of grad F:
    the chained H_delta(x^n, x^{n-1}) = H(x^n) + delta |x^n - x^{n-1}|^2 is non-increasing."""
    H, W = 24, 24
    clean, f = _small_problem(H, W, looks=4, seed=3)
    bank = synth.dct_bank(); theta = synth.theta_weights(1)
    # rho'' in [-1/4, 2] => |grad^2 F| <= 2 * lam_max(sum theta K^T K) <= 2 * 49 * theta_max (periodic, DCT bank)
    L_hat = 2 * 49 * float(theta.max()) * 1.01
    beta = 0.8
    alpha = 1.9 * (1 - beta) / L_hat
    p = oracle.Params(model=oracle.IDIV, boundary=oracle.PERIODIC, lam1=10.0, beta=beta, step_mode=oracle.FIXED,
                      alpha_fixed=alpha)
    res = oracle.ipiano(p, f, bank, theta, 60)
    st = res.stats
    Hn = st[:, 0] + st[:, 1]
    delta = beta / (2 * alpha)
    Hd = Hn + delta * st[:, 6]
    H0 = oracle.energy_F(f, bank, theta, oracle.IDIV, oracle.PERIODIC) + oracle.energy_G(f, f, oracle.IDIV, 10.0, 0)
    assert np.all(np.diff(np.concatenate([[H0], Hd])) <= 1e-12 * abs(H0))


def test_stationarity_residual_vanishes():
    H, W = 8, 8
    f = np.random.default_rng(4).uniform(40, 200, (H, W))
    bank = synth.dct_bank(); theta = synth.theta_weights(4)
    p = oracle.Params(model=oracle.COMBINED, lam1=358.0, lam2=0.0104, beta=0.8)
    oracle.set_threads(1)
    try:
        res = oracle.ipiano(p, f, bank, theta, 4000, L0=1.0)
    finally:
        oracle.set_threads(0)
    assert res.status == oracle.OK
    a = 1.9 * (1 - p.beta) / res.L
    g = oracle.grad_F(res.x, bank, theta)
    r = np.max(np.abs(res.x - oracle.prox(res.x - a * g, f, a, oracle.COMBINED, p.lam1, p.lam2))) / a
    g0 = oracle.grad_F(np.log(f), bank, theta)
    r0 = np.max(np.abs(np.log(f) - oracle.prox(np.log(f) - a * g0, f, a, oracle.COMBINED, p.lam1, p.lam2))) / a
    assert r <= 1e-8 * max(1.0, r0)


def test_convex_regime_unique_minimiser():
    H, W = 8, 8
    f = np.random.default_rng(5).uniform(40, 200, (H, W))
    bank = synth.dct_bank(); theta = synth.theta_weights(5)
    lam = 10.0
    Ks = dense.k_matrices(H, W, bank, oracle.PERIODIC)
    A = sum(t * K.T @ K for K, t in zip(Ks, theta))
    assert lam > 0.25 * np.linalg.eigvalsh(A).max()       # strict convexity certificate
    p = oracle.Params(model=oracle.IDIV, boundary=oracle.PERIODIC, lam1=lam, beta=0.8)
    oracle.set_threads(1)
    try:
        res = oracle.ipiano(p, f, bank, theta, 3000, L0=1.0)
    finally:
        oracle.set_threads(0)

    def fun(u):
        u2 = u.reshape(H, W)
        e = dense.energy_F(u2, Ks, theta, oracle.IDIV) + dense.energy_G(u2, f, oracle.IDIV, lam, 0.0)
        g = dense.grad_F(u2, Ks, theta, oracle.IDIV) + lam * (u2 - f * f / u2)
        return e, g.ravel()

    opt = so.minimize(fun, f.ravel(), jac=True, method="L-BFGS-B", bounds=[(1e-6, None)] * (H * W),
                      options=dict(ftol=1e-15, gtol=1e-11, maxiter=20000))
    assert np.max(np.abs(res.x.ravel() - opt.x)) <= 1e-7 * np.max(np.abs(opt.x))


def test_thread_count_independence_and_resume():
    clean, f = _small_problem(40, 36, looks=1, seed=6)
    bank = synth.dct_bank(); theta = synth.theta_weights(1)
    p = oracle.Params(model=oracle.COMBINED, lam1=160.0, lam2=0.004, beta=0.8)
    oracle.set_threads(1)
    a = oracle.ipiano(p, f, bank, theta, 8)
    oracle.set_threads(4)
    b = oracle.ipiano(p, f, bank, theta, 8)
    c1 = oracle.ipiano(p, f, bank, theta, 5)
    c2 = oracle.ipiano(p, f, bank, theta, 3, L0=c1.L, x_cur=c1.x, x_prev=c1.x_prev)
    oracle.set_threads(0)
    assert np.array_equal(a.x, b.x) and np.array_equal(a.stats, b.stats)
    assert np.array_equal(a.x, c2.x) and np.array_equal(a.stats[5:], c2.stats)


def test_line_search_exhaustion_status():
    clean, f = _small_problem(16, 16, looks=1, seed=7)
    bank = synth.dct_bank(); theta = synth.theta_weights(1)
    p = oracle.Params(model=oracle.COMBINED, lam1=160.0, lam2=0.004, beta=0.8, max_backtracks=0)
    res = oracle.ipiano(p, f, bank, theta, 5, L0=1e-6)
    assert res.status == oracle.ELINESEARCH
    assert np.array_equal(res.x, np.log(f.astype(np.float64)))   # left at the last accepted iterate


def test_nonfinite_status():
    """A trial whose energy overflows (weights theta_i = 1e300: F sums 1e300 log(1 + y^2) over the image) ends
    the run with ENONFINITE in the fixed-step mode, before any iterate is taken; under backtracking such a trial
    is rejected like any other and the line search runs out."""
    clean, f = _small_problem(16, 16, looks=1, seed=9)
    bank = synth.dct_bank()
    theta = np.full(len(bank), 1e300)
    x0 = np.log(f.astype(np.float64))
    p = oracle.Params(model=oracle.COMBINED, lam1=160.0, lam2=0.004, beta=0.8, step_mode=oracle.FIXED, alpha_fixed=1e-3)
    res = oracle.ipiano(p, f, bank, theta, 5)
    assert res.status == oracle.ENONFINITE
    assert np.array_equal(res.x, x0)
    pb = oracle.Params(model=oracle.COMBINED, lam1=160.0, lam2=0.004, beta=0.8, max_backtracks=3)
    res = oracle.ipiano(pb, f, bank, theta, 5, L0=1.0)
    assert res.status == oracle.ELINESEARCH
    assert np.array_equal(res.x, x0)
