"""Pins of the oracle's energies, gradient and prox (CPU only).

  * F and G against the dense brute force (explicit K_i matrices).
  * grad F against central differences of F (every pixel at 8x8; random
    directions on larger images), for the three models and boundary maps.
  * prox against a library minimiser of its defining objective (eq. (subproblem)),
    against the Lambert-W closed forms that exist when one of the two data
    terms is absent, nonexpansiveness and the bracket [what, log f].
  * I-divergence prox (the closed form printed in Sec. II-C) against the
    library minimiser and the quadratic it solves.
"""
import numpy as np
import pytest
import scipy.optimize as so
import scipy.special as sp

import oracle
import synth
from oracle import dense

MODELS = [oracle.COMBINED, oracle.LOG, oracle.IDIV]
BCS = [oracle.SYMMETRIC, oracle.ZERO, oracle.PERIODIC]


def _state(model, shape, seed=0):
    r = np.random.default_rng(seed)
    u = r.uniform(20, 240, shape)
    return np.log(u) if model != oracle.IDIV else u


@pytest.mark.parametrize("model", MODELS)
@pytest.mark.parametrize("bc", BCS)
def test_energy_and_gradient_match_dense(model, bc):
    H, W = 8, 8
    bank = synth.random_bank(11)[:6]
    theta = np.linspace(0.1, 0.5, 6)
    x = _state(model, (H, W))
    Ks = dense.k_matrices(H, W, bank, bc)
    assert oracle.energy_F(x, bank, theta, model, bc) == pytest.approx(dense.energy_F(x, Ks, theta, model), rel=1e-13)
    g = oracle.grad_F(x, bank, theta, model, bc)
    gd = dense.grad_F(x, Ks, theta, model)
    assert np.max(np.abs(g - gd)) <= 1e-12 * np.max(np.abs(gd))
    f = np.random.default_rng(5).uniform(20, 240, (H, W))
    lam1 = 10.0 if model == oracle.IDIV else 160.0
    assert oracle.energy_G(x, f, model, lam1, 0.004) == pytest.approx(dense.energy_G(x, f, model, lam1, 0.004),
                                                                       rel=1e-13)


def _fd_check(x, bank, theta, model, bc, dirs):
    """Fourth-order (Richardson) central differences of F along each direction."""
    g = oracle.grad_F(x, bank, theta, model, bc)
    h = 1e-5 * max(np.max(np.abs(x)), 1.0)
    for d in dirs:
        f1 = oracle.energy_F(x + h * d, bank, theta, model, bc) - oracle.energy_F(x - h * d, bank, theta, model, bc)
        f2 = oracle.energy_F(x + 2 * h * d, bank, theta, model, bc) - oracle.energy_F(x - 2 * h * d, bank, theta,
                                                                                     model, bc)
        fd = (8 * f1 - f2) / (12 * h)
        an = float(np.sum(g * d))
        assert abs(fd - an) <= 1e-7 * max(abs(an), np.linalg.norm(g) * np.linalg.norm(d) * 1e-2), (fd, an)


@pytest.mark.parametrize("model", MODELS)
@pytest.mark.parametrize("bc", BCS)
def test_gradient_every_pixel_finite_differences(model, bc):
    H, W = 8, 8
    bank = synth.dct_bank()
    theta = synth.theta_weights(1)
    x = _state(model, (H, W), seed=1)
    dirs = []
    for j in range(H * W):
        e = np.zeros(H * W); e[j] = 1.0
        dirs.append(e.reshape(H, W))
    _fd_check(x, bank, theta, model, bc, dirs)


@pytest.mark.parametrize("model", MODELS)
def test_gradient_random_directions_large(model):
    H, W = 61, 47
    bank = synth.random_bank(12)
    theta = synth.theta_weights(2)
    x = _state(model, (H, W), seed=2)
    r = np.random.default_rng(9)
    _fd_check(x, bank, theta, model, oracle.SYMMETRIC, [r.standard_normal((H, W)) for _ in range(3)])


def test_rho_derivative_finite_differences():
    # rho(x) = log(1 + x^2), rho'(x) = 2x / (1 + x^2) (Sec. II-A / II-C); a one-filter,
    # one-pixel-support image reduces the gradient to theta * rho'(y) * k.
    H, W = 8, 8
    k = np.zeros((7, 7)); k[3, 3] = 1.0  # identity filter: K = I
    for y0 in [-30.0, -1.0, -0.2, 0.0, 0.5, 2.0, 100.0]:
        u = np.full((H, W), y0)
        g = oracle.grad_F(u, k[None], np.array([0.7]), oracle.IDIV, oracle.ZERO)
        assert np.allclose(g, 0.7 * 2 * y0 / (1 + y0 * y0), rtol=1e-14, atol=1e-15)
        h = 1e-6 * max(1.0, abs(y0))
        num = (np.log1p((y0 + h) ** 2) - np.log1p((y0 - h) ** 2)) / (2 * h)
        assert abs(num - 2 * y0 / (1 + y0 * y0)) <= 1e-8 * max(1.0, abs(num))


# ------------------------------------------------------------------ prox
def _prox_objective(w, what, f, tau, model, lam1, lam2):
    f2 = f * f
    if model == oracle.IDIV:
        return 0.5 * (w - what) ** 2 + tau * 0.5 * lam1 * (w * w - 2 * f2 * np.log(w))
    g = 0.5 * lam1 * (2 * w + f2 * np.exp(-2 * w))
    if model == oracle.COMBINED:
        g += 0.5 * lam2 * (np.exp(2 * w) - 2 * f2 * w)
    return 0.5 * (w - what) ** 2 + tau * g


@pytest.mark.parametrize("model,lam1,lam2", [(oracle.COMBINED, 160.0, 0.004), (oracle.COMBINED, 550.0, 0.02),
                                             (oracle.LOG, 310.0, 0.0), (oracle.IDIV, 10.0, 0.0)])
def test_prox_minimises_its_objective(model, lam1, lam2):
    r = np.random.default_rng(4)
    n = 40
    f = r.uniform(5, 400, n)
    tau = 10 ** r.uniform(-6, -1, n)
    if model == oracle.IDIV:
        what = r.uniform(-100, 400, n)
    else:
        what = np.log(f) + r.uniform(-3, 3, n)
    for j in range(n):
        out = oracle.prox(np.array([what[j]]), np.array([f[j]]), tau[j], model, lam1, lam2)[0]
        lo = 1e-9 if model == oracle.IDIV else min(what[j], np.log(f[j])) - 1
        hi = max(what[j], np.log(f[j]) if model != oracle.IDIV else f[j]) + 1 + abs(what[j])
        res = so.minimize_scalar(_prox_objective, bounds=(lo, hi), method="bounded",
                                 args=(what[j], f[j], tau[j], model, lam1, lam2),
                                 options=dict(xatol=1e-12, maxiter=2000))
        # the oracle's value is at least as good as the library minimiser's, and close to it
        assert _prox_objective(out, what[j], f[j], tau[j], model, lam1, lam2) <= res.fun + 1e-9 * (1 + abs(res.fun))
        assert abs(out - res.x) <= 1e-5 * max(1.0, abs(res.x))


def test_prox_log_model_lambert_w():
    """lam2 = 0: w* = a + W0(2 tau lam1 f^2 e^{-2a}) / 2 with a = what - tau lam1 (from eq. (subproblem);
    the paper names the Lambert W route in Sec. II-C)."""
    r = np.random.default_rng(6)
    f = r.uniform(5, 300, 500)
    what = np.log(f) + r.uniform(-4, 4, 500)
    tau = 10 ** r.uniform(-5, 0, 500)
    lam1 = 160.0
    got = np.array([oracle.prox(what[j:j + 1], f[j:j + 1], tau[j], oracle.LOG, lam1, 0.0)[0] for j in range(500)])
    a = what - tau * lam1
    ref = a + 0.5 * np.real(sp.lambertw(2 * tau * lam1 * f * f * np.exp(-2 * a)))
    assert np.max(np.abs(got - ref) / np.maximum(1, np.abs(ref))) <= 1e-12


def test_prox_combined_lam1_zero_lambert_w():
    """lam1 = 0: w* = a - W0(2 tau lam2 e^{2a}) / 2 with a = what + tau lam2 f^2."""
    r = np.random.default_rng(7)
    f = r.uniform(5, 300, 300)
    what = np.log(f) + r.uniform(-2, 2, 300)
    tau = 10 ** r.uniform(-6, -3, 300)
    lam2 = 0.02
    got = np.array([oracle.prox(what[j:j + 1], f[j:j + 1], tau[j], oracle.COMBINED, 0.0, lam2)[0]
                    for j in range(300)])
    a = what + tau * lam2 * f * f
    ref = a - 0.5 * np.real(sp.lambertw(2 * tau * lam2 * np.exp(2 * a)))
    assert np.max(np.abs(got - ref) / np.maximum(1, np.abs(ref))) <= 1e-12


def test_prox_nonexpansive_and_bracketed():
    r = np.random.default_rng(8)
    n = 2000
    f = np.full(n, 87.0)
    what = np.log(87.0) + r.uniform(-5, 5, n)
    out = oracle.prox(what, f, 3e-3, oracle.COMBINED, 160.0, 0.004)
    lo = np.minimum(what, np.log(f)); hi = np.maximum(what, np.log(f))
    assert np.all(out >= lo) and np.all(out <= hi)
    order = np.argsort(what)
    assert np.all(np.diff(out[order]) >= 0)                             # monotone
    assert np.all(np.diff(out[order]) <= np.diff(what[order]) + 1e-15)  # 1-Lipschitz


def test_prox_idiv_closed_form():
    """Sec. II-C prints u_p = (uhat + sqrt(uhat^2 + 4 (1 + tau lam) tau lam f^2)) / (2 (1 + tau lam))."""
    r = np.random.default_rng(10)
    n = 1000
    f = r.uniform(1, 300, n)
    uh = r.uniform(-500, 500, n)
    tau, lam = 0.05, 10.0
    out = oracle.prox(uh, f, tau, oracle.IDIV, lam, 0.0)
    a = 1 + tau * lam
    assert np.all(out > 0)
    resid = a * out * out - uh * out - tau * lam * f * f
    assert np.max(np.abs(resid) / (a * out * out + np.abs(uh * out) + tau * lam * f * f)) <= 1e-14
    pos = uh >= 0
    printed = (uh + np.sqrt(uh * uh + 4 * a * tau * lam * f * f)) / (2 * a)
    assert np.max(np.abs(out[pos] - printed[pos]) / printed[pos]) <= 1e-14
