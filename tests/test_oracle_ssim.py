"""Pins of the FP64 SSIM oracle against what its definition fixes."""
import math

import numpy as np

import oracle
from oracle import quality as S


def _brute(x, y, peak=255.0):
    """The same index by explicit loops over windows and taps (no vectorisation)."""
    w = S.gaussian_window()
    H, W = x.shape
    c1, c2 = (0.01 * peak) ** 2, (0.03 * peak) ** 2
    vals = []
    for i in range(H - 10):
        for j in range(W - 10):
            mx = my = sxx = syy = sxy = 0.0
            for a in range(11):
                for b in range(11):
                    xv, yv, wv = x[i + a, j + b], y[i + a, j + b], w[a, b]
                    mx += wv * xv; my += wv * yv
                    sxx += wv * xv * xv; syy += wv * yv * yv; sxy += wv * xv * yv
            vx, vy, cxy = sxx - mx * mx, syy - my * my, sxy - mx * my
            vals.append(((2 * mx * my + c1) * (2 * cxy + c2)) / ((mx * mx + my * my + c1) * (vx + vy + c2)))
    return float(np.mean(vals))


def test_window_is_the_normalised_gaussian():
    w = S.gaussian_window()
    assert w.shape == (11, 11)
    assert abs(w.sum() - 1.0) < 1e-15
    assert abs(w[5, 6] / w[5, 5] - math.exp(-1.0 / (2 * 1.5 ** 2))) < 1e-14
    assert np.allclose(w, w.T)


def test_identical_images_give_one():
    x = np.random.default_rng(0).uniform(0, 255, (40, 37))
    assert abs(oracle.ssim(x, x) - 1.0) < 1e-12


def test_constant_images_closed_form():
    mx, my = 80.0, 120.0
    x, y = np.full((20, 25), mx), np.full((20, 25), my)
    c1 = (0.01 * 255) ** 2
    assert abs(oracle.ssim(x, y) - (2 * mx * my + c1) / (mx * mx + my * my + c1)) < 1e-12


def test_against_brute_force_loops():
    r = np.random.default_rng(1)
    x = r.uniform(0, 255, (16, 19))
    y = np.clip(x + r.normal(0, 30, x.shape), 0, 255)
    assert abs(oracle.ssim(x, y) - _brute(x, y)) < 1e-12


def test_symmetric_and_bounded():
    r = np.random.default_rng(2)
    x = r.uniform(0, 255, (30, 30))
    y = r.uniform(0, 255, (30, 30))
    assert abs(oracle.ssim(x, y) - oracle.ssim(y, x)) < 1e-14
    assert oracle.ssim(x, y) <= 1.0
