"""Pins of the seeded input generators (CPU only).

The speckle generator follows the L-look Nakagami amplitude law (Sec. II-B).
Table 2 prints the PSNR of the speckled input for L = 8, 3, 1; the gaps between
those entries do not depend on the images, because the MSE of an L-look
amplitude is mean(c^2) * m_L with m_L = E[(sqrt(n) - 1)^2] = 2 - 2 Gamma(L + 1/2) / (Gamma(L) sqrt(L)),
n ~ Gamma(L, 1/L).
"""
import json
import math
import os

import numpy as np
import pytest

import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def m_L(L):
    return 2.0 - 2.0 * math.exp(math.lgamma(L + 0.5) - math.lgamma(L)) / math.sqrt(L)


def test_closed_form_gaps_match_table2():
    g = json.load(open(os.path.join(GOLDEN, "table2_noisy_psnr.json")))["psnr"]
    gap83 = g["8"] - g["3"]
    gap31 = g["3"] - g["1"]
    assert abs(10 * math.log10(m_L(3) / m_L(8)) - gap83) <= 0.01
    assert abs(10 * math.log10(m_L(1) / m_L(3)) - gap31) <= 0.01
    # the literal reading f = c * n does not reproduce the printed gaps
    v = lambda L: 1.0 / L  # E[(n - 1)^2] for n ~ Gamma(L, 1/L)
    miss = max(abs(10 * math.log10(v(3) / v(8)) - gap83), abs(10 * math.log10(v(1) / v(3)) - gap31))
    assert miss > 0.25


def test_generated_noisy_psnr_gaps_match_table2():
    g = json.load(open(os.path.join(GOLDEN, "table2_noisy_psnr.json")))["psnr"]
    clean = synth.shapes_cosine_image(2, 0, 512, 512)
    ps = {L: synth.psnr(synth.speckle(clean, L, 2, 0), clean) for L in (1, 3, 8)}
    assert abs((ps[8] - ps[3]) - (g["8"] - g["3"])) <= 0.03
    assert abs((ps[3] - ps[1]) - (g["3"] - g["1"])) <= 0.03


def test_lambda_table_matches_paper():
    t = json.load(open(os.path.join(GOLDEN, "lambda_table.json")))["synthetic"]
    for L, (l1, l2) in t.items():
        assert synth.default_lambdas(int(L)) == pytest.approx((l1, l2))
    assert synth.default_lambdas(4) == pytest.approx((358.0, 0.0104))
    assert synth.default_lambdas(2) == pytest.approx((235.0, 0.006))


def test_generators_are_seeded_and_positive():
    a = synth.config1().f
    b = synth.config1().f
    assert a.dtype == np.float32 and np.array_equal(a, b) and np.all(a > 0)
    c = synth.config4(0, 256, 256)
    assert c.clean.mean() == pytest.approx(100.0 * (1 + 39 * 0 / 1), rel=0.5)
    assert np.sum(c.clean >= 1999) >= 30
    sizes = synth.config3_sizes()
    assert len(sizes) == 64 and all(128 <= h <= 1024 and 128 <= w <= 1024 and L in (1, 2, 4, 8) for h, w, L in sizes)
