"""The warm start's energy test (CPU only): the energy H = F + G is sign-indefinite (the lambda2 term of the
combined data term is negative on bright pixels), so the fallback margin is taken on |H_plain|."""
import os

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _rule():
    # warmstart.py imports the package (which needs torch, not the GPU); load it the same way
    from paper_1404_5344_amd import warmstart
    return warmstart


def test_fallback_margin_on_positive_and_negative_energies():
    ws = _rule()
    tol = ws.FALLBACK_TOL
    assert tol == 0.005
    # positive plain energy: up to +0.5 % is accepted
    assert not ws.needs_fallback(100.4, 100.0)
    assert ws.needs_fallback(100.6, 100.0)
    # negative plain energy: a higher (less negative) warm energy by more than 0.5 % of |H| falls back ...
    assert ws.needs_fallback(-99.4, -100.0)
    assert not ws.needs_fallback(-99.6, -100.0)
    # ... and a lower energy never does (a ratio test would have inverted both)
    assert not ws.needs_fallback(-150.0, -100.0)
    assert not ws.needs_fallback(50.0, 100.0)


def test_energy_gap_sign():
    ws = _rule()
    assert ws.energy_gap(101.0, 100.0) > 0
    assert ws.energy_gap(-99.0, -100.0) > 0        # higher energy: positive gap even for negative H
    assert ws.energy_gap(-101.0, -100.0) < 0
    assert abs(ws.energy_gap(-99.0, -100.0) - 0.01) < 1e-12
