"""The FP64 oracle under AddressSanitizer + UndefinedBehaviorSanitizer (CPU only).

oracle/sanitize_main.c calls every exported oracle routine on small seeded inputs (sides from 1 to 16,
all boundary conditions and data models, both step modes, the warm-start network) and checks one property
per operator; the build aborts on the first memory error or undefined behaviour.  Plus a pin of the
symmetric boundary map on sides below the filter radius against numpy's own symmetric padding.
"""
import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = [os.path.join(ROOT, "oracle", n) for n in ("sanitize_main.c", "foe_oracle.c", "cnn_oracle.c")]


def _sanitizer_build(tmp_path):
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    exe = str(tmp_path / "oracle_san")
    cmd = ["gcc", "-std=c11", "-g", "-O1", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           "-fno-omit-frame-pointer", "-Wall", "-Wno-unknown-pragmas", "-o", exe] + SRC + ["-lm"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0 and ("libasan" in r.stderr or "libubsan" in r.stderr):
        pytest.skip("sanitizer runtime not installed: " + r.stderr[-200:])
    assert r.returncode == 0, r.stderr
    return exe


def test_oracle_clean_under_asan_and_ubsan(tmp_path):
    exe = _sanitizer_build(tmp_path)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    env.pop("LD_PRELOAD", None)
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    out = r.stdout + r.stderr
    print(out[-2000:])
    assert "AddressSanitizer" not in out and "runtime error" not in out and "LeakSanitizer" not in out
    assert r.returncode == 0
    assert "0 failures" in r.stdout


@pytest.mark.parametrize("shape", [(1, 1), (1, 6), (2, 5), (3, 2), (5, 4)])
def test_symmetric_map_on_sides_below_the_radius(shape):
    """y = K x with the half-sample symmetric extension equals the valid correlation of numpy's symmetric
    padding by 3 (which reflects repeatedly when the side is smaller than the padding)."""
    rng = np.random.default_rng(sum(shape))
    H, W = shape
    x = rng.standard_normal((H, W))
    k = rng.standard_normal((7, 7))
    xp = np.pad(x, 3, mode="symmetric")
    ref = np.zeros((H, W))
    for py in range(H):
        for px in range(W):
            # y(p) = sum_{a,b} k[a][b] x_ext(p + 3 - a, p + 3 - b); padded index = extended index + 3
            ref[py, px] = sum(k[a, b] * xp[py + 6 - a, px + 6 - b] for a in range(7) for b in range(7))
    np.testing.assert_allclose(oracle.forward(x, k, oracle.SYMMETRIC), ref, rtol=1e-12, atol=1e-12)
