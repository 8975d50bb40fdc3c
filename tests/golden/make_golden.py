"""Write stored oracle results used by the GPU parity tests.

Calls only the FP64 oracle (oracle/) and the seeded generators (synth/).  Run:
    python tests/golden/make_golden.py [config2] [config3] [config4_<tile>] [sar_preset]
Each output records the generator recipe, the model parameters and the oracle's
per-iteration trajectory, so a test can compare without re-running a long oracle.
"""
from __future__ import annotations

import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle  # noqa: E402
import synth  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))


def config2(iters: int = 300):
    pr = synth.config2()
    bank = synth.dct_bank()
    theta = synth.theta_weights(2)
    p = oracle.Params(model=oracle.COMBINED, boundary=oracle.SYMMETRIC, lam1=pr.lam1, lam2=pr.lam2, beta=0.8)
    t = time.time()
    r = oracle.ipiano(p, pr.f, bank, theta, iters, L0=1.0)
    dt = time.time() - t
    u = r.u()
    out = {
        "what": "FP64 oracle, config 2: 512x512 shapes+cosine image, L = 1 speckle, COMBINED model, "
                "SYMMETRIC boundary, DCT bank, theta seed 2, backtracking (L0 = 1, eta_up = 2, eta_down = 1), "
                "beta = 0.8, 300 iterations",
        "status": r.status,
        "lam1": pr.lam1, "lam2": pr.lam2,
        "psnr_noisy": synth.psnr(pr.f, pr.clean),
        "psnr_final": synth.psnr(u, pr.clean),
        "F": r.stats[:, 0].tolist(), "G": r.stats[:, 1].tolist(), "L": r.stats[:, 2].tolist(),
        "trials": r.stats[:, 4].tolist(),
        "u_sample_idx": list(range(0, 512 * 512, 4099)),
        "u_sample": u.ravel()[::4099].tolist(),
        "oracle_seconds": dt, "oracle_threads": oracle.get_threads(),
    }
    with open(os.path.join(HERE, "config2_oracle.json"), "w") as fh:
        json.dump(out, fh)
    print("config2: psnr", out["psnr_noisy"], "->", out["psnr_final"], "in", dt, "s")


def sar_preset(iters: int = 300):
    """The real-SAR parameters of Sec. III-C (L = 5, lambda = (50, 0.15)) on a 256x256 SAR-like image, with a
    seeded learned-style bank (not zero-sum, norms 0.2-5, weights up to 5)."""
    pr = synth.sar_preset()
    bank, theta = synth.learned_style_bank(6)
    p = oracle.Params(model=oracle.COMBINED, boundary=oracle.SYMMETRIC, lam1=pr.lam1, lam2=pr.lam2, beta=0.8)
    t = time.time()
    r = oracle.ipiano(p, pr.f, bank, theta, iters, L0=1.0)
    dt = time.time() - t
    u = r.u()
    H, W = pr.f.shape
    sample = list(range(0, H * W, 257))
    targets = np.argsort(pr.clean.ravel())[-40:].tolist()
    idx = sorted(set(sample) | set(targets))
    out = {
        "what": "FP64 oracle, real-SAR preset of Sec. III-C: 256x256 SAR-like GRF image with 40 point targets "
                "(config id 6), L = 5 speckle, lambda = (50, 0.15), COMBINED model, SYMMETRIC boundary, "
                "learned-style bank (seed 6), backtracking (L0 = 1, eta_up = 2, eta_down = 1), beta = 0.8, "
                "300 iterations; PSNR peak = max of the clean image",
        "status": r.status,
        "lam1": pr.lam1, "lam2": pr.lam2, "peak": pr.peak,
        "psnr_noisy": synth.psnr(pr.f, pr.clean, pr.peak),
        "psnr_final": synth.psnr(u, pr.clean, pr.peak),
        "F": r.stats[:, 0].tolist(), "G": r.stats[:, 1].tolist(), "L": r.stats[:, 2].tolist(),
        "trials": r.stats[:, 4].tolist(),
        "u_sample_idx": idx, "u_sample": u.ravel()[idx].tolist(),
        "oracle_seconds": dt, "oracle_threads": oracle.get_threads(),
    }
    with open(os.path.join(HERE, "sar_preset_oracle.json"), "w") as fh:
        json.dump(out, fh)
    print("sar_preset: psnr", out["psnr_noisy"], "->", out["psnr_final"], "in", dt, "s, status", r.status, flush=True)


def config4(iters: int = 300, index: int = 0):
    pr = synth.config4(index)
    bank = synth.dct_bank()
    theta = synth.theta_weights(4)
    p = oracle.Params(model=oracle.COMBINED, boundary=oracle.SYMMETRIC, lam1=pr.lam1, lam2=pr.lam2, beta=0.8)
    t = time.time()
    r = oracle.ipiano(p, pr.f, bank, theta, iters, L0=1.0)
    dt = time.time() - t
    u = r.u()
    H, W = pr.f.shape
    sample = list(range(0, H * W, 4099))
    targets = np.argsort(pr.clean.ravel())[-40:].tolist()     # the 40 point targets
    idx = sorted(set(sample) | set(targets))
    out = {
        "what": f"FP64 oracle, config 4 tile {index}: {H}x{W} SAR-like GRF image with 40 point targets, L = 1 "
                "speckle, COMBINED model, SYMMETRIC boundary, DCT bank, theta seed 4, backtracking (L0 = 1, "
                "eta_up = 2, eta_down = 1), beta = 0.8, 300 iterations; PSNR peak = max of the clean image",
        "status": r.status,
        "lam1": pr.lam1, "lam2": pr.lam2, "peak": pr.peak,
        "psnr_noisy": synth.psnr(pr.f, pr.clean, pr.peak),
        "psnr_final": synth.psnr(u, pr.clean, pr.peak),
        "F": r.stats[:, 0].tolist(), "G": r.stats[:, 1].tolist(), "L": r.stats[:, 2].tolist(),
        "trials": r.stats[:, 4].tolist(),
        "u_sample_idx": idx,
        "u_sample": u.ravel()[idx].tolist(),
        "oracle_seconds": dt, "oracle_threads": oracle.get_threads(),
    }
    with open(os.path.join(HERE, f"config4_tile{index}_oracle.json"), "w") as fh:
        json.dump(out, fh)
    print("config4: psnr", out["psnr_noisy"], "->", out["psnr_final"], "in", dt, "s")


# the first four images of the seeded uneven batch (sides from {128, ..., 1024}, looks from {1, 2, 4, 8})
CONFIG3_IMAGES = 4


def config3(iters: int = 300):
    bank = synth.dct_bank()
    theta = synth.theta_weights(3)
    sizes = synth.config3_sizes()[:CONFIG3_IMAGES]
    images = []
    for i, (H, W, L) in enumerate(sizes):
        pr = synth.config3_image(i, H, W, L)
        p = oracle.Params(model=oracle.COMBINED, boundary=oracle.SYMMETRIC, lam1=pr.lam1, lam2=pr.lam2, beta=0.8)
        t = time.time()
        r = oracle.ipiano(p, pr.f, bank, theta, iters, L0=1.0)
        dt = time.time() - t
        u = r.u()
        idx = list(range(0, H * W, 997))
        images.append({
            "index": i, "H": H, "W": W, "looks": L, "status": r.status,
            "lam1": pr.lam1, "lam2": pr.lam2,
            "psnr_noisy": synth.psnr(pr.f, pr.clean),
            "psnr_final": synth.psnr(u, pr.clean),
            "F": r.stats[:, 0].tolist(), "G": r.stats[:, 1].tolist(), "L": r.stats[:, 2].tolist(),
            "trials": r.stats[:, 4].tolist(),
            "u_sample_idx": idx, "u_sample": u.ravel()[idx].tolist(),
            "oracle_seconds": dt,
        })
        print(f"config3 image {i} {H}x{W} L={L}: psnr {images[-1]['psnr_noisy']:.4f} -> "
              f"{images[-1]['psnr_final']:.4f} in {dt:.1f} s", flush=True)
    out = {
        "what": f"FP64 oracle, config 3: the first {CONFIG3_IMAGES} images of the seeded uneven batch "
                "(shapes+cosine generator, lambda from the looks), COMBINED model, SYMMETRIC boundary, DCT bank, "
                "theta seed 3, backtracking (L0 = 1, eta_up = 2, eta_down = 1), beta = 0.8, 300 iterations each",
        "images": images, "oracle_threads": oracle.get_threads(),
    }
    with open(os.path.join(HERE, "config3_oracle.json"), "w") as fh:
        json.dump(out, fh)


if __name__ == "__main__":
    which = sys.argv[1:] or ["config2"]
    for w in which:
        if w.startswith("config4_"):
            config4(index=int(w.split("_")[1]))
        else:
            globals()[w]()
