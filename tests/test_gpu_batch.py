"""Batched solver: one fused launch over the tiles of many uneven images per trial.

  * each image of a batch gives bitwise the same iterates, stats and output as a
    single-image solver on that image (same tile configuration): the per-tile work and the
    per-image reductions are identical;
  * images of a batch against the FP64 oracle (free-running backtracking: final PSNR within
    0.05 dB, the bound of the single-image backtracking runs), and the first four images of the
    seeded uneven batch (sides up to 960) over 300 iterations against stored oracle runs;
  * the tile-shape autotuner picks a valid configuration, caches it, and results under the
    other tile configuration stay at the parity bar.
"""
import json
import os

import numpy as np
import pytest

import oracle
import synth
from gpu_helpers import make_solver, torch_dev

pytestmark = pytest.mark.gpu

SIZES = [(64, 96), (128, 128), (70, 45), (200, 130), (33, 257), (128, 64)]
LOOKS = [1, 2, 4, 8, 1, 4]


def _problems():
    return [synth.config3_image(i, H, W, L) for i, ((H, W), L) in enumerate(zip(SIZES, LOOKS))]


def test_batch_equals_single_image_solves():
    import paper_1404_5344_amd as foe
    torch, dev = torch_dev()
    probs = _problems()
    bank, theta = synth.dct_bank(), synth.theta_weights(3)
    iters = 40
    p = foe.default_params(0, 0, max_iters=iters)
    b = foe.BatchSolver(p, SIZES, LOOKS, bank, theta)
    f = b.pack([torch.from_numpy(pr.f) for pr in probs]).to(dev)
    out, sums, stats, st = b.solve(f)
    outs = b.unpack(out)
    for i, pr in enumerate(probs):
        s = make_solver(pr.f.shape[0], pr.f.shape[1], bank, theta, max_iters=iters, looks=pr.looks)
        r = s.solve(torch.from_numpy(pr.f).to(dev))
        assert torch.equal(r.u, outs[i]), i
        assert np.array_equal(r.stats, stats[i]), i
        assert sums[i]["iters_done"] == iters
        s.close()
    b.close()


def test_batch_image_against_oracle():
    import paper_1404_5344_amd as foe
    torch, dev = torch_dev()
    probs = _problems()
    bank, theta = synth.dct_bank(), synth.theta_weights(3)
    iters = 30
    p = foe.default_params(0, 0, max_iters=iters)
    b = foe.BatchSolver(p, SIZES, LOOKS, bank, theta)
    out, sums, stats, st = b.solve(b.pack([torch.from_numpy(pr.f) for pr in probs]).to(dev))
    outs = b.unpack(out)
    for i in (2, 4):   # the two images with ragged tiles
        pr = probs[i]
        ref = oracle.ipiano(oracle.Params(lam1=pr.lam1, lam2=pr.lam2), pr.f, bank, theta, iters, L0=1.0)
        d = abs(synth.psnr(outs[i].cpu().numpy(), pr.clean) - synth.psnr(ref.u(), pr.clean))
        same_L = bool(np.array_equal(stats[i][:, 2], ref.stats[:, 2]))
        print(f"batch image {i} {SIZES[i]}: PSNR diff {d:.4f} dB, same L sequence {same_L}")
        assert d <= 0.05, (i, d)
    b.close()


def test_autotuner_and_tile_configs(tmp_path):
    import paper_1404_5344_amd as foe
    torch, dev = torch_dev()
    os.environ["FOE_TUNE_CACHE"] = str(tmp_path / "tune.txt")
    try:
        probs = _problems()
        bank, theta = synth.dct_bank(), synth.theta_weights(3)
        p = foe.default_params(0, 0, max_iters=20)
        b = foe.BatchSolver(p, SIZES, LOOKS, bank, theta)
        f = b.pack([torch.from_numpy(pr.f) for pr in probs]).to(dev)
        c = b.autotune(f, reps=2)
        assert c in (0, 1, 2, 3)
        assert (tmp_path / "tune.txt").read_text().strip().endswith(str(c))
        # a fixed step removes accept/reject decisions, so the tile shapes differ only in floating-point
        # summation order
        pf = foe.default_params(0, 0, max_iters=20, step_mode=1, alpha_fixed=2e-6)
        bf = foe.BatchSolver(pf, SIZES, LOOKS, bank, theta)
        res = {}
        for cfg in (0, 1, 2, 3):
            bf.set_tile_config(cfg)
            out, sums, stats, st = bf.solve(f)
            res[cfg] = out.cpu().numpy()
        assert np.max(np.abs(res[0] - res[1]) / res[0]) <= 1e-5
        assert np.max(np.abs(res[0] - res[2]) / res[0]) <= 1e-5
        assert np.max(np.abs(res[0] - res[3]) / res[0]) <= 1e-5
        bf.close()
        # the BF16 engine's strips take 32-column tiles of 16-row blocks: no 32 x 8 or 64 x 8 tiles
        pb = foe.default_params(0, 0, max_iters=20, precision=1)
        bb = foe.BatchSolver(pb, SIZES, LOOKS, bank, theta)
        for cfg in (2, 3):
            with pytest.raises(RuntimeError):
                bb.set_tile_config(cfg)
        assert bb.autotune(f, reps=2) in (0, 1)
        bb.close()
        # a second tuner call hits the cache, and so does another batch in the same size bucket (other
        # sizes, the same count of 32 x 32 tiles up to a power of two): no new cache line
        assert b.autotune(f, reps=2) == c
        sizes2 = SIZES[:-1] + [(120, 64)]
        probs2 = [synth.config3_image(i, H, W, L) for i, ((H, W), L) in enumerate(zip(sizes2, LOOKS))]
        b2 = foe.BatchSolver(p, sizes2, LOOKS, bank, theta)
        f2 = b2.pack([torch.from_numpy(pr.f) for pr in probs2]).to(dev)
        n_lines = len((tmp_path / "tune.txt").read_text().strip().splitlines())
        assert b2.autotune(f2, reps=2) == c
        assert len((tmp_path / "tune.txt").read_text().strip().splitlines()) == n_lines
        b2.close()
        # a single image is a bucket of its own
        s1 = make_solver(64, 96, bank, theta, max_iters=20)
        c1 = s1.autotune(torch.from_numpy(probs[0].f).to(dev), reps=2)
        assert c1 in (0, 1, 2, 3)
        lines = (tmp_path / "tune.txt").read_text().strip().splitlines()
        assert len(lines) == n_lines + 1 and "_single" in lines[-1] and "_batch" in lines[0]
        s1.close()
        b.close()
    finally:
        del os.environ["FOE_TUNE_CACHE"]


def test_uneven_batch_against_stored_oracle_runs():
    """The first four images of the seeded uneven batch, 300 iterations each, in one batch against the stored
    FP64 oracle runs (tests/golden/config3_oracle.json): final PSNR within 0.05 dB, the largest absolute error
    on the stored output sample stated."""
    import paper_1404_5344_amd as foe
    torch, dev = torch_dev()
    ref = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "config3_oracle.json")))
    imgs = ref["images"]
    sizes = [(im["H"], im["W"]) for im in imgs]
    looks = [im["looks"] for im in imgs]
    probs = [synth.config3_image(im["index"], im["H"], im["W"], im["looks"]) for im in imgs]
    bank, theta = synth.dct_bank(), synth.theta_weights(3)
    b = foe.BatchSolver(foe.default_params(0, 0, max_iters=300), sizes, looks, bank, theta)
    out, sums, stats, st = b.solve(b.pack([torch.from_numpy(pr.f) for pr in probs]).to(dev))
    outs = b.unpack(out)
    for i, (pr, im) in enumerate(zip(probs, imgs)):
        u = outs[i].cpu().numpy()
        d = abs(synth.psnr(u, pr.clean) - im["psnr_final"])
        err = np.abs(u.ravel()[im["u_sample_idx"]].astype(np.float64) - np.array(im["u_sample"]))
        H = stats[i][-1, 0] + stats[i][-1, 1]
        H_ora = im["F"][-1] + im["G"][-1]
        print(f"batch image {i} {im['H']}x{im['W']} L={im['looks']}: PSNR {synth.psnr(u, pr.clean):.4f} vs oracle "
              f"{im['psnr_final']:.4f} (diff {d:.4f} dB), energy rel diff {abs(H - H_ora) / abs(H_ora):.2e}, "
              f"max abs err on {err.size} sampled pixels {err.max():.3e}")
        assert sums[i]["iters_done"] == 300
        assert d <= 0.05, (i, d)
    b.close()


def test_per_image_latency_from_device_timestamps():
    """foe_batch_latency: every image of a batch completes after a positive time and no later than the whole
    iteration loop (the solver's event pair around it, with a little slack), the last one after at least half
    of it; a single-image solve reports about its loop time."""
    import paper_1404_5344_amd as foe
    torch, dev = torch_dev()
    probs = _problems()
    bank, theta = synth.dct_bank(), synth.theta_weights(3)
    p = foe.default_params(0, 0, max_iters=60)
    b = foe.BatchSolver(p, SIZES, LOOKS, bank, theta)
    f = b.pack([torch.from_numpy(pr.f) for pr in probs]).to(dev)
    b.solve(f)
    lat = b.latency()
    loop_ms, launches = b.last_timing()
    print("latency ms per image:", np.round(lat, 4), "loop", round(loop_ms, 4), "ms over", launches, "launches")
    assert lat.shape == (len(SIZES),)
    assert np.all(lat > 0.0)
    assert np.all(lat <= loop_ms * 1.05 + 0.1)
    assert lat.max() >= 0.5 * loop_ms
    b.close()
    pr = probs[1]
    s = make_solver(pr.f.shape[0], pr.f.shape[1], bank, theta, max_iters=60, looks=pr.looks)
    s.solve(torch.from_numpy(pr.f).to(dev))
    (one,) = s.latency()
    loop_ms, _ = s.last_timing()
    print("single image latency", one, "loop", loop_ms)
    assert 0.5 * loop_ms <= one <= loop_ms * 1.05 + 0.1
    s.close()
