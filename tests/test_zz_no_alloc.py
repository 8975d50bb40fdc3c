"""The allocation-free entry point (foe_solve_noalloc) against foe_solve through the C ABI.

The two run the same kernels in the same order on the same inputs, so u, the per-iteration stats and the
summary must agree bit for bit.  Two calls in a row, the second on a smaller image with other looks and
iteration count, check that the shared workspace keeps nothing from one call that the next one reads.
"""
import numpy as np
import pytest

import synth
from gpu_helpers import torch_dev

pytestmark = pytest.mark.gpu


def _reference(foe, p, bank, theta, f):
    with foe.Solver(p, bank, theta) as s:
        r = s.solve(f)
        u = r.u.clone()
    return u, r.summary, r.stats


@pytest.mark.parametrize("order", ["large_then_small"])
def test_noalloc_matches_solve_on_two_calls(order):
    import paper_1404_5344_amd as foe
    torch, dev = torch_dev()
    bank, theta = synth.dct_bank(), synth.theta_weights(2)
    cases = [(synth.config2(), 300, 1), (synth.config3_image(5, 100, 77, 4), 40, 4)]
    for pr, iters, looks in cases:
        H, W = pr.f.shape
        print(f"noalloc case {H}x{W} looks {looks} iters {iters}", flush=True)
        p = foe.default_params(H, W, looks=looks, max_iters=iters)
        f = torch.from_numpy(pr.f).to(dev)
        u_ref, sum_ref, stats_ref = _reference(foe, p, bank, theta, f)
        r = foe.solve_noalloc(p, bank, theta, f)
        torch.cuda.synchronize()
        assert r.summary["iters_done"] == iters
        assert torch.equal(r.u, u_ref), float((r.u - u_ref).abs().max())
        assert np.array_equal(r.stats, stats_ref)
        assert r.summary == sum_ref
        psnr = synth.psnr(r.u.cpu().numpy(), pr.clean)
        print(f"  identical to foe_solve; PSNR {psnr:.4f} dB, trials {r.summary['total_trials']}", flush=True)


def test_noalloc_reports_bad_input_and_recovers():
    import paper_1404_5344_amd as foe
    torch, dev = torch_dev()
    bank, theta = synth.dct_bank(), synth.theta_weights(1)
    pr = synth.config1()
    p = foe.default_params(64, 64, looks=4, max_iters=20)
    bad = pr.f.copy()
    bad[3, 5] = -1.0
    with pytest.raises(foe.FoeError) as e:
        foe.solve_noalloc(p, bank, theta, torch.from_numpy(bad).to(dev))
    assert e.value.status == foe.EINPUT
    f = torch.from_numpy(pr.f).to(dev)
    u_ref, sum_ref, stats_ref = _reference(foe, p, bank, theta, f)
    r = foe.solve_noalloc(p, bank, theta, f)
    assert torch.equal(r.u, u_ref) and np.array_equal(r.stats, stats_ref)
