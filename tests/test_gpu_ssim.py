"""SSIM on the GPU against the FP64 SSIM oracle (FP32 window sums, FP64 block sums).

Bar: 1e-5 absolute on the mean index.  The FP32 variance sigma^2 = E[x^2] - mu^2 loses about
2^-24 * 255^2 ~ 4e-3 to cancellation, against C2 = (0.03 * 255)^2 = 58.5 in the denominator: a relative
error below 1e-4 per position, which averages down over the map."""
import numpy as np
import pytest

import oracle
import synth
from gpu_helpers import torch_dev

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("shape", [(11, 11), (37, 45), (64, 64), (100, 131), (33, 257)])
def test_ssim_matches_oracle(shape):
    import paper_1404_5344_amd as foe
    torch, dev = torch_dev()
    r = np.random.default_rng(shape[0] * 1000 + shape[1])
    clean = synth.shapes_image(9, shape[0], shape[0], shape[1]).astype(np.float32)
    noisy = (clean * np.sqrt(r.gamma(4.0, 0.25, clean.shape))).astype(np.float32)
    u = torch.from_numpy(noisy).to(dev)
    ref = torch.from_numpy(clean).to(dev)
    got = foe.ssim(u, ref)
    want = oracle.ssim(noisy, clean)
    print(f"{shape}: SSIM gpu {got:.7f} oracle {want:.7f}")
    assert abs(got - want) <= 1e-5
    assert abs(foe.ssim(ref, ref) - 1.0) <= 1e-6


def test_ssim_of_a_solve_and_peak():
    import paper_1404_5344_amd as foe
    torch, dev = torch_dev()
    pr = synth.config4(0, 256, 256)
    u = torch.from_numpy(pr.f).to(dev)
    ref = torch.from_numpy(pr.clean.astype(np.float32)).to(dev)
    got = foe.ssim(u, ref, pr.peak)
    want = oracle.ssim(pr.f, pr.clean.astype(np.float32), pr.peak)
    assert abs(got - want) <= 1e-5


def test_ssim_rejects_small_images():
    import paper_1404_5344_amd as foe
    torch, dev = torch_dev()
    x = torch.ones(10, 40, device=dev)
    with pytest.raises(foe.FoeError):
        foe.ssim(x, x)
