"""The real-SAR parameters of Sec. III-C (L = 5, lambda1 = 50, lambda2 = 0.15) on a 256x256 SAR-like image with a
learned-style filter bank (not zero-sum, norms 0.2-5, weights up to 5), 300 backtracking iterations, against the
stored FP64 oracle run (tests/golden/make_golden.py sar_preset).

Bars: those of the other free backtracking runs (final PSNR within 0.05 dB, final energy within 1e-4 relative) for
the FP32 path and the BF16 engine; the largest absolute error on the stored sample of output pixels is printed.
"""
import json
import os

import numpy as np
import pytest

import synth
from gpu_helpers import torch_dev

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "sar_preset_oracle.json")


@pytest.mark.parametrize("name,kw", [("fp32", {}), ("bf16", dict(precision=1))])
def test_sar_preset_against_stored_oracle(name, kw):
    ref = json.load(open(GOLDEN))
    torch, dev = torch_dev()
    pr = synth.sar_preset()
    bank, theta = synth.learned_style_bank(6)
    H, W = pr.f.shape
    import paper_1404_5344_amd as foe
    p = foe.real_sar_params(H, W, max_iters=300, **kw)
    assert (p.looks, p.lambda1, p.lambda2) == (5, pr.lam1, pr.lam2)
    s = foe.Solver(p, bank, theta)
    out = s.solve(torch.from_numpy(pr.f).to(dev))
    u = out.u.cpu().numpy()
    psnr = synth.psnr(u, pr.clean, pr.peak)
    Hgpu = out.stats[-1, 0] + out.stats[-1, 1]
    Hora = ref["F"][-1] + ref["G"][-1]
    idx = np.array(ref["u_sample_idx"])
    err = np.abs(u.ravel()[idx].astype(np.float64) - np.array(ref["u_sample"]))
    print(f"SAR preset {name}: PSNR {psnr:.4f} vs oracle {ref['psnr_final']:.4f} (noisy {ref['psnr_noisy']:.4f}), "
          f"energy rel diff {abs(Hgpu - Hora) / abs(Hora):.2e}, max abs err on {len(idx)} sampled pixels "
          f"{err.max():.3e}, status {out.summary}")
    assert abs(psnr - ref["psnr_final"]) <= 0.05
    assert abs(Hgpu - Hora) <= 1e-4 * abs(Hora)
    s.close()
