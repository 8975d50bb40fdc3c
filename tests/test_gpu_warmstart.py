"""Warm start of the solve by the learned network: what it gains over the method without it.

  * a network trained here from scratch (1024 seeded 128 x 128 pairs whose targets are the plain
    solver's 300-iteration outputs, 3 epochs on the GPU kernels) starts held-out 256 x 256 images
    closer to the solution: after 10 iterations from the network's u0 the PSNR is higher than
    after 10 iterations from log f, on every image;
  * the shipped network (trained by ``python -m paper_1404_5344_amd.warmstart`` on 20000 pairs) on
    held-out 512 x 512 images: 40 iterations from its u0 reach the plain 300-iteration PSNR within
    0.01 dB, end within 0.5 % of the plain energy (so no fallback), and beat 40 iterations from
    log f;
  * the fallback replaces an image whose energy is too high by the plain result.
"""
import os

import numpy as np
import pytest

import synth
from gpu_helpers import torch_dev

pytestmark = pytest.mark.gpu


def _psnrs(u, clean):
    return np.array([synth.psnr(u[i].cpu().numpy(), clean[i]) for i in range(len(clean))])


def test_network_trained_here_gains_over_log_f():
    import paper_1404_5344_amd as foe
    from paper_1404_5344_amd import warmstart as ws
    torch, dev = torch_dev()
    bank, theta = synth.dct_bank(), synth.theta_weights(5)
    f_np, looks = ws.training_inputs(1024, workers=1)
    f = torch.from_numpy(f_np).to(dev)
    u = ws.plain_targets(f, looks, bank, theta)
    net = foe.WarmStartNet(foe.cnn_init_params(0))
    losses = ws.train(net, f, u, 3, log=None)
    assert losses[-1] < losses[0]
    probs = [synth.config5_eval(i, 256, 256) for i in range(3)]
    fe = torch.from_numpy(np.stack([p.f for p in probs])).to(dev)
    clean = [p.clean for p in probs]
    iters = 10
    b = foe.BatchSolver(foe.default_params(0, 0, max_iters=iters), [(256, 256)] * 3, [p.looks for p in probs],
                        bank, theta)
    u_log, _, _, _ = b.solve(fe.reshape(-1).contiguous())
    u_warm, _, _ = ws.warm_solve(b, net, fe)
    p_log, p_warm = _psnrs(u_log.reshape(fe.shape), clean), _psnrs(u_warm, clean)
    print("PSNR after", iters, "iterations: from log f", p_log, "from the network", p_warm)
    assert np.all(p_warm > p_log)
    b.close()
    net.close()


def test_shipped_network_on_held_out_images():
    from paper_1404_5344_amd import warmstart as ws
    torch, dev = torch_dev()
    assert os.path.exists(ws.WEIGHTS), ws.WEIGHTS
    n = 4
    f_np, clean, looks = ws.held_out(n, workers=1)
    f = torch.from_numpy(f_np).to(dev)
    net = ws.load()
    u_plain, u_short, u_warm, rec = ws.evaluate(net, f, looks, synth.dct_bank(), synth.theta_weights(5))
    p_plain, p_short, p_warm = _psnrs(u_plain, clean), _psnrs(u_short, clean), _psnrs(u_warm, clean)
    for i in range(n):
        print(f"image {i}: plain 300 {p_plain[i]:.3f} dB, 40 from log f {p_short[i]:.3f}, "
              f"network + 40 {p_warm[i]:.3f}; energy gap {ws.energy_gap(rec[i]['H_warm'], rec[i]['H_plain']):.2e}")
    assert not any(r["fallback"] for r in rec)
    assert np.all(p_warm >= p_plain - 0.01)
    assert np.mean(p_warm) > np.mean(p_short)
    net.close()


def test_fallback_takes_the_plain_result(monkeypatch):
    from paper_1404_5344_amd import warmstart as ws
    torch, dev = torch_dev()
    f_np, clean, looks = ws.held_out(2, workers=1)
    f = torch.from_numpy(f_np[:, :128, :128].copy()).to(dev)
    net = ws.load()
    # a tolerance of -inf sends every image to the fallback
    monkeypatch.setattr(ws, "FALLBACK_TOL", float("-inf"))
    u_plain, _, u_out, rec = ws.evaluate(net, f, looks, synth.dct_bank(), synth.theta_weights(5), 5, 20)
    assert all(r["fallback"] for r in rec)
    assert torch.equal(u_out, u_plain)
    net.close()
