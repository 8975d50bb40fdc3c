"""Warm start of the iPiano solve by a small learned network (an extension; the paper always
starts from x^0 = log f).

Pipeline, every step on the GPU through the library's own kernels:
  1. training pairs: seeded speckled 128 x 128 images (looks alternating 1 / 4) and the plain
     solver's 300-iteration output for each, computed by the batched solver;
  2. training: Adam on the mean squared log-amplitude error, forward and backward passes by the
     network kernels (``WarmStartNet``);
  3. inference: u0 = network(f), then a short iPiano run from u0; when that run ends at an energy
     more than 0.5 % above the plain run's, the plain run is the answer (fallback).

Run as a script to train a network and write its parameters, or to evaluate saved parameters:
    python -m paper_1404_5344_amd.warmstart --images 20000 --epochs 8 --out weights.npy
    python -m paper_1404_5344_amd.warmstart --evaluate 256 --out weights.npy
"""
from __future__ import annotations

import argparse
import os
import time
from concurrent.futures import ProcessPoolExecutor

import numpy as np

from . import BatchSolver, WarmStartNet, cnn_init_params, default_params

FALLBACK_TOL = 0.005        # warm-start energy above the plain one by this fraction of |H_plain| -> fallback


def needs_fallback(H_warm: float, H_plain: float, tol: float | None = None) -> bool:
    """The energy test of the warm start: fall back to the plain run when the warm-started energy exceeds the
    plain run's by more than tol |H_plain|.  The energy is sign-indefinite (the lambda2 term of the data term is
    negative on bright pixels), so the margin is taken on |H_plain|, not as a ratio."""
    tol = FALLBACK_TOL if tol is None else tol
    return H_warm - H_plain > tol * abs(H_plain)


def energy_gap(H_warm: float, H_plain: float) -> float:
    """(H_warm - H_plain) / |H_plain|: positive when the warm start ends at a higher energy."""
    return (H_warm - H_plain) / abs(H_plain)
WEIGHTS = os.path.join(os.path.dirname(os.path.abspath(__file__)), "weights", "warmstart_cnn.npy")


def _train_image(i):
    import synth
    p = synth.config5_train(i)
    return p.f, p.looks


def training_inputs(n_images: int, workers: int = 8):
    """Noisy 128 x 128 training images (float32 [n, 128, 128]) and their looks, from the seeded
    generator; generated in host worker processes."""
    if workers <= 1:
        res = [_train_image(i) for i in range(n_images)]
    else:
        with ProcessPoolExecutor(max_workers=workers) as ex:
            res = list(ex.map(_train_image, range(n_images), chunksize=64))
    return np.stack([r[0] for r in res]), [r[1] for r in res]


def plain_targets(f, looks, bank, theta, iters: int = 300, batch: int = 256):
    """The plain solver's output (x^0 = log f, `iters` iterations) for every image of f
    (CUDA tensor [n, H, W]), solved `batch` images per batched launch."""
    import torch
    n, H, W = f.shape
    out = torch.empty_like(f)
    solvers = {}
    for s in range(0, n, batch):
        m = min(batch, n - s)
        key = (m, tuple(looks[s:s + m]))
        if key not in solvers:
            p = default_params(0, 0, max_iters=iters)
            solvers[key] = BatchSolver(p, [(H, W)] * m, list(looks[s:s + m]), bank, theta)
        b = solvers[key]
        u, _, _, _ = b.solve(f[s:s + m].reshape(-1).contiguous())
        out[s:s + m] = u.reshape(m, H, W)
    for b in solvers.values():
        b.close()
    return out


def train(net: WarmStartNet, f, u, epochs: int, batch: int = 32, lr: float = 1e-3, seed: int = 0,
          lr_final: float = 1e-4, log=print):
    """Adam over shuffled mini-batches; the learning rate decays geometrically from lr to
    lr_final over the run.  Returns the mean loss of each epoch."""
    import torch
    n = f.shape[0]
    rng = np.random.Generator(np.random.PCG64(seed))
    steps = epochs * (n // batch)
    k = 0
    losses = []
    for e in range(epochs):
        order = torch.from_numpy(rng.permutation(n)).to(f.device)
        tot = 0.0
        t0 = time.perf_counter()
        for s in range(n // batch):
            idx = order[s * batch:(s + 1) * batch]
            rate = lr * (lr_final / lr) ** (k / max(steps - 1, 1))
            tot += net.train_step(f[idx].contiguous(), u[idx].contiguous(), rate)
            k += 1
        losses.append(tot / (n // batch))
        if log:
            log(f"epoch {e}: loss {losses[-1]:.5f} ({time.perf_counter() - t0:.1f} s)")
    return losses


def infer(net: WarmStartNet, f, chunk: int = 16):
    """u0 = network(f) for a batch [n, H, W], `chunk` images per call (the network keeps the
    activations of one call: 162 planes per image)."""
    import torch
    u0 = torch.empty_like(f)
    for s in range(0, f.shape[0], chunk):
        net.infer(f[s:s + chunk], out=u0[s:s + chunk])
    return u0


def warm_solve(batch: BatchSolver, net: WarmStartNet, f):
    """u0 = network(f) for every image of a batch of equal-size images (CUDA tensor [n, H, W]),
    then the batch solver's iterations from u0.  Returns (u, summaries, u0)."""
    u0 = infer(net, f)
    u, sums, _, _ = batch.solve(f.reshape(-1).contiguous(), init=u0.reshape(-1).contiguous())
    return u.reshape(f.shape), sums, u0


def evaluate(net: WarmStartNet, f, looks, bank, theta, iters_warm: int = 40, iters_plain: int = 300):
    """Held-out evaluation of a batch of equal-size images: the plain run (x^0 = log f,
    iters_plain iterations), the same number of iterations as the warm start but from log f, and
    the warm start (network, then iters_warm iterations) with its energy fallback.  Returns
    (u_plain, u_short, u_warm_or_fallback, records) with per-image energies and fallback flags."""
    n, H, W = f.shape
    looks = list(looks)
    sizes = [(H, W)] * n
    bp = BatchSolver(default_params(0, 0, max_iters=iters_plain), sizes, looks, bank, theta)
    bs = BatchSolver(default_params(0, 0, max_iters=iters_warm), sizes, looks, bank, theta)
    fp = f.reshape(-1).contiguous()
    u_plain, s_plain, _, _ = bp.solve(fp)
    u_short, s_short, _, _ = bs.solve(fp)
    u_warm, s_warm, _ = warm_solve(bs, net, f)
    u_plain, u_short = u_plain.reshape(f.shape), u_short.reshape(f.shape)
    records = []
    out = u_warm.clone()
    for i in range(n):
        fb = needs_fallback(s_warm[i]["H"], s_plain[i]["H"])
        if fb:
            out[i] = u_plain[i]
        records.append(dict(H_plain=s_plain[i]["H"], H_short=s_short[i]["H"], H_warm=s_warm[i]["H"], fallback=fb))
    bp.close()
    bs.close()
    return u_plain, u_short, out, records


def save(net: WarmStartNet, path: str = WEIGHTS):
    master, _ = net.params()
    os.makedirs(os.path.dirname(path), exist_ok=True)
    np.save(path, master)


def load(path: str = WEIGHTS, stream=None) -> WarmStartNet:
    return WarmStartNet(np.load(path), stream=stream)


def _eval_image(i):
    import synth
    p = synth.config5_eval(i)
    return p.f, p.clean, p.looks


def held_out(n_images: int, workers: int = 8):
    """Held-out 512 x 512 evaluation images (seed space disjoint from training): noisy f
    [n, 512, 512] float32, clean [n, 512, 512] float64, looks."""
    if workers <= 1:
        res = [_eval_image(i) for i in range(n_images)]
    else:
        with ProcessPoolExecutor(max_workers=workers) as ex:
            res = list(ex.map(_eval_image, range(n_images)))
    return np.stack([r[0] for r in res]), np.stack([r[1] for r in res]), [r[2] for r in res]


def report(n_images: int, path: str = WEIGHTS, iters_warm: int = 40, iters_plain: int = 300, workers: int = 8,
           quiet: bool = False) -> dict:
    """Held-out evaluation: PSNR and energy of the warm start (with fallback) against the plain
    run and against the same iteration count from log f (printed as one JSON line unless quiet)."""
    import json
    import synth
    import torch
    f_np, clean, looks = held_out(n_images, workers)
    f = torch.from_numpy(f_np).to("cuda:0")
    net = load(path)
    u_plain, u_short, u_warm, rec = evaluate(net, f, looks, synth.dct_bank(), synth.theta_weights(5), iters_warm,
                                             iters_plain)
    ps = lambda u: np.array([synth.psnr(u[i].cpu().numpy(), clean[i]) for i in range(n_images)])
    p_plain, p_short, p_warm = ps(u_plain), ps(u_short), ps(u_warm)
    gap = np.array([energy_gap(r["H_warm"], r["H_plain"]) for r in rec])
    out = dict(images=n_images, iters_warm=iters_warm, iters_plain=iters_plain,
               psnr_noisy=float(np.mean([synth.psnr(f_np[i], clean[i]) for i in range(n_images)])),
               psnr_plain=float(p_plain.mean()), psnr_same_iters_from_log_f=float(p_short.mean()),
               psnr_warm=float(p_warm.mean()), psnr_warm_minus_plain_min=float((p_warm - p_plain).min()),
               energy_gap_mean=float(gap.mean()), energy_gap_max=float(gap.max()),
               fallback_rate=float(np.mean([r["fallback"] for r in rec])))
    net.close()
    if not quiet:
        print(json.dumps(out), flush=True)
    return out


def time_kernels(reps: int = 20):
    """Wall time of the shipped network's inference on one 512 x 512 image and of one loss-and-gradient
    evaluation on a batch of 32 images of 128 x 128 (medians over reps calls, inputs resident)."""
    import numpy as np
    import torch
    dev = torch.device("cuda:0")
    net = load()
    g = torch.Generator(device="cpu").manual_seed(0)
    f = (torch.rand(1, 512, 512, generator=g) * 200 + 1).to(dev)
    fb = (torch.rand(32, 128, 128, generator=g) * 200 + 1).to(dev)
    ut = fb * 1.1
    out = {}
    for name, fn in (("infer_512x512_ms", lambda: net.infer(f)), ("loss_grad_32x128x128_ms", lambda: net.loss_grad(fb, ut))):
        for _ in range(3):
            fn()
        ts = []
        for _ in range(reps):
            torch.cuda.synchronize()
            t = time.perf_counter()
            fn()
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t)
        out[name] = round(float(np.median(ts)) * 1e3, 4)
        print(name, out[name], flush=True)
    net.close()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--time", action="store_true", help="time the network's inference and gradient kernels")
    ap.add_argument("--evaluate", type=int, default=0, help="evaluate the saved network on this many held-out images")
    ap.add_argument("--images", type=int, default=20000)
    ap.add_argument("--epochs", type=int, default=8)
    ap.add_argument("--batch", type=int, default=32)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--out", default=WEIGHTS)
    a = ap.parse_args()
    if a.time:
        time_kernels()
        return
    if a.evaluate:
        report(a.evaluate, a.out)
        return
    import synth
    t0 = time.perf_counter()
    f_np, looks = training_inputs(a.images)
    print(f"generated {a.images} training images in {time.perf_counter() - t0:.1f} s", flush=True)
    import torch
    dev = torch.device("cuda:0")
    f = torch.from_numpy(f_np).to(dev)
    t0 = time.perf_counter()
    u = plain_targets(f, looks, synth.dct_bank(), synth.theta_weights(5))
    torch.cuda.synchronize()
    print(f"plain 300-iteration targets in {time.perf_counter() - t0:.1f} s", flush=True)
    net = WarmStartNet(cnn_init_params(a.seed))
    t0 = time.perf_counter()
    train(net, f, u, a.epochs, a.batch, a.lr, a.seed, log=lambda m: print(m, flush=True))
    print(f"trained in {time.perf_counter() - t0:.1f} s", flush=True)
    save(net, a.out)
    print(f"wrote {a.out}", flush=True)


if __name__ == "__main__":
    main()
