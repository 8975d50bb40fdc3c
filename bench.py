"""Throughput of the iPiano-FoE despeckling hot path on one MI355X.

One step = one full solve of the 512x512 single-look workload (init, 300 iPiano iterations with
backtracking, output) on synthetic input resident in HBM.  Prints one JSON line:
  value         Mpixel-iterations/s = H * W * accepted iterations / wall time per step
  roofline      the fused trial kernel: algorithmic flops per launch (9,408 per pixel: forward and adjoint
                bank) / its mean in-solve launch duration (the solver's HIP event pair on its stream
                around the iteration loop, over the trial launches), against the FP32 vector peak; traffic =
                HBM bytes per launch from the committed hardware-counter summary when it was taken
                on the current kernel sources, else null
  engines       the solver's default forward bank is the split-FP16 matrix-core engine (each FP32
                operand as an FP16 head plus a scaled FP16 tail, exact products, FP32 accumulation;
                the parity bars of the FP32 path); the same workload on the FP32-operand matrix-core
                engine is timed beside it (fp32_operand_engine)
  cpu_baseline  the FP64 oracle on the host cores over a bounded sample of the same workload
  forms         time-to-PSNR of the batched, BF16 and warm-started forms against the plain FP32
                solver on their own workloads (the wall time to reach the plain run's final PSNR
                minus 0.01 dB, or 0.05 dB for BF16; the crossing iteration is found with a PSNR probe
                and a separate run of exactly that many iterations is timed), and time-to-energy (H
                within 0.5 % of the plain final H) for the BF16 and warm-started forms; the warm start
                also on the 256 held-out images, the unfused gradient, the Lambert-W prox and the run-time
                points of Sec. III-D
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

METRIC = "Mpixel-iters/s iPiano-FoE on 1 GPU; time-to-PSNR vs plain FP32; roofline %"
PEAK_FP32_TFLOPS = 157.3      # MI355X published FP32 peak, vector and matrix cores alike
PEAK_F16_MFMA_TFLOPS = 2500.0  # MI355X published dense FP16 matrix peak
# the split forward bank issues 3 FP16 products per FP32 product over 64 tap slots for 49 taps
SPLIT_FWD_PEAK = PEAK_F16_MFMA_TFLOPS / 3.0 * 49.0 / 64.0
# forward bank at that rate and adjoint bank (same flops) at the FP32 peak
MIXED_PEAK_TFLOPS = 2.0 / (1.0 / SPLIT_FWD_PEAK + 1.0 / PEAK_FP32_TFLOPS)
NF, KK = 48, 49
FLOP_PER_PX_TRIAL = 2 * 2 * NF * KK   # forward bank on x+ and adjoint bank, one FMA = 2 flop
KERNEL_SOURCES = ["common.hpp", "device_math.hpp", "kernels_trial.hpp", "foe_lib.hip"]   # kernels and their launch shapes
TRAFFIC_SUMMARY = os.path.join(ROOT, "profiles", "foe_trial_kernel_512x512_hbm_traffic.md")
UNFUSED_TRAFFIC_SUMMARY = os.path.join(ROOT, "profiles", "foe_trial_kernel_unfused_512x512_hbm_traffic.md")
TILE_SHAPES = ["32x32", "32x16", "32x8", "64x8"]   # foe_set_tile_config indices


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for n in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_1404_5344_amd", "csrc", n), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(path=None, key="HBM bytes per launch"):
    """HBM bytes per launch (or per trial) from a committed counter summary, or None when the summary
    is missing or was taken on other kernel sources."""
    path = path or TRAFFIC_SUMMARY
    if not os.path.exists(path):
        return None
    text = open(path).read()
    m_hash = re.search(r"kernel source hash:\s*([0-9a-f]+)", text)
    m_bytes = re.search(re.escape(key) + r":\s*([0-9.eE+]+)", text)
    if not m_hash or not m_bytes or m_hash.group(1) != kernel_source_hash():
        return None
    return float(m_bytes.group(1))


def _oracle_rate(pr, bank, theta, seconds_target):
    """The FP64 oracle on a bounded sample of the workload: Mpixel-it/s, accepted iterations, trials, seconds."""
    import oracle
    p = oracle.Params(lam1=pr.lam1, lam2=pr.lam2)
    H, W = pr.f.shape
    # calibrate on 2 iterations, then run a bounded sample
    t = time.perf_counter()
    oracle.ipiano(p, pr.f, bank, theta, 2, L0=1.0)
    t2 = time.perf_counter() - t
    iters = int(max(2, min(60, seconds_target / max(t2 / 2, 1e-3))))
    t = time.perf_counter()
    r = oracle.ipiano(p, pr.f, bank, theta, iters, L0=1.0)
    dt = time.perf_counter() - t
    n_acc = int(r.stats.shape[0])
    return H * W * n_acc / dt / 1e6, n_acc, int(r.stats[:, 4].sum()), dt


def cpu_baseline(pr, bank, theta, seconds_target=15.0):
    import oracle
    cores = oracle.get_threads()
    v, n_acc, trials, dt = _oracle_rate(pr, bank, theta, seconds_target)
    oracle.set_threads(1)
    try:
        v1, n1, _, dt1 = _oracle_rate(pr, bank, theta, seconds_target / 2)
    finally:
        oracle.set_threads(cores)
    return {"value": round(v, 4), "unit": "Mpixel-iters/s", "cores": cores, "kind": "oracle",
            "sample": f"FP64 oracle, same 512x512 input, first {n_acc} iterations from x0 = log f "
                      f"({trials} trials), {dt:.1f} s on {cores} threads",
            "one_core": {"value": round(v1, 4), "cores": 1, "sample": f"first {n1} iterations, {dt1:.1f} s"},
            "host_cpu": _cpu_model()}


def _cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


# ------------------------------------------------------------------------------------ forms
def _sync():
    import torch
    torch.cuda.synchronize()


def _wall(fn, reps=3):
    """Median wall time of fn() over reps runs (after one untimed run), GPU synchronised."""
    fn()
    ts = []
    for _ in range(reps):
        _sync()
        t = time.perf_counter()
        fn()
        _sync()
        ts.append(time.perf_counter() - t)
    return float(np.median(ts))


def _psnr_t(u, clean_t, peak):
    import torch
    mse = torch.mean((u.double() - clean_t) ** 2).item()
    return 10.0 * math.log10(peak * peak / mse)


def _crossing(traj, target):
    hit = np.nonzero(np.asarray(traj) >= target)[0]
    return int(hit[0]) if hit.size else None


def _probe(solver, f, x0, clean_t, peak, iters, exp=True, energy=None):
    """PSNR after 0..iters iterations from x^0 = x^{-1} = x0 (single-image solver); with energy (a solver
    of FP32 accuracy on the same problem) also the energy H = F + G of every iterate."""
    import torch
    x, xp, L = x0.clone(), x0.clone(), 1.0
    out = [_psnr_t(torch.exp(x) if exp else x, clean_t, peak)]
    hs = [sum(energy.eval_energy(x, f))] if energy is not None else None
    for _ in range(iters):
        L, _, _ = solver.solve_from(f, x, xp, L, 1)
        out.append(_psnr_t(torch.exp(x), clean_t, peak))
        if energy is not None:
            hs.append(sum(energy.eval_energy(x, f)))
    return out if energy is None else (out, hs)


ENERGY_TOL = 0.005   # time-to-energy: H within 0.5 % of the plain solve's final H


def _energy_crossing(hs, h_ref):
    """First iteration whose energy is within ENERGY_TOL of h_ref (relative to abs(h_ref)), or None."""
    hit = np.nonzero(np.asarray(hs) - h_ref <= ENERGY_TOL * abs(h_ref))[0]
    return int(hit[0]) if hit.size else None


def _run_from(solver, f, x0, k):
    """Closure running exactly k iterations from x0 (state copies made outside the timed call)."""
    state = {}

    def prep():
        state["x"], state["xp"] = x0.clone(), x0.clone()

    def run():
        if k > 0:
            solver.solve_from(f, state["x"], state["xp"], 1.0, k)
    return prep, run


def _wall_prepped(prep, run, reps=3):
    prep()
    run()
    ts = []
    for _ in range(reps):
        prep()
        _sync()
        t = time.perf_counter()
        run()
        _sync()
        ts.append(time.perf_counter() - t)
    return float(np.median(ts))


def form_bf16(dev):
    """BF16 filter bank against the FP32 solve: time-to-PSNR and time-to-energy on the first 2048 x 2048 SAR-like
    tile, then the four tiles in one batch in each precision (per-tile PSNR, batch throughput)."""
    import torch
    import paper_1404_5344_amd as foe
    import synth
    pr = synth.config4(0)
    bank, theta = synth.dct_bank(), synth.theta_weights(4)
    f = torch.from_numpy(pr.f).to(dev)
    clean = torch.from_numpy(pr.clean).to(dev)
    x0 = torch.log(f)
    res, hs = {}, {}
    solvers = {}
    for name, kw in (("fp32", {}), ("bf16", dict(precision=1))):
        p = foe.default_params(2048, 2048, lambda1=pr.lam1, lambda2=pr.lam2, max_iters=300, **kw)
        solvers[name] = foe.Solver(p, bank, theta)
        res[name], hs[name] = _probe(solvers[name], f, x0, clean, pr.peak, 300, energy=solvers.get("fp32", solvers[name]))
    target = res["fp32"][-1] - 0.05
    out = {"workload": "2048x2048 SAR-like tile 0, L=1, 300 iterations", "tol_db": 0.05,
           "psnr_final_fp32": round(res["fp32"][-1], 4), "psnr_final_bf16": round(res["bf16"][-1], 4),
           "energy_tol_rel": ENERGY_TOL, "H_final_fp32": hs["fp32"][-1], "H_final_bf16": hs["bf16"][-1]}
    for name in ("fp32", "bf16"):
        k = _crossing(res[name], target)
        out[f"reached_{name}"] = k is not None
        k = 300 if k is None else k
        prep, run = _run_from(solvers[name], f, x0, k)
        out[f"iters_{name}"] = k
        out[f"seconds_{name}"] = round(_wall_prepped(prep, run), 5)
        # time to energy: the first iterate whose H (FP32-accuracy evaluation) is within 0.5 % of the
        # FP32 solve's final H
        ke = _energy_crossing(hs[name], hs["fp32"][-1])
        out[f"energy_reached_{name}"] = ke is not None
        ke = 300 if ke is None else ke
        prep, run = _run_from(solvers[name], f, x0, ke)
        out[f"energy_iters_{name}"] = ke
        out[f"energy_seconds_{name}"] = round(_wall_prepped(prep, run), 5)
        # throughput of the full 300 iterations in this precision
        prep, run = _run_from(solvers[name], f, x0, 300)
        t300 = _wall_prepped(prep, run, reps=2)
        out[f"mpix_it_s_{name}"] = round(2048 * 2048 * 300 / t300 / 1e6, 1)
    out["speedup"] = round(out["seconds_fp32"] / out["seconds_bf16"], 3)
    out["energy_speedup"] = round(out["energy_seconds_fp32"] / out["energy_seconds_bf16"], 3)
    for s in solvers.values():
        s.close()
    # the whole workload, the four tiles in one batch, in each precision: per-tile final PSNR and the
    # throughput of the batch
    tiles = [pr] + [synth.config4(i) for i in (1, 2, 3)]
    n = 2048 * 2048
    fb = torch.cat([torch.from_numpy(q.f).reshape(-1) for q in tiles]).to(dev)
    four = {"workload": "4 x 2048x2048 SAR-like tiles in one batch, L=1, 300 iterations"}
    for name, kw in (("fp32", {}), ("bf16", dict(precision=1))):
        b = foe.BatchSolver(foe.default_params(0, 0, max_iters=300, **kw), [(2048, 2048)] * 4, [q.looks for q in tiles],
                            bank, theta, lambda1=[q.lam1 for q in tiles], lambda2=[q.lam2 for q in tiles])
        u = b.solve(fb)[0]
        four[f"psnr_{name}"] = [round(synth.psnr(u[i * n:(i + 1) * n].reshape(2048, 2048).cpu().numpy(), q.clean, q.peak), 4)
                                for i, q in enumerate(tiles)]
        t = _wall(lambda: b.solve(fb), reps=2)
        four[f"mpix_it_s_{name}"] = round(4 * n * 300 / t / 1e6, 1)
        b.close()
    four["max_abs_psnr_diff_db"] = round(max(abs(a - c) for a, c in zip(four["psnr_fp32"], four["psnr_bf16"])), 4)
    four["speedup"] = round(four["mpix_it_s_bf16"] / four["mpix_it_s_fp32"], 3)
    out["four_tiles"] = four
    return out


def form_batched(dev, n_images=64):
    """64 uneven images in one batched solve against one single-image solve per image."""
    import torch
    import paper_1404_5344_amd as foe
    import synth
    sizes = synth.config3_sizes(n_images)
    probs = [synth.config3_image(i, H, W, L) for i, (H, W, L) in enumerate(sizes)]
    bank, theta = synth.dct_bank(), synth.theta_weights(3)
    hw = [(H, W) for H, W, _ in sizes]
    looks = [L for _, _, L in sizes]
    b = foe.BatchSolver(foe.default_params(0, 0, max_iters=300), hw, looks, bank, theta)
    b.autotune(b.pack([torch.from_numpy(p.f) for p in probs]).to(dev), reps=3)
    f = b.pack([torch.from_numpy(p.f) for p in probs]).to(dev)
    clean = b.pack([torch.from_numpy(p.clean) for p in probs]).to(dev).double()
    offs = torch.tensor(b.offsets, device=dev)
    npx = (offs[1:] - offs[:-1]).double()

    def psnrs(x):
        d2 = (torch.exp(x).double() - clean) ** 2
        cs = torch.cat([torch.zeros(1, dtype=torch.float64, device=dev), torch.cumsum(d2, 0)])
        mse = (cs[offs[1:]] - cs[offs[:-1]]) / npx
        return (10.0 * torch.log10(255.0 ** 2 / mse)).cpu().numpy()

    x0 = torch.log(f)
    x, xp, L = x0.clone(), x0.clone(), [1.0] * n_images
    traj = [psnrs(x)]
    for _ in range(300):
        L, _, _ = b.solve_from(f, x, xp, L, 1)
        traj.append(psnrs(x))
    traj = np.stack(traj)                          # [301, n]
    target = traj[-1] - 0.01
    ks = [_crossing(traj[:, i], target[i]) for i in range(n_images)]
    ks = [300 if k is None else k for k in ks]
    K = max(ks)

    def prep():
        prep.x, prep.xp = x0.clone(), x0.clone()

    def run_batch(k):
        return lambda: b.solve_from(f, prep.x, prep.xp, [1.0] * n_images, k)
    t_batch = _wall_prepped(prep, run_batch(K))
    t_batch300 = _wall_prepped(prep, run_batch(300), reps=2)
    lat = b.latency()   # per-image, device timestamps, of the last 300-iteration batch run
    # one solver per image, run one after the other
    singles = []
    for i, (H, W) in enumerate(hw):
        p = foe.default_params(H, W, looks=looks[i], max_iters=300)
        singles.append(foe.Solver(p, bank, theta))
    views = b.unpack(f)
    x0v = [torch.log(v).contiguous() for v in views]
    fv = [v.contiguous() for v in views]

    def seq(kk):
        def run():
            for i, s in enumerate(singles):
                if kk[i] > 0:
                    xi, xpi = x0v[i].clone(), x0v[i].clone()
                    s.solve_from(fv[i], xi, xpi, 1.0, kk[i])
        return run
    t_seq = _wall(seq(ks), reps=1)
    t_seq300 = _wall(seq([300] * n_images), reps=1)
    total_px = sum(H * W for H, W in hw)
    for s in singles:
        s.close()
    b.close()
    return {"workload": f"{n_images} images, sides U{{128..1024}} step 64, L in {{1,2,4,8}}, 300 iterations",
            "tol_db": 0.01, "pixels": total_px, "iters_max": K, "iters_mean": round(float(np.mean(ks)), 1),
            "seconds_batched": round(t_batch, 5), "seconds_one_by_one": round(t_seq, 5),
            "speedup": round(t_seq / t_batch, 3),
            "mpix_it_s_batched": round(total_px * 300 / t_batch300 / 1e6, 1),
            "mpix_it_s_one_by_one": round(total_px * 300 / t_seq300 / 1e6, 1),
            "latency_s_batched_all_images": round(t_batch300, 4),
            "latency_ms_per_image_device": {"p50": round(float(np.percentile(lat, 50)), 3),
                                            "p95": round(float(np.percentile(lat, 95)), 3),
                                            "max": round(float(lat.max()), 3), "min": round(float(lat.min()), 3)},
            "latency_s_one_by_one_mean_image": round(t_seq300 / n_images, 5)}


def form_warm(dev):
    """Learned warm start on a held-out 512 x 512 image against the plain solve from log f."""
    import torch
    import paper_1404_5344_amd as foe
    import synth
    from paper_1404_5344_amd import warmstart as ws
    pr = synth.config5_eval(0)
    bank, theta = synth.dct_bank(), synth.theta_weights(5)
    f = torch.from_numpy(pr.f).to(dev)
    clean = torch.from_numpy(pr.clean).to(dev)
    s = foe.Solver(foe.default_params(512, 512, looks=pr.looks, max_iters=300), bank, theta)
    net = ws.load()
    x0 = torch.log(f)
    u0 = net.infer(f.reshape(1, 512, 512)).reshape(512, 512)
    plain, h_plain = _probe(s, f, x0, clean, 255.0, 300, energy=s)
    warm, h_warm = _probe(s, f, torch.log(u0), clean, 255.0, 40, energy=s)
    target = plain[-1] - 0.01
    # time to energy: the first iterate with H within 0.5 % of the plain final H
    ke_plain = _energy_crossing(h_plain, h_plain[-1])
    ke_warm = _energy_crossing(h_warm, h_plain[-1])
    k_plain = _crossing(plain, target)
    k_plain = 300 if k_plain is None else k_plain
    k_warm = _crossing(warm, target)
    prep, run = _run_from(s, f, x0, k_plain)
    t_plain = _wall_prepped(prep, run)
    f3 = f.reshape(1, 512, 512)
    if k_warm is not None:
        def run_w():
            w = torch.log(net.infer(f3).reshape(512, 512))
            if k_warm > 0:
                s.solve_from(f, w, w.clone(), 1.0, k_warm)
        fallback = False
    else:   # the 40 warm iterations miss the target: the plain solve follows
        def run_w():
            w = torch.log(net.infer(f3).reshape(512, 512))
            s.solve_from(f, w, w.clone(), 1.0, 40)
            x, xp = x0.clone(), x0.clone()
            s.solve_from(f, x, xp, 1.0, k_plain)
        fallback = True
    t_warm = _wall(run_w)
    t_net = _wall(lambda: net.infer(f3))
    energy = {"energy_tol_rel": ENERGY_TOL, "H_final_plain": h_plain[-1], "H_network_only": h_warm[0],
              "H_network_plus_40": h_warm[-1], "energy_iters_plain": ke_plain, "energy_iters_warm": ke_warm}
    prep, run = _run_from(s, f, x0, ke_plain)
    te_plain = _wall_prepped(prep, run)
    energy["energy_seconds_plain"] = round(te_plain, 5)
    if ke_warm is not None:
        def run_we():
            w = torch.log(net.infer(f3).reshape(512, 512))
            if ke_warm > 0:
                s.solve_from(f, w, w.clone(), 1.0, ke_warm)
        te_warm = _wall(run_we)
        energy["energy_seconds_warm"] = round(te_warm, 5)
        energy["energy_speedup"] = round(te_plain / te_warm, 3)
    else:
        energy["energy_seconds_warm"] = None   # not reached in 40 iterations: the fallback would run
        energy["energy_speedup"] = None
    net.close()
    s.close()
    return {"workload": "held-out 512x512 image, L=1; network + up to 40 iterations vs plain 300", "tol_db": 0.01,
            "psnr_final_plain": round(plain[-1], 4), "psnr_network_only": round(warm[0], 4),
            "psnr_network_plus_40": round(warm[-1], 4), "iters_plain": k_plain, "iters_warm": k_warm,
            "fallback": fallback, "seconds_plain": round(t_plain, 5), "seconds_warm": round(t_warm, 5),
            "seconds_network": round(t_net, 5), "speedup": round(t_plain / t_warm, 3), **energy}


def form_warm_eval(dev, n_images=256):
    """The warm start on the 256 held-out 512 x 512 evaluation images (seeds disjoint from the network's training
    images), batched: mean PSNR of network + 40 iterations (with the energy fallback) against the plain 300
    iterations and against 40 iterations from log f; the energy gap to the plain run and the fallback rate."""
    from paper_1404_5344_amd import warmstart as ws
    out = ws.report(n_images, workers=1, quiet=True)
    out["workload"] = f"{n_images} held-out 512x512 images, L in {{1, 2, 4, 8}}, DCT bank"
    return {k: (round(v, 5) if isinstance(v, float) else v) for k, v in out.items()}


def form_unfused(dev, steps=5):
    """The same 512 x 512 solve with the gradient split in two launches that exchange the 48 z planes
    through HBM (forward half writes them, adjoint half reads them), against the fused kernel."""
    import torch
    import paper_1404_5344_amd as foe
    import synth
    pr = synth.config2()
    bank, theta = synth.dct_bank(), synth.theta_weights(2)
    H, W = pr.f.shape
    f = torch.from_numpy(pr.f).to(dev)
    out = {"workload": "512x512 config of the main line, 300 iterations, gradient unfused"}
    for name, fusion in (("fused", 0), ("unfused", 1)):
        p = foe.default_params(H, W, lambda1=pr.lam1, lambda2=pr.lam2, max_iters=300, fusion=fusion)
        s = foe.Solver(p, bank, theta)
        s.solve(f)
        t = _wall(lambda: s.solve(f), reps=steps)
        r = s.solve(f)
        out[f"mpix_it_s_{name}"] = round(H * W * r.summary["iters_done"] / t / 1e6, 1)
        out[f"psnr_{name}"] = round(synth.psnr(r.u.cpu().numpy(), pr.clean), 4)
        ms_loop, n_trials = s.last_timing()   # in-solve: the solver's event pair around its iteration loop
        ms = ms_loop / n_trials
        out[f"us_per_trial_{name}"] = round(ms * 1e3, 2)
        if fusion:
            # algorithmic HBM bytes of one unfused trial: forward half reads f, x^n, x^(n-1), grad F(x^n)
            # (16 B/px) and writes x+ (4) and z (4 * 48); adjoint half reads z (4 * 48) and x+ (4) and
            # writes grad F(x+) (4)
            bpp = 16 + 4 + 4 * NF + 4 * NF + 4 + 4
            out["algorithmic_bytes_per_px_trial"] = bpp
            out["hbm_gb_s_algorithmic"] = round(bpp * H * W / (ms * 1e-3) / 1e9, 1)
            out["hbm_frac_of_8tb_s_algorithmic"] = round(bpp * H * W / (ms * 1e-3) / 8e12, 4)
            meas = measured_traffic(UNFUSED_TRAFFIC_SUMMARY, "HBM bytes per trial")
            if meas is not None:
                out["hbm_gb_s_counters"] = round(meas / (ms * 1e-3) / 1e9, 1)
                out["hbm_frac_of_8tb_s_counters"] = round(meas / (ms * 1e-3) / 8e12, 4)
        s.close()
    return out


def form_lambertw(dev, steps=5):
    """LOG model (lambda2 = 0) on the 512 x 512 image: the prox of eq. (subproblem) by Newton's method
    and by its Lambert-W closed form."""
    import paper_1404_5344_amd as foe
    import synth
    import torch
    pr = synth.config2()
    bank, theta = synth.dct_bank(), synth.theta_weights(2)
    H, W = pr.f.shape
    f = torch.from_numpy(pr.f).to(dev)
    out = {"workload": "512x512 image of the main line, LOG model (lambda 160, 0), 300 iterations"}
    for name, method in (("newton", 0), ("lambertw", 1)):
        p = foe.default_params(H, W, model=1, lambda1=pr.lam1, lambda2=0.0, max_iters=300, prox_method=method)
        s = foe.Solver(p, bank, theta)
        s.solve(f)
        t = _wall(lambda: s.solve(f), reps=steps)
        r = s.solve(f)
        out[f"mpix_it_s_{name}"] = round(H * W * r.summary["iters_done"] / t / 1e6, 1)
        out[f"psnr_{name}"] = round(synth.psnr(r.u.cpu().numpy(), pr.clean), 4)
        ms_loop, n_trials = s.last_timing()
        out[f"us_per_trial_{name}"] = round(ms_loop / n_trials * 1e3, 2)
        s.close()
    return out


def form_context(dev):
    """The run-time experiment of Sec. III-D: L = 8 images of 512x512, 481x321 and 256x256, lambda = (550, 0.02),
    300 iterations on the GPU, beside the paper's GTX 680 times (its iteration count unstated: context only).
    The FP64 oracle's times on the same images are in cpu_baseline.context."""
    import torch
    import paper_1404_5344_amd as foe
    import synth
    paper_s = {(512, 512): 0.6, (321, 481): 0.41, (256, 256): 0.2}
    bank, theta = synth.dct_bank(), synth.theta_weights(7)
    out = {"workload": "shapes+cosine images at L=8, lambda (550, 0.02), DCT bank, 300 iterations"}
    for (H, W) in synth.CONTEXT_SIZES:
        pr = synth.context_image(H, W)
        p = foe.default_params(H, W, lambda1=pr.lam1, lambda2=pr.lam2, max_iters=300, looks=8)
        s = foe.Solver(p, bank, theta)
        f = torch.from_numpy(pr.f).to(dev)
        cfg = s.autotune(f, reps=5)   # the tile shape for this size (smaller tiles fill more CUs on small images)
        r = s.solve(f)
        t = _wall(lambda: s.solve(f), reps=5)
        n_it = r.summary["iters_done"]
        out[f"{W}x{H}"] = {"gpu_ms_per_solve": round(t * 1e3, 3), "gpu_mpix_it_s": round(H * W * n_it / t / 1e6, 1),
                           "tile": TILE_SHAPES[cfg],
                           "psnr_noisy": round(synth.psnr(pr.f, pr.clean), 4),
                           "psnr_gpu": round(synth.psnr(r.u.cpu().numpy(), pr.clean), 4),
                           "paper_gtx680_s_per_solve": paper_s[(H, W)]}
        s.close()
    return out


def cpu_context():
    """The FP64 oracle on the Sec. III-D images (cpu_baseline leg): a bounded sample of iterations on all host
    cores and on one core, scaled to Mpixel-it/s and to seconds per 300 iterations."""
    import oracle
    import synth
    bank, theta = synth.dct_bank(), synth.theta_weights(7)
    cores = oracle.get_threads()
    out = {}
    for (H, W) in synth.CONTEXT_SIZES:
        pr = synth.context_image(H, W)
        po = oracle.Params(lam1=pr.lam1, lam2=pr.lam2)
        rec = {}
        for label, nthreads, iters in (("all_cores", cores, 2), ("one_core", 1, 1)):
            oracle.set_threads(nthreads)
            try:
                t0 = time.perf_counter()
                ro = oracle.ipiano(po, pr.f, bank, theta, iters, L0=1.0)
                dt = time.perf_counter() - t0
            finally:
                oracle.set_threads(cores)
            n = max(int(ro.stats.shape[0]), 1)
            rec[f"{label}_mpix_it_s"] = round(H * W * n / dt / 1e6, 4)
            rec[f"{label}_s_per_300_iterations"] = round(dt / n * 300, 1)
        out[f"{W}x{H}"] = rec
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--iters", type=int, default=300)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-forms", action="store_true")
    ap.add_argument("--unfused", action="store_true",
                    help="time the unfused gradient (z planes through HBM) on the main workload (for profiling)")
    ap.add_argument("--precision", choices=("fp32", "bf16"), default="fp32",
                    help="bf16: the main workload on the BF16 engine (for profiling; the headline is fp32)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="also run a plain device-to-device copy of this many MiB (a known-size kernel for "
                         "scaling hardware byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the workload is a single-GPU solve, and runs on several GPUs are "
              "not provided", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_1404_5344_amd as foe
    import synth

    assert torch.cuda.is_available(), "bench.py needs the GPU"
    dev = torch.device("cuda:0")
    pr = synth.config2()
    bank, theta = synth.dct_bank(), synth.theta_weights(2)
    H, W = pr.f.shape
    bf16 = args.precision == "bf16"
    p = foe.default_params(H, W, lambda1=pr.lam1, lambda2=pr.lam2, max_iters=args.iters, looks=1,
                           fusion=1 if args.unfused else 0, precision=1 if bf16 else 0)
    stream = torch.cuda.current_stream()
    s = foe.Solver(p, bank, theta, stream=stream)
    f = torch.from_numpy(pr.f).to(dev)
    out = torch.empty_like(f)
    log(f"bench: {H}x{W}, {args.iters} iterations, warmup {args.warmup}, steps {args.steps}")
    for _ in range(args.warmup):
        s.solve(f, out=out)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    iters_total = 0
    trials_total = 0
    loop_ms = 0.0
    launches = 0
    for k in range(args.steps):
        r = s.solve(f, out=out)
        iters_total += r.summary["iters_done"]
        trials_total += r.summary["total_trials"]
        ms_k, n_k = s.last_timing()
        loop_ms += ms_k
        launches += n_k
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    psnr = synth.psnr(out.cpu().numpy(), pr.clean)
    ssim = foe.ssim(out, torch.from_numpy(pr.clean.astype(np.float32)).to(dev))
    log(f"bench: {dt * 1e3 / args.steps:.3f} ms/step, psnr {psnr:.4f} dB, trials/iter {trials_total / iters_total:.4f}")

    # dominant kernel: the fused trial kernel.  Its in-solve launch time is the solver's own HIP event pair
    # on its stream around the iteration loop (graph-launched trials with the in-kernel line-search
    # decision, plus the few decide kernels and state pulls between graphs) divided by the trial launches.
    ms_launch = loop_ms / launches
    flop = FLOP_PER_PX_TRIAL * H * W
    achieved = flop / (ms_launch * 1e-3) / 1e12
    t_bar = trials_total / iters_total
    # the per-step form: 4,704 (T + 1) flop per pixel-iteration over the whole step's wall time
    flop_step = FLOP_PER_PX_TRIAL // 2 * (t_bar + 1.0) * H * W * iters_total / args.steps
    traffic = measured_traffic()
    roofline = {"bound": "alu", "achieved": round(achieved, 3), "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                "frac": round(achieved / PEAK_FP32_TFLOPS, 4), "traffic": traffic,
                "kernel": "foe_trial_kernel (forward bank on split-FP16 MFMA with FP32 accumulation, adjoint on "
                          + ("BF16 MFMA as a Toeplitz GEMM)" if bf16 else "FP32 VALU)"),
                "ms_per_launch": round(ms_launch, 5), "launches_per_step": round(launches / args.steps, 2),
                "flop_per_launch": flop,
                "frac_per_step": round(flop_step / (dt / args.steps) / 1e12 / PEAK_FP32_TFLOPS, 4),
                "frac_mixed_peak": round(achieved / MIXED_PEAK_TFLOPS, 4),
                "limiter": "VALU issue in the adjoint (plain FP32 FMAs with VGPR operands, about 2.2 cycles "
                           "per wave instruction per SIMD) and LDS/VALU in the forward (split-FP16 MFMA operands "
                           "from LDS, rcp and log per value); stage cycles in profiles/",
                "mixed_peak_tflops": round(MIXED_PEAK_TFLOPS, 1),
                "kernel_source_hash": kernel_source_hash()}
    s.close()
    # the same workload on the FP32-operand matrix-core engine
    fp32_engine = None
    p32 = None if bf16 else foe.default_params(H, W, lambda1=pr.lam1, lambda2=pr.lam2, max_iters=args.iters, looks=1,
                             fusion=1 if args.unfused else 0, engine=foe.ENGINE_MFMA)
    if p32 is not None:
        s32 = foe.Solver(p32, bank, theta, stream=stream)
        out32 = torch.empty_like(f)
        s32.solve(f, out=out32)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        it32 = 0
        loop32, n32 = 0.0, 0
        for k in range(args.steps):
            it32 += s32.solve(f, out=out32).summary["iters_done"]
            ms_k, n_k = s32.last_timing()
            loop32 += ms_k
            n32 += n_k
        torch.cuda.synchronize()
        dt32 = time.perf_counter() - t0
        fp32_engine = {"value": round(H * W * it32 / dt32 / 1e6, 2),
                       "ms_per_step": round(dt32 * 1e3 / args.steps, 4), "ms_per_launch": round(loop32 / n32, 5),
                       "psnr_db": round(synth.psnr(out32.cpu().numpy(), pr.clean), 4)}
        s32.close()
        log(f"bench: FP32-operand engine {fp32_engine}")
    if args.copy_calibration:
        n = args.copy_calibration * (1 << 20) // 4
        a = torch.ones(n, device=dev)
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        log(f"bench: copy calibration, {n * 4} bytes read and written per copy")
    value = H * W * iters_total / dt / 1e6
    res = {
        "metric": METRIC, "value": round(value, 2), "unit": "Mpixel-iters/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(dt * 1e3 / args.steps, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": ("bf16 (adjoint bank; forward as split-f16 products)" if bf16
                                                   else "f32 (forward bank as split-f16 products)"), "data": "synthetic",
        "config": {"workload": "512x512 shapes+cosine image, L=1 speckle, COMBINED model (lambda 160, 0.004), "
                               "48 DCT 7x7 filters, SYMMETRIC boundary, beta 0.8, backtracking, "
                               f"{args.iters} iterations per step" + (", gradient unfused" if args.unfused else "")
                               + (", BF16 engine" if bf16 else ""),
                   "pixels": H * W, "iterations": args.iters, "trials_per_iter": round(trials_total / iters_total, 4),
                   "psnr_db": round(psnr, 4), "ssim": round(ssim, 5),
                   "forward_bank": "split-FP16 MFMA: FP32 operand = FP16 head + FP16 tail / 4096, three exact "
                                   "FP16 products per FP32 product, FP32 accumulation"},
        "roofline": roofline,
    }
    if fp32_engine is not None:
        res["fp32_operand_engine"] = fp32_engine
    if not args.no_forms:
        forms = {}
        for name, fn in (("batched", form_batched), ("bf16", form_bf16), ("warm_start", form_warm),
                         ("warm_start_eval", form_warm_eval),
                         ("unfused", form_unfused), ("lambertw", form_lambertw), ("context", form_context)):
            t = time.perf_counter()
            log(f"bench: form {name}")
            forms[name] = fn(dev)
            log(f"bench: form {name}: {forms[name]} ({time.perf_counter() - t:.1f} s)")
        res["forms"] = forms
    if not args.no_cpu_baseline:
        log("bench: timing the FP64 oracle on the host")
        res["cpu_baseline"] = cpu_baseline(pr, bank, theta)
        if not args.no_forms:
            res["cpu_baseline"]["context"] = cpu_context()
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
