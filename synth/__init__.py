"""Seeded synthetic inputs for the FoE despeckling path.

This module is shared by the tests, the benchmark and the oracle-side checks.
It holds input *generation* only -- none of the method's arithmetic (no
filtering, no energy, no prox, no iPiano step).  Every array is generated in
float64 from ``numpy.random.Generator(PCG64(SeedSequence([config_id, index,
purpose])))`` and cast once to float32, so the HIP path and the oracle consume
identical float32 inputs.

Purposes (the third seed word):
  0 clean image, 1 speckle, 2 filter weights theta, 3 cosine field,
  4 Gaussian random field, 5 point targets, 6 random filter bank.

Paper passages the generators stand in for:
  * speckle: the Nakagami amplitude law with L looks (Sec. II-B, the
    likelihood p(f|u) before eq. (dataterm1)).  An amplitude f with that law is
    f = u * sqrt(n), n ~ Gamma(L, scale 1/L) (the intensity f^2 is u^2 times a
    unit-mean Gamma variate).  This reading reproduces the gaps between the
    "Noisy" PSNR entries of Table 2 for L = 8, 3, 1.
  * filter bank: the paper's 48 learned 7x7 filters (Fig. 1) are not
    published with the text; the 48 non-DC 7x7 DCT-II basis filters stand in.
  * images: 8-bit amplitude scale, as in the test images of Sec. III.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

PURPOSE_CLEAN = 0
PURPOSE_SPECKLE = 1
PURPOSE_THETA = 2
PURPOSE_COSINE = 3
PURPOSE_GRF = 4
PURPOSE_TARGETS = 5
PURPOSE_RANDOM_BANK = 6

FLT_MIN = float(np.finfo(np.float32).tiny)


def rng(config_id: int, index: int, purpose: int) -> np.random.Generator:
    """The one seeding rule used by every generator."""
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([int(config_id), int(index), int(purpose)])))


# ---------------------------------------------------------------- filter bank
def dct_bank(ksize: int = 7) -> np.ndarray:
    """The (ksize^2 - 1) non-DC separable DCT-II basis filters, row-major (p, q) order.

    k_pq[a][b] = c_p(a) c_q(b), c_p(n) = s_p cos(pi (2n+1) p / (2 ksize)),
    s_0 = sqrt(1/ksize), s_p = sqrt(2/ksize).  Returns float32 [48, 7, 7].
    """
    n = np.arange(ksize, dtype=np.float64)
    c = np.empty((ksize, ksize), dtype=np.float64)
    for p in range(ksize):
        s = math.sqrt(1.0 / ksize) if p == 0 else math.sqrt(2.0 / ksize)
        c[p] = s * np.cos(np.pi * (2.0 * n + 1.0) * p / (2.0 * ksize))
    bank = []
    for p in range(ksize):
        for q in range(ksize):
            if p == 0 and q == 0:
                continue
            bank.append(np.outer(c[p], c[q]))
    return np.asarray(bank, dtype=np.float64).astype(np.float32)


def theta_weights(config_id: int, nf: int = 48, lo: float = 0.05, hi: float = 0.5) -> np.ndarray:
    """Positive filter weights theta_i ~ U[lo, hi] (float32 [nf])."""
    return rng(config_id, 0, PURPOSE_THETA).uniform(lo, hi, size=nf).astype(np.float32)


def random_bank(seed: int, nf: int = 48, ksize: int = 7) -> np.ndarray:
    """Seeded random non-separable filters (zero-mean, unit-norm rows), float32 [nf, k, k].

    Used to check that nothing in the path relies on the DCT bank's structure
    (separability, flip symmetry)."""
    r = rng(seed, 0, PURPOSE_RANDOM_BANK)
    k = r.standard_normal((nf, ksize * ksize))
    k -= k.mean(axis=1, keepdims=True)
    k /= np.linalg.norm(k, axis=1, keepdims=True)
    return k.reshape(nf, ksize, ksize).astype(np.float32)


def learned_style_bank(seed: int, nf: int = 48, ksize: int = 7) -> tuple[np.ndarray, np.ndarray]:
    """Seeded filters of the kind a learned FoE bank has (Sec. II-A, Fig. 1): not zero-sum (each filter
    keeps a random mean), norms spread log-uniformly over [0.2, 5], and weights theta_i ~ U[0.05, 5].
    Returns (filters float32 [nf, k, k], theta float32 [nf])."""
    r = rng(seed, 1, PURPOSE_RANDOM_BANK)
    k = r.standard_normal((nf, ksize * ksize)) + r.uniform(-0.5, 0.5, (nf, 1))
    k /= np.linalg.norm(k, axis=1, keepdims=True)
    k *= np.exp(r.uniform(np.log(0.2), np.log(5.0), (nf, 1)))
    theta = r.uniform(0.05, 5.0, nf)
    return k.reshape(nf, ksize, ksize).astype(np.float32), theta.astype(np.float32)


# ---------------------------------------------------------------- clean images
def shapes_image(config_id: int, index: int, H: int, W: int, n_shapes: int = 12,
                 lo: float = 10.0, hi: float = 255.0) -> np.ndarray:
    """Piecewise-constant image: U[lo,hi] background plus n_shapes axis-aligned
    rectangles / ellipses (probability 1/2 each), centre ~ U(image), half-axes
    ~ U[H/16, H/4] x U[W/16, W/4], value ~ U[lo, hi], painted in order (float64)."""
    r = rng(config_id, index, PURPOSE_CLEAN)
    img = np.full((H, W), r.uniform(lo, hi), dtype=np.float64)
    yy, xx = np.meshgrid(np.arange(H, dtype=np.float64), np.arange(W, dtype=np.float64), indexing="ij")
    for _ in range(n_shapes):
        is_rect = r.uniform() < 0.5
        cy = r.uniform(0, H)
        cx = r.uniform(0, W)
        ay = r.uniform(H / 16.0, H / 4.0)
        ax = r.uniform(W / 16.0, W / 4.0)
        val = r.uniform(lo, hi)
        if is_rect:
            m = (np.abs(yy - cy) <= ay) & (np.abs(xx - cx) <= ax)
        else:
            m = ((yy - cy) / ay) ** 2 + ((xx - cx) / ax) ** 2 <= 1.0
        img[m] = val
    return img


def cosine_field(config_id: int, index: int, H: int, W: int, amp: float = 30.0) -> np.ndarray:
    """A * cos(2 pi (ky y / H + kx x / W) + phi), (ky, kx) ~ U{1,2,3}^2, phi ~ U[0, 2 pi)."""
    r = rng(config_id, index, PURPOSE_COSINE)
    ky = int(r.integers(1, 4))
    kx = int(r.integers(1, 4))
    phi = r.uniform(0.0, 2.0 * np.pi)
    y = np.arange(H, dtype=np.float64)[:, None]
    x = np.arange(W, dtype=np.float64)[None, :]
    return amp * np.cos(2.0 * np.pi * (ky * y / H + kx * x / W) + phi)


def shapes_cosine_image(config_id: int, index: int, H: int, W: int) -> np.ndarray:
    """Shapes image plus a random-phase cosine gradient field, clipped to [10, 255]."""
    return np.clip(shapes_image(config_id, index, H, W) + cosine_field(config_id, index, H, W), 10.0, 255.0)


def grf_sar_image(config_id: int, index: int, H: int, W: int, exponent: float = -2.5,
                  mean: float = 100.0, n_targets: int = 40, target_factor: float = 20.0) -> np.ndarray:
    """SAR-like amplitude: exp of a Gaussian random field with power spectrum
    |k|^exponent (DC zeroed, unit std), scaled to the given mean, plus single-pixel
    point targets at target_factor * mean."""
    r = rng(config_id, index, PURPOSE_GRF)
    noise = r.standard_normal((H, W))
    ky = np.fft.fftfreq(H)[:, None]
    kx = np.fft.fftfreq(W)[None, :]
    kk = np.sqrt(ky * ky + kx * kx)
    amp = np.zeros_like(kk)
    nz = kk > 0
    amp[nz] = kk[nz] ** (exponent / 2.0)   # power ~ |k|^exponent => amplitude ~ |k|^(exponent/2)
    g = np.real(np.fft.ifft2(np.fft.fft2(noise) * amp))
    g = (g - g.mean()) / g.std()
    clean = np.exp(g)
    clean *= mean / clean.mean()
    rt = rng(config_id, index, PURPOSE_TARGETS)
    ys = rt.integers(0, H, size=n_targets)
    xs = rt.integers(0, W, size=n_targets)
    clean[ys, xs] = target_factor * mean
    return clean


# ---------------------------------------------------------------- speckle
def speckle(clean: np.ndarray, looks: int, config_id: int, index: int, literal: bool = False) -> np.ndarray:
    """Observed amplitude under L-look Nakagami speckle, cast to float32 and floored at FLT_MIN.

    Default (Nakagami amplitude): f = c * sqrt(n), n ~ Gamma(L, 1/L).
    literal=True gives f = c * n (kept only as a generator option)."""
    r = rng(config_id, index, PURPOSE_SPECKLE)
    n = r.gamma(shape=float(looks), scale=1.0 / float(looks), size=clean.shape)
    f = clean * (n if literal else np.sqrt(n))
    f32 = f.astype(np.float32)
    return np.maximum(f32, np.float32(FLT_MIN))


def psnr(u: np.ndarray, clean: np.ndarray, peak: float = 255.0) -> float:
    """PSNR = 10 log10(peak^2 / MSE) over all pixels, u not clipped."""
    d = np.asarray(u, np.float64) - np.asarray(clean, np.float64)
    mse = float(np.mean(d * d))
    return 10.0 * math.log10(peak * peak / mse)


# ---------------------------------------------------------------- lambda table
# lambda1, lambda2 the paper prints for L = 1, 3, 8 (Sec. III-B); other L are
# interpolated linearly in L, and L > 8 takes the L = 8 values.
PAPER_LAMBDA = {1: (160.0, 0.004), 3: (310.0, 0.008), 8: (550.0, 0.02)}


def default_lambdas(looks: int) -> tuple[float, float]:
    if looks in PAPER_LAMBDA:
        return PAPER_LAMBDA[looks]
    if looks >= 8:
        return PAPER_LAMBDA[8]
    lo, hi = (1, 3) if looks < 3 else (3, 8)
    t = (looks - lo) / (hi - lo)
    a, b = PAPER_LAMBDA[lo], PAPER_LAMBDA[hi]
    return (a[0] + t * (b[0] - a[0]), a[1] + t * (b[1] - a[1]))


# ---------------------------------------------------------------- configs
@dataclass
class Problem:
    clean: np.ndarray      # float64 [H, W]
    f: np.ndarray          # float32 [H, W]
    looks: int
    lam1: float
    lam2: float
    peak: float


def config1(index: int = 0, H: int = 64, W: int = 64) -> Problem:
    """64x64 shapes image, L = 4 speckle."""
    clean = shapes_image(1, index, H, W)
    f = speckle(clean, 4, 1, index)
    l1, l2 = default_lambdas(4)
    return Problem(clean, f, 4, l1, l2, 255.0)


def config2(index: int = 0, H: int = 512, W: int = 512, looks: int = 1) -> Problem:
    """512x512 shapes + cosine image, single-look speckle."""
    clean = shapes_cosine_image(2, index, H, W)
    f = speckle(clean, looks, 2, index)
    l1, l2 = default_lambdas(looks)
    return Problem(clean, f, looks, l1, l2, 255.0)


def config3_sizes(n: int = 64) -> list[tuple[int, int, int]]:
    """(H, W, L) of the uneven batch: sides ~ U{128, 192, ..., 1024}, L ~ U{1, 2, 4, 8}."""
    r = rng(3, 0, PURPOSE_CLEAN)
    sides = np.arange(128, 1025, 64)
    out = []
    for _ in range(n):
        H = int(r.choice(sides))
        W = int(r.choice(sides))
        L = int(r.choice([1, 2, 4, 8]))
        out.append((H, W, L))
    return out


def config3_image(index: int, H: int, W: int, looks: int) -> Problem:
    clean = shapes_cosine_image(3, index + 1, H, W)
    f = speckle(clean, looks, 3, index + 1)
    l1, l2 = default_lambdas(looks)
    return Problem(clean, f, looks, l1, l2, 255.0)


def config4(index: int = 0, H: int = 2048, W: int = 2048) -> Problem:
    """SAR-like 2048^2 tile, L = 1; PSNR peak = max(clean)."""
    clean = grf_sar_image(4, index, H, W)
    f = speckle(clean, 1, 4, index)
    l1, l2 = default_lambdas(1)
    return Problem(clean, f, 1, l1, l2, float(clean.max()))


def config5_train(index: int, H: int = 128, W: int = 128) -> Problem:
    """Warm-start training image: shapes image at 128^2, L alternating 1 / 4."""
    looks = 1 if index % 2 == 0 else 4
    clean = shapes_image(5, index, H, W)
    f = speckle(clean, looks, 5, index)
    l1, l2 = default_lambdas(looks)
    return Problem(clean, f, looks, l1, l2, 255.0)


def config5_eval(index: int, H: int = 512, W: int = 512, looks: int = 1) -> Problem:
    """Held-out warm-start evaluation image (disjoint seed space: config id 50)."""
    clean = shapes_cosine_image(50, index, H, W)
    f = speckle(clean, looks, 50, index)
    l1, l2 = default_lambdas(looks)
    return Problem(clean, f, looks, l1, l2, 255.0)


# ---------------------------------------------------------------- presets of the paper's other experiments
# The real-SAR experiment (Sec. III-C): an L = 5 image despeckled with lambda1 = 50, lambda2 = 0.15.  The
# JSTARS image is not available; a SAR-like GRF image with point targets stands in for it.
SAR_PRESET_LOOKS = 5
SAR_PRESET_LAMBDA = (50.0, 0.15)


def sar_preset(index: int = 0, H: int = 256, W: int = 256) -> Problem:
    """SAR-like image (GRF with point targets, config id 6) under L = 5 speckle, with the real-SAR
    lambdas of Sec. III-C; PSNR peak = max(clean)."""
    clean = grf_sar_image(6, index, H, W)
    f = speckle(clean, SAR_PRESET_LOOKS, 6, index)
    return Problem(clean, f, SAR_PRESET_LOOKS, SAR_PRESET_LAMBDA[0], SAR_PRESET_LAMBDA[1], float(clean.max()))


# The run-time experiment (Sec. III-D): L = 8 images of 512 x 512, 481 x 321 and 256 x 256 (the combined
# model with lambda1 = 550, lambda2 = 0.02, the L = 8 values of Sec. III-B).
CONTEXT_SIZES = ((512, 512), (321, 481), (256, 256))   # (H, W): 481 x 321 as 481 wide


def context_image(H: int, W: int, index: int = 0) -> Problem:
    """Shapes + cosine image (config id 7) of the given size under L = 8 speckle, lambda = (550, 0.02)."""
    clean = shapes_cosine_image(7, index, H, W)
    f = speckle(clean, 8, 7, index)
    l1, l2 = default_lambdas(8)
    return Problem(clean, f, 8, l1, l2, 255.0)
