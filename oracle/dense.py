"""Dense brute force for tiny images -- TEST INFRASTRUCTURE.

The paper treats each filter as an N x N sparse matrix K_i with K_i u equal to
the 2-D convolution k_i * u (Sec. II-C, the text after the gradient of F).
This module materialises those matrices explicitly for images of a few dozen
pixels: P maps the image to its 3-pixel extension, C_i is the valid true
convolution on the extension, K_i = C_i P.  Energies and gradients then follow
from plain matrix-vector products; K_i^T is the NumPy transpose.  It shares no
code with foe_oracle.c and serves as an independent pin for it.
"""
from __future__ import annotations

import numpy as np

R = 3
KS = 7


def _src(q: int, n: int, bc: int) -> int:
    if 0 <= q < n:
        return q
    if bc == 0:      # half-sample symmetric: ... c b a | a b c ... | ... c b a
        return -1 - q if q < 0 else 2 * n - 1 - q
    if bc == 2:      # periodic
        return q % n
    return -1        # zero


def extension_matrix(H: int, W: int, bc: int) -> np.ndarray:
    He, We = H + 2 * R, W + 2 * R
    P = np.zeros((He * We, H * W))
    for ey in range(He):
        sy = _src(ey - R, H, bc)
        for ex in range(We):
            sx = _src(ex - R, W, bc)
            if sy >= 0 and sx >= 0:
                P[ey * We + ex, sy * W + sx] = 1.0
    return P


def conv_matrix(H: int, W: int, k: np.ndarray) -> np.ndarray:
    """C: valid true convolution on the extension; output pixel p reads
    extension sample (p_y + 3 - a, p_x + 3 - b) with weight k[a, b]."""
    He, We = H + 2 * R, W + 2 * R
    C = np.zeros((H * W, He * We))
    for py in range(H):
        for px in range(W):
            for a in range(KS):
                for b in range(KS):
                    ey = py + R - a + R
                    ex = px + R - b + R
                    C[py * W + px, ey * We + ex] += k[a, b]
    return C


def k_matrices(H: int, W: int, bank: np.ndarray, bc: int) -> list[np.ndarray]:
    P = extension_matrix(H, W, bc)
    return [conv_matrix(H, W, np.asarray(k, np.float64)) @ P for k in bank]


def rho(x):
    return np.log1p(x * x)


def drho(x):
    return 2.0 * x / (1.0 + x * x)


def amplitude(x, model):
    return np.exp(x) if model in (0, 1) else x


def energy_F(x: np.ndarray, Ks, theta, model: int) -> float:
    u = amplitude(np.asarray(x, np.float64).ravel(), model)
    return float(sum(t * rho(K @ u).sum() for K, t in zip(Ks, theta)))


def grad_F(x: np.ndarray, Ks, theta, model: int) -> np.ndarray:
    u = amplitude(np.asarray(x, np.float64).ravel(), model)
    g = sum(t * (K.T @ drho(K @ u)) for K, t in zip(Ks, theta))
    if model in (0, 1):
        g = u * g
    return g.reshape(np.shape(x))


def energy_G(x, f, model, lam1, lam2) -> float:
    x = np.asarray(x, np.float64); f2 = np.asarray(f, np.float64) ** 2
    if model == 2:
        return float(0.5 * lam1 * np.sum(x * x - 2 * f2 * np.log(x)))
    g = 0.5 * lam1 * np.sum(2 * x + f2 * np.exp(-2 * x))
    if model == 0:
        g += 0.5 * lam2 * np.sum(np.exp(2 * x) - 2 * f2 * x)
    return float(g)
