"""Pins of the oracle's filter operators K_i and K_i^T (CPU only).

K_i u is the 2-D convolution of the image with k_i (Sec. II-A, eq. (FOEmodel);
Sec. II-C: K_i is the N x N sparse matrix of that convolution).  The pins:
  * scipy.ndimage.convolve in the three boundary modes (library routine),
  * periodic convolution through the FFT (library routine),
  * explicit dense K_i matrices at tiny sizes (brute force), for K and K^T,
  * the adjoint identity <K u, v> = <u, K^T v> at larger, ragged sizes.
"""
import numpy as np
import pytest
import scipy.ndimage as ndi

import oracle
import synth
from oracle import dense

BCS = [(oracle.SYMMETRIC, "reflect"), (oracle.ZERO, "constant"), (oracle.PERIODIC, "wrap")]


@pytest.mark.parametrize("bc,mode", BCS)
@pytest.mark.parametrize("shape", [(8, 8), (13, 21), (40, 33)])
def test_forward_matches_scipy_convolve(bc, mode, shape):
    r = np.random.default_rng(1)
    x = r.uniform(10, 255, shape)
    for k in list(synth.random_bank(3)[:4]) + list(synth.dct_bank()[[0, 7, 47]]):
        k = np.asarray(k, np.float64)
        ref = ndi.convolve(x, k, mode=mode, cval=0.0)
        got = oracle.forward(x, k, bc)
        assert np.max(np.abs(got - ref)) <= 1e-12 * np.max(np.abs(ref))


def test_periodic_forward_matches_fft():
    r = np.random.default_rng(2)
    H, W = 24, 31
    x = r.standard_normal((H, W))
    k = np.asarray(synth.random_bank(4)[5], np.float64)
    kp = np.zeros((H, W))
    # place k centred at (0, 0): tap (a, b) multiplies x(p + 3 - a, p + 3 - b)  => offset (a - 3, b - 3)
    for a in range(7):
        for b in range(7):
            kp[(a - 3) % H, (b - 3) % W] += k[a, b]
    ref = np.real(np.fft.ifft2(np.fft.fft2(x) * np.fft.fft2(kp)))
    got = oracle.forward(x, k, oracle.PERIODIC)
    assert np.max(np.abs(got - ref)) <= 1e-12 * np.max(np.abs(ref))


@pytest.mark.parametrize("bc", [oracle.SYMMETRIC, oracle.ZERO, oracle.PERIODIC])
@pytest.mark.parametrize("shape", [(8, 8), (7, 9), (4, 5)])
def test_dense_matrices_forward_and_transpose(bc, shape):
    H, W = shape
    bank = synth.random_bank(7)[:3]
    Ks = dense.k_matrices(H, W, bank, bc)
    N = H * W
    for i, k in enumerate(bank):
        # Column j of the oracle's K is K e_j; column j of its K^T is K^T e_j.
        Kora = np.zeros((N, N))
        KTora = np.zeros((N, N))
        for j in range(N):
            e = np.zeros(N); e[j] = 1.0
            Kora[:, j] = oracle.forward(e.reshape(H, W), k, bc).ravel()
            KTora[:, j] = oracle.adjoint(e.reshape(H, W), k, bc).ravel()
        assert np.max(np.abs(Kora - Ks[i])) <= 1e-13
        assert np.max(np.abs(KTora - Ks[i].T)) <= 1e-13
        assert np.max(np.abs(KTora - Kora.T)) <= 1e-13


@pytest.mark.parametrize("bc", [oracle.SYMMETRIC, oracle.ZERO, oracle.PERIODIC])
@pytest.mark.parametrize("shape", [(37, 53), (64, 64), (5, 70)])
def test_adjoint_identity(bc, shape):
    r = np.random.default_rng(3)
    u = r.standard_normal(shape)
    v = r.standard_normal(shape)
    for k in synth.random_bank(9)[:3]:
        lhs = float(np.sum(oracle.forward(u, k, bc) * v))
        rhs = float(np.sum(u * oracle.adjoint(v, k, bc)))
        assert abs(lhs - rhs) <= 1e-13 * (abs(lhs) + np.sqrt(u.size))


def test_dct_bank_is_orthonormal_and_zero_sum():
    bank = synth.dct_bank().astype(np.float64).reshape(48, 49)
    gram = bank @ bank.T
    assert np.max(np.abs(gram - np.eye(48))) < 1e-6  # float32 storage
    assert np.max(np.abs(bank.sum(axis=1))) < 1e-6
