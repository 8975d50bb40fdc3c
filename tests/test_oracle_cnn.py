"""Pins of the FP64 warm-start network oracle (CPU only): the chain-rule gradient against
central differences of the loss, and the forward pass against an independent NumPy/SciPy
evaluation of the same network (scipy.signal.correlate2d with zero padding)."""
import numpy as np
import scipy.signal as ss

import oracle


def _params(seed=0, scale=0.3):
    r = np.random.default_rng(seed)
    return r.standard_normal(oracle.cnn_num_params()) * scale


def _net_numpy(params, f):
    a = np.log(f) - oracle.CNN_SHIFT
    a = a[None]
    o = 0
    for l, (cin, cout) in enumerate(oracle.CNN_LAYERS):
        w = params[o:o + cout * cin * 9].reshape(cout, cin, 3, 3); o += cout * cin * 9
        b = params[o:o + cout]; o += cout
        out = np.empty((cout,) + f.shape)
        for co in range(cout):
            out[co] = b[co] + sum(ss.correlate2d(a[ci], w[co, ci], mode="same", boundary="fill") for ci in range(cin))
        a = np.maximum(out, 0) if l < 5 else out
    return np.log(f) + a[0]


def test_parameter_count():
    assert oracle.cnn_num_params() == 320 + 4 * 9248 + 289


def test_forward_matches_scipy():
    r = np.random.default_rng(1)
    f = r.uniform(10, 250, (9, 11))
    p = _params(2, 0.1)
    assert np.max(np.abs(oracle.cnn_forward(p, f) - _net_numpy(p, f))) <= 1e-10


def test_gradient_finite_differences():
    r = np.random.default_rng(3)
    f = r.uniform(10, 250, (2, 6, 7))
    ut = f * np.exp(0.3 * r.standard_normal(f.shape))
    p = _params(4, 0.15)
    loss, g = oracle.cnn_loss_grad(p, f, ut)
    sizes = [cout * cin * 9 + cout for cin, cout in oracle.CNN_LAYERS]
    starts = np.cumsum([0] + sizes[:-1])
    idx = []
    for s, n in zip(starts, sizes):   # a few weights and the last bias of every layer
        idx += list(s + r.choice(n - 1, 4, replace=False)) + [s + n - 1]
    h = 1e-6
    for i in idx:
        e = np.zeros_like(p); e[i] = h
        fd = (oracle.cnn_loss_grad(p + e, f, ut, False)[0] - oracle.cnn_loss_grad(p - e, f, ut, False)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1e-3, abs(g[i])), (i, fd, g[i])
    d = r.standard_normal(p.size)
    fd = (oracle.cnn_loss_grad(p + h * d, f, ut, False)[0] - oracle.cnn_loss_grad(p - h * d, f, ut, False)[0]) / (2 * h)
    assert abs(fd - g @ d) <= 1e-6 * abs(g @ d)


def test_relu_margin_special_cases():
    # zero weights: every pre-activation equals its layer's bias
    import oracle
    p = np.zeros(oracle.cnn_num_params())
    off = 0
    biases = [0.5, 0.7, 0.3, 0.9, 0.6, 0.2]
    for l, (ci, co) in enumerate(oracle.CNN_LAYERS):
        off += co * ci * 9
        p[off:off + co] = biases[l]
        off += co
    f = np.full((1, 5, 6), 3.0)
    assert oracle.cnn_relu_margin(p, f) == 0.3      # layers 1-5 only; the output layer has no ReLU
    p[oracle.CNN_LAYERS[0][1] * 9:oracle.CNN_LAYERS[0][1] * 10] = -0.05
    assert oracle.cnn_relu_margin(p, f) == 0.05
