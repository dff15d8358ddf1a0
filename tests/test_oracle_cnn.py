"""Pins of the oracle CNN (FP64 forward/backward of the learned stage), CPU only."""
import numpy as np
import pytest

from oracle import cnn


def test_one_layer_is_a_correlation():
    rng = np.random.default_rng(0)
    x = rng.standard_normal((2, 3, 11))
    w = rng.standard_normal((4, 3, 5))
    b = rng.standard_normal(4)
    y = cnn.conv1d(x, w, b)
    for bb in range(2):
        for o in range(4):
            ref = b[o] + sum(np.correlate(np.pad(x[bb, c], 2), w[o, c], mode="valid") for c in range(3))
            assert np.allclose(y[bb, o], ref, atol=1e-12)


def test_dilated_layer_is_a_correlation_with_the_stuffed_kernel():
    rng = np.random.default_rng(5)
    x = rng.standard_normal((2, 3, 23))
    w = rng.standard_normal((4, 3, 5))
    b = rng.standard_normal(4)
    for d in (2, 3, 4):
        y = cnn.conv1d(x, w, b, d)
        for bb in range(2):
            for o in range(4):
                ws = [np.zeros(4 * d + 1) for _ in range(3)]
                for c in range(3):
                    ws[c][::d] = w[o, c]  # taps at offsets (k - 2) d
                ref = b[o] + sum(np.correlate(np.pad(x[bb, c], 2 * d), ws[c], mode="valid") for c in range(3))
                assert np.allclose(y[bb, o], ref, atol=1e-12)
        # a dilated output point sees only inputs at multiples of d from it
        xi = np.zeros((1, 3, 23))
        xi[0, 1, 11] = 1.0
        yi = cnn.conv1d(xi, w, np.zeros(4), d)
        nz = set(np.nonzero(np.abs(yi[0]).sum(axis=0))[0].tolist())
        assert nz <= {11 + m * d for m in range(-2, 3)}


@pytest.mark.parametrize("dil", [None, (1, 2, 3)])
def test_gradients_match_central_differences(dil):
    rng = np.random.default_rng(1)
    params = cnn.init_params(channels=(3, 4, 4, 2), K=3, seed=2)
    params = [(w, rng.standard_normal(b.shape) * 0.1) for w, b in params]
    x = rng.standard_normal((3, 3, 13))
    t = rng.standard_normal((3, 2, 13))
    y, acts = cnn.forward(params, x, dil)
    grads = cnn.backward(params, acts, cnn.loss_grad(y, t), dil)
    eps = 1e-6
    for li, (w, b) in enumerate(params):
        for arr, g in ((w, grads[li][0]), (b, grads[li][1])):
            flat = arr.reshape(-1)
            gflat = g.reshape(-1)
            for idx in rng.choice(flat.size, size=min(6, flat.size), replace=False):
                old = flat[idx]
                flat[idx] = old + eps
                lp = cnn.loss(cnn.forward(params, x, dil)[0], t)
                flat[idx] = old - eps
                lm = cnn.loss(cnn.forward(params, x, dil)[0], t)
                flat[idx] = old
                fd = (lp - lm) / (2 * eps)
                assert abs(fd - gflat[idx]) <= 1e-6 * max(1.0, abs(fd)), (li, idx, fd, gflat[idx])


@pytest.mark.parametrize("dil", [None, (1, 2, 4, 8)])
def test_translation_equivariance_away_from_the_edges(dil):
    rng = np.random.default_rng(3)
    params = cnn.init_params(seed=4)
    x = np.zeros((1, 8, 200))
    x[0, :, 90:100] = rng.standard_normal((8, 10))
    y1, _ = cnn.forward(params, x, dil)
    y2, _ = cnn.forward(params, np.roll(x, 7, axis=2), dil)
    assert np.allclose(np.roll(y1, 7, axis=2)[:, :, 70:130], y2[:, :, 70:130], atol=1e-12)


def test_bf16_rounding():
    v = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 2 ** -9, 3.14159265, -2.5e-3])
    r = cnn.bf16_round(v)
    assert r[0] == 1.0
    assert r[1] == 1.0  # exactly halfway between 1 and 1 + 2^-7: ties to even
    assert r[2] == 1.0
    assert np.all(np.abs(r - v) <= np.abs(v) * 2 ** -8)
