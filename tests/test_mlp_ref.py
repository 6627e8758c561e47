"""Pins of the float64 proposal-network reference (finite differences, closed forms)."""
import numpy as np

from oracle import mlp_ref as R


def test_bf16_rounding_known_values():
    x = np.array([1.0, 1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -9, -2.5, 0.0, 65280.0, 1.0 + 2.0 ** -7],
                 dtype=np.float32)
    got = R.bf16(x)
    # 1 + 2^-8 is halfway between 1 and 1 + 2^-7: ties to even -> 1; 1 + 3*2^-9 rounds up
    assert list(got) == [1.0, 1.0, 1.0 + 2.0 ** -7, -2.5, 0.0, 65280.0, 1.0 + 2.0 ** -7]


def test_zero_weights_give_output_bias():
    din, h, dout = 5, 4, 3
    p = np.zeros(R.num_params(din, h, dout))
    p[-dout:] = [0.5, -1.0, 2.0]
    d, _ = R.forward(p, np.ones((2, din)), din, h, dout, mirror=False)
    assert np.array_equal(d, np.tile([0.5, -1.0, 2.0], (2, 1)))


def test_loss_gradient_wrt_output_closed_form():
    # with W3 = 0 and b3 free, dL/db3 = mean_b -(sigmoid(z) - y), z = -(lam + b3)
    din, h, dout = 3, 2, 4
    rng = np.random.default_rng(0)
    p = rng.normal(0, 0.3, R.num_params(din, h, dout))
    W1, b1, W2, b2, W3, b3 = R.split(p, din, h, dout)
    W3[:] = 0.0
    x = rng.integers(0, 2, (6, din))
    y = rng.integers(0, 2, (6, dout))
    lam = rng.uniform(1, 5, dout)
    _, g = R.loss_and_grads(p, x, y, lam, din, h, dout, mirror=False)
    z = -(lam[None, :] + b3[None, :])
    want = (-(1 / (1 + np.exp(-z)) - y)).mean(0)
    assert np.allclose(g[-dout:], want, rtol=1e-12, atol=1e-14)


def test_gradients_match_finite_differences():
    din, h, dout = 6, 5, 4
    rng = np.random.default_rng(1)
    p = rng.normal(0, 0.5, R.num_params(din, h, dout))
    x = rng.integers(0, 2, (7, din)).astype(float)
    y = rng.integers(0, 2, (7, dout))
    lam = rng.uniform(0.5, 4, dout)
    _, g = R.loss_and_grads(p, x, y, lam, din, h, dout, mirror=False)
    eps = 1e-6
    for i in rng.choice(p.size, 40, replace=False):
        e = np.zeros_like(p)
        e[i] = eps
        lp, _ = R.loss_and_grads(p + e, x, y, lam, din, h, dout, mirror=False)
        lm, _ = R.loss_and_grads(p - e, x, y, lam, din, h, dout, mirror=False)
        fd = (lp - lm) / (2 * eps)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(fd)), (i, fd, g[i])


def test_adam_first_step_is_sign_step():
    g = np.array([0.3, -2.0, 1e-3])
    p1, m, v = R.adam(np.zeros(3), g, np.zeros(3), np.zeros(3), 1, lr=0.01)
    assert np.allclose(p1, -0.01 * np.sign(g), rtol=1e-4)
