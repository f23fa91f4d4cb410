"""Pins of the FP64 CPU reference of the surrogate network.

The reference gradient is checked against central finite differences of its
own loss (directional derivatives along random directions and along single
coordinates of every layer), and the bf16 rounding helper against exactly
representable values and the round-to-nearest-even rule.
"""
import numpy as np
import pytest

from oracle import mlp_oracle as mo


def _problem(seed, M=16, out=28, F=22):
    rng = np.random.default_rng(seed)
    theta = np.zeros(mo.NPARAMS)
    for l, ((n, k), (ow, ob)) in enumerate(zip(mo.SHAPES, mo.OFFSETS)):
        kv = F if l == 0 else k
        nv = out if l == 3 else n
        W = np.zeros((n, k))
        W[:nv, :kv] = rng.standard_normal((nv, kv)) * np.sqrt(2.0 / kv)
        theta[ow:ow + n * k] = W.ravel()
        theta[ob:ob + nv] = 0.1 * rng.standard_normal(nv)
    X = np.zeros((M, mo.PAD))
    X[:, :F] = rng.standard_normal((M, F))
    T = rng.standard_normal((M, out))
    wo = rng.uniform(0.5, 2.0, size=out)
    return theta, X, T, wo


@pytest.mark.parametrize("seed", [0, 1])
def test_gradient_matches_central_differences(seed):
    theta, X, T, wo = _problem(seed)
    _, g = mo.loss_and_grad(theta, X, T, wo)
    rng = np.random.default_rng(100 + seed)
    h = 1e-5
    for _ in range(4):
        v = rng.standard_normal(mo.NPARAMS)
        lp, _ = mo.loss_and_grad(theta + h * v, X, T, wo)
        lm, _ = mo.loss_and_grad(theta - h * v, X, T, wo)
        fd = (lp - lm) / (2 * h)
        assert abs(fd - g @ v) <= 1e-7 * max(abs(fd), 1e-3)
    # single coordinates in each weight block and bias block
    for (n, k), (ow, ob) in zip(mo.SHAPES, mo.OFFSETS):
        for idx in (ow + 3, ow + (n // 2) * k + 5, ob + 1):
            e = np.zeros(mo.NPARAMS)
            e[idx] = 1.0
            lp, _ = mo.loss_and_grad(theta + 1e-4 * e, X, T, wo)
            lm, _ = mo.loss_and_grad(theta - 1e-4 * e, X, T, wo)
            fd = (lp - lm) / 2e-4
            assert abs(fd - g[idx]) <= 1e-7 * max(abs(fd), 1e-4) + 1e-11, idx


def test_padding_has_zero_gradient():
    theta, X, T, wo = _problem(3)
    _, g = mo.loss_and_grad(theta, X, T, wo)
    ow0, _ = mo.OFFSETS[0]
    W0 = g[ow0:ow0 + mo.HID * mo.PAD].reshape(mo.HID, mo.PAD)
    assert np.all(W0[:, 22:] == 0.0)
    ow3, ob3 = mo.OFFSETS[3]
    W3 = g[ow3:ow3 + mo.PAD * mo.HID].reshape(mo.PAD, mo.HID)
    assert np.all(W3[28:, :] == 0.0) and np.all(g[ob3 + 28:ob3 + 64] == 0.0)


def test_bf16_rounding():
    exact = np.array([1.0, -2.5, 0.15625, 3.0 * 2.0 ** -20, 0.0])
    np.testing.assert_array_equal(mo.to_bf16(exact), exact)
    # 1 + 2^-8 is a tie between 1 and 1 + 2^-7: rounds to the even mantissa (1)
    assert mo.to_bf16(np.array([1.0 + 2.0 ** -8]))[0] == 1.0
    # 1 + 3 * 2^-8 is a tie between 1 + 2^-7 and 1 + 2^-6: rounds to 1 + 2^-6
    assert mo.to_bf16(np.array([1.0 + 3 * 2.0 ** -8]))[0] == 1.0 + 2.0 ** -6
    x = np.random.default_rng(0).standard_normal(10000)
    r = mo.to_bf16(x)
    assert np.max(np.abs(r - x) / np.abs(x)) <= 2.0 ** -8 * (1 + 1e-12)


def test_linear_limit_is_least_squares_gradient():
    """With all hidden weights zero the output is the constant b_3: the bias
    gradient is then 2 wo (b_3 - mean T) / sum wo per output."""
    theta, X, T, wo = _problem(4)
    for (n, k), (ow, ob) in zip(mo.SHAPES, mo.OFFSETS):
        theta[ow:ow + n * k] = 0.0
    _, g = mo.loss_and_grad(theta, X, T, wo)
    _, ob3 = mo.OFFSETS[3]
    b3 = theta[ob3:ob3 + 28]
    expect = 2.0 * wo * (b3 - T.mean(0)) / wo.sum()
    np.testing.assert_allclose(g[ob3:ob3 + 28], expect, rtol=1e-12, atol=1e-15)
