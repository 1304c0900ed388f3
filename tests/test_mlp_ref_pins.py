"""Pins of the CPU reference of the surrogate network (oracle/mlp_ref.py).

The surrogate has no counterpart in the paper; these pins tie the reference to
arithmetic facts instead: bfloat16 rounding against hand-worked values and
torch's own conversion, the forward pass against a hand-computed network, the
backward pass against float64 central finite differences, and Adam against its
closed form under a constant gradient.
"""
import numpy as np
import pytest
import torch

from oracle import mlp_ref as R


def test_bf16_round_hand_values():
    one = 1.0
    ulp = 2.0 ** -7                       # bf16 keeps 7 fraction bits
    cases = {
        one: one,
        one + ulp / 2: one,               # tie -> even (fraction 0)
        one + 3 * ulp / 2: one + 2 * ulp,  # tie -> even (fraction 2)
        one + ulp / 2 + 2.0 ** -20: one + ulp,
        -(one + ulp / 2 + 2.0 ** -20): -(one + ulp),
        3.0: 3.0,
        0.0: 0.0,
    }
    for x, want in cases.items():
        assert float(R.bf16_round(np.array([x], np.float32))[0]) == want, x
    assert R.bf16_bits(np.array([1.0], np.float32))[0] == 0x3F80
    assert R.bf16_bits(np.array([-2.0], np.float32))[0] == 0xC000


def test_bf16_round_matches_torch_conversion():
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.standard_normal(100000).astype(np.float32) * 10.0 ** rng.integers(-6, 6, 100000),
                        np.array([np.inf, -np.inf, 1e-40, -1e-40], np.float32)]).astype(np.float32)
    mine = R.bf16_round(x)
    theirs = torch.from_numpy(x).to(torch.bfloat16).to(torch.float32).numpy()
    assert np.array_equal(mine.view(np.uint32), theirs.view(np.uint32))


def _tiny_params():
    # 2 inputs -> 2 -> 2 -> 2 -> 1 with small integers, values exact in bf16
    return {
        "W1": np.array([[1.0, -1.0], [0.5, 2.0]]), "b1": np.array([0.0, 1.0]),
        "W2": np.array([[1.0, 0.0], [-1.0, 1.0]]), "b2": np.array([0.5, -3.0]),
        "W3": np.array([[2.0, 1.0], [0.0, -1.0]]), "b3": np.array([0.0, 0.25]),
        "w4": np.array([1.5, -2.0]), "b4": np.array([0.125]),
    }


def test_forward_hand_computed():
    p = _tiny_params()
    x = np.array([[2.0, 4.0]])
    # z1 = [2*1 + 4*0.5 + 0, 2*(-1) + 4*2 + 1] = [4, 7]       h1 = [4, 7]
    # z2 = [4*1 + 7*(-1) + 0.5, 4*0 + 7*1 - 3] = [-2.5, 4]     h2 = [0, 4]
    # z3 = [0*2 + 4*0 + 0, 0*1 + 4*(-1) + 0.25] = [0, -3.75]   h3 = [0, 0]
    # y  = 0*1.5 + 0*(-2) + 0.125
    for bf in (False, True):
        y, _ = R.forward(p, x, bf16=bf)
        assert y[0] == 0.125
    x2 = np.array([[1.0, 0.0]])
    # z1 = [1, -1 + 1] = [1, 0]; h1 = [1, 0]
    # z2 = [1 + 0.5, 0 - 3] -> h2 = [1.5, 0]
    # z3 = [3, 1.5 + 0.25] -> h3 = [3, 1.75]
    # y = 4.5 - 3.5 + 0.125 = 1.125
    y, _ = R.forward(p, x2, bf16=False)
    assert y[0] == 1.125


def test_backward_vs_finite_differences():
    rng = np.random.default_rng(1)
    in_dim, hidden, n = 4, 8, 16
    p = R.init_params(3, in_dim, hidden)
    for k in ("b1", "b2", "b3", "b4"):
        p[k] = rng.standard_normal(p[k].shape) * 0.1
    X = rng.standard_normal((n, in_dim))
    t = rng.standard_normal(n)
    _, g = R.loss_and_grad(p, X, t, bf16=False)
    h = 1e-6
    for name, _ in R.param_shapes(in_dim, hidden):
        flat = p[name].ravel()
        for idx in range(flat.size):
            q = {k: v.copy() for k, v in p.items()}
            q[name].ravel()[idx] += h
            lp, _ = R.loss_and_grad(q, X, t, bf16=False)
            q[name].ravel()[idx] -= 2 * h
            lm, _ = R.loss_and_grad(q, X, t, bf16=False)
            fd = (lp - lm) / (2 * h)
            an = g[name].ravel()[idx]
            assert abs(fd - an) <= 1e-6 + 1e-5 * abs(fd), (name, idx, fd, an)


def test_backward_detects_dropped_relu_mask():
    # a gradient that forgets a ReLU mask differs from finite differences
    rng = np.random.default_rng(2)
    p = R.init_params(5, 4, 8)
    X = rng.standard_normal((32, 4))
    t = rng.standard_normal(32)
    _, g = R.loss_and_grad(p, X, t, bf16=False)
    _, (x, h1, h2, h3, W1, W2, W3, w4) = R.forward(p, X, bf16=False)
    y = h3 @ w4 + p["b4"][0]
    dy = 2 * (y - t) / len(t)
    dz3_unmasked = np.outer(dy, w4)
    assert not np.allclose(h2.T @ dz3_unmasked, g["W3"])


def test_adam_closed_form_constant_gradient():
    # with a constant gradient g, the bias-corrected moments are g and g^2, so
    # every step moves each weight by lr * g / (|g| + eps)
    p = {"w": np.array([0.5, -1.0, 2.0])}
    g = {"w": np.array([0.25, -4.0, 1e-3])}
    m = {"w": np.zeros(3)}
    v = {"w": np.zeros(3)}
    lr = 1e-2
    cur = p
    for step in range(1, 6):
        cur = R.adam(cur, g, m, v, step, lr)
        want = p["w"] - step * lr * g["w"] / (np.abs(g["w"]) + 1e-8)
        assert np.allclose(cur["w"], want, rtol=0, atol=1e-6)


def test_flatten_roundtrip_and_count():
    p = R.init_params(0)
    flat = R.flatten(p)
    assert flat.size == 32 * 256 + 256 + 2 * (256 * 256 + 256) + 256 + 1
    q = R.unflatten(flat)
    for k in p:
        assert np.array_equal(p[k], q[k])


def test_init_is_he_uniform():
    p = R.init_params(7)
    for name, fan in (("W1", 32), ("W2", 256), ("W3", 256), ("w4", 256)):
        lim = np.sqrt(6.0 / fan)
        assert np.abs(p[name]).max() <= lim
        assert abs(np.var(p[name]) - lim ** 2 / 3) < 0.1 * lim ** 2 / 3
