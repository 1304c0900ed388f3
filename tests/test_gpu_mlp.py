"""GPU parity of the surrogate kernels against the CPU reference (oracle/mlp_ref.py).

Tolerances: the GPU sums bf16 products in fp32 on the MFMA units in an order of
its own, the reference in float64; a hidden activation whose value lies next to
a bf16 rounding boundary can then round one bf16 step (2^-8 relative) apart,
which the next layers carry.  Forward: max |y_gpu - y_ref| <= 1e-2 * max |y_ref|.
Gradients: cosine >= 0.999 and relative norm difference <= 2e-2 per tensor.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import mlp_ref as R  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def H():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1602_05510_amd import hesp
    return hesp


def _x_bits(X):
    return torch.from_numpy(R.bf16_bits(X.astype(np.float32)).view(np.int16)).cuda()


def _rand_x(rng, n):
    # depth-like 0/1/2 features in the first 20 columns, rate-like values in the next 8, zero padding
    X = np.zeros((n, 32), np.float32)
    X[:, :20] = rng.integers(0, 3, (n, 20))
    X[:, 20:28] = rng.normal(0.0, 1.5, (n, 8))
    return X


def _params(seed):
    p = R.init_params(seed)
    rng = np.random.default_rng(seed + 100)
    for k in ("b1", "b2", "b3", "b4"):
        p[k] = (rng.standard_normal(p[k].shape) * 0.05).astype(np.float32).astype(np.float64)
    return p


def test_param_count(H):
    assert H.MLP.param_count() == R.flatten(R.init_params(0)).size


def test_set_get_roundtrip(H):
    m = H.MLP(1)
    p = R.flatten(_params(2)).astype(np.float32)
    m.set_params(p)
    assert np.array_equal(m.get_params(), p)


def test_create_is_he_uniform(H):
    m = H.MLP(123)
    q = R.unflatten(m.get_params())
    for name, fan in (("W1", 32), ("W2", 256), ("W3", 256), ("w4", 256)):
        lim = np.sqrt(6.0 / fan)
        assert np.abs(q[name]).max() <= lim + 1e-7
        assert abs(np.var(q[name]) - lim ** 2 / 3) < 0.1 * lim ** 2 / 3
    for name in ("b1", "b2", "b3", "b4"):
        assert not q[name].any()
    m2 = H.MLP(123)
    assert np.array_equal(m2.get_params(), m.get_params())


def test_features_bits(H):
    rng = np.random.default_rng(0)
    n, n_top = 777, 20
    dep = rng.integers(0, 4, (n, n_top)).astype(np.uint8)
    rate = rng.normal(0, 2, 8).astype(np.float32)
    x = torch.empty((n, 32), dtype=torch.int16, device="cuda")
    H.mlp_features(torch.from_numpy(dep).cuda(), n, n_top, torch.from_numpy(rate).cuda(), x)
    want = np.zeros((n, 32), np.float32)
    want[:, :n_top] = dep
    want[:, n_top:n_top + 8] = rate
    assert np.array_equal(x.cpu().numpy().view(np.uint16), R.bf16_bits(want))


def test_features_rejects_too_many(H):
    x = torch.empty((4, 32), dtype=torch.int16, device="cuda")
    dep = torch.zeros(4 * 30, dtype=torch.uint8, device="cuda")
    rate = torch.zeros(8, dtype=torch.float32, device="cuda")
    with pytest.raises(H.HespError):
        H.mlp_features(dep, 4, 30, rate, x)


def test_targets(H):
    ms = np.array([1, 1000, 123456789, 10 ** 12], np.int64)
    t = torch.empty(4, dtype=torch.float32, device="cuda")
    H.mlp_targets(torch.from_numpy(ms).cuda(), 15.0, 2.0, t)
    want = (np.log(ms.astype(np.float64)) - 15.0) / 2.0
    assert np.allclose(t.cpu().numpy(), want, rtol=1e-6, atol=1e-6)


@pytest.mark.parametrize("n", [1, 63, 64, 1000, 4097])
def test_forward_parity(H, n):
    rng = np.random.default_rng(n)
    p = _params(n)
    X = _x_bits_src = _rand_x(rng, n)
    m = H.MLP(0)
    m.set_params(R.flatten(p).astype(np.float32))
    y = torch.empty(n, dtype=torch.float32, device="cuda")
    m.forward(_x_bits(X), y)
    got = y.cpu().numpy().astype(np.float64)
    want, _ = R.forward(p, X, bf16=True)
    err = np.abs(got - want).max()
    assert err <= 1e-2 * max(np.abs(want).max(), 1e-3), (err, np.abs(want).max())


def test_forward_large_sampled(H):
    # a 2^20-row forward pass (the per-platform scoring size), checked on 2048 sampled rows
    n = 1 << 20
    rng = np.random.default_rng(9)
    p = _params(9)
    X = _rand_x(rng, n)
    m = H.MLP(0)
    m.set_params(R.flatten(p).astype(np.float32))
    y = torch.empty(n, dtype=torch.float32, device="cuda")
    m.forward(_x_bits(X), y)
    idx = np.sort(rng.choice(n, 2048, replace=False))
    idx[-1] = n - 1
    got = y.cpu().numpy()[idx].astype(np.float64)
    want, _ = R.forward(p, X[idx], bf16=True)
    assert np.abs(got - want).max() <= 1e-2 * np.abs(want).max()


def _cos(a, b):
    return float(np.dot(a, b) / (np.linalg.norm(a) * np.linalg.norm(b) + 1e-30))


@pytest.mark.parametrize("batch", [512, 2048])
def test_grad_parity(H, batch):
    rng = np.random.default_rng(batch)
    p = _params(batch + 1)
    X = _rand_x(rng, batch)
    t = rng.normal(0, 1, batch)
    m = H.MLP(0)
    m.set_params(R.flatten(p).astype(np.float32))
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    m.grad(_x_bits(X), torch.from_numpy(t.astype(np.float32)).cuda(), batch, loss)
    g = R.unflatten(m.get_grads())
    want_loss, want = R.loss_and_grad(p, X, t.astype(np.float32).astype(np.float64), bf16=True)
    assert abs(float(loss.item()) - want_loss) <= 1e-2 * want_loss
    for k in want:
        a, b = g[k].ravel(), want[k].ravel()
        if np.linalg.norm(b) == 0:
            assert np.linalg.norm(a) == 0, k
            continue
        assert _cos(a, b) >= 0.999, (k, _cos(a, b))
        assert np.linalg.norm(a - b) <= 2e-2 * np.linalg.norm(b), (k, np.linalg.norm(a - b) / np.linalg.norm(b))
        # element by element: both sides round the same operands to bf16, so they
        # differ by fp32 accumulation order and the rare bf16 rounding it flips (one
        # bf16 step, 2^-8 relative, of one term of a sum over the batch); a wrong
        # row or column of a weight gradient is far outside this bound
        assert np.abs(a - b).max() <= 1e-2 * np.abs(b).max(), (k, np.abs(a - b).max() / np.abs(b).max())


def test_grad_rejects_bad_batch(H):
    m = H.MLP(0)
    x = torch.zeros((500, 32), dtype=torch.int16, device="cuda")
    t = torch.zeros(500, dtype=torch.float32, device="cuda")
    with pytest.raises(H.HespError):
        m.grad(x, t, 500)


def test_adam_step_parity(H):
    rng = np.random.default_rng(5)
    p = _params(5)
    X = _rand_x(rng, 1024)
    t = rng.normal(0, 1, 1024).astype(np.float32)
    m = H.MLP(0)
    m.set_params(R.flatten(p).astype(np.float32))
    xd, td = _x_bits(X), torch.from_numpy(t).cuda()
    mom = {k: np.zeros_like(v) for k, v in p.items()}
    vel = {k: np.zeros_like(v) for k, v in p.items()}
    cur = p
    lr = 1e-3
    for step in (1, 2, 3):
        m.grad(xd, td, 1024)
        g = R.unflatten(m.get_grads())
        m.adam(lr)
        cur = R.adam(cur, g, mom, vel, step, lr)
        got = R.unflatten(m.get_params())
        for k in cur:
            assert np.abs(got[k] - cur[k]).max() <= 1e-6 + 1e-5 * lr, (step, k)
        # continue from the GPU's own weights so both sides see the same gradients
        cur = {k: v.copy() for k, v in got.items()}


def test_train_reduces_loss(H):
    # a target that is a smooth function of the features is learnt
    rng = np.random.default_rng(11)
    n = 16384
    X = _rand_x(rng, n)
    t = (np.tanh(X[:, :20].sum(1) / 10.0) + 0.3 * X[:, 20]).astype(np.float32)
    t = (t - t.mean()) / t.std()
    m = H.MLP(3)
    xd, td = _x_bits(X), torch.from_numpy(t).cuda()
    steps = 400
    loss = torch.zeros(steps, dtype=torch.float32, device="cuda")
    m.train(xd, td, 1024, steps, 1e-3, seed=7, loss=loss)
    l = loss.cpu().numpy()
    assert np.isfinite(l).all()
    assert l[-20:].mean() < 0.1 * l[:5].mean(), (l[:5], l[-20:])
    y = torch.empty(n, dtype=torch.float32, device="cuda")
    m.forward(xd, y)
    mse = float(((y.cpu().numpy() - t) ** 2).mean())
    assert mse < 0.1
