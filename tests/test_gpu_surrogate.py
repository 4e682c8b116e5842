"""Surrogate MLP kernels (BF16 operands on the matrix cores, FP32 accumulation) against the
FP64 reference network, which rounds to BF16 at the same points and accumulates exactly.

Tolerances: the GPU and the reference differ only by FP32 accumulation order and by the
rare BF16 rounding that flips because an FP32 sum sits on a rounding boundary (about one
element in 1e4).  A flip moves one product term by one BF16 ulp (2^-8 relative), so an
output differs from the reference by far less than 1e-3 of the sum of the absolute values
of its terms; a transposed operand, a wrong index or a missing term fails by O(1)."""
import numpy as np
import pytest

from oracle import mlp

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    from paper_2210_08024_amd import ism
    torch.cuda.set_device(0)
    ism.init(0)
    return torch


def _abs_scale_out(theta, Xs):
    """Sum over the output layer's terms of |W4| |h3| + |b4| (the scale of each output)."""
    _, cache = mlp.forward(theta, Xs)
    W4, b4 = mlp.unflatten(np.asarray(theta, dtype=np.float64))[-1]
    h3 = cache[-1][0]
    return np.abs(h3) @ np.abs(mlp.bf16(W4)).T + np.abs(b4)


def _inputs(B, seed):
    rng = np.random.default_rng(seed)
    X = rng.normal(0.0, 1.0, (B, 10)).astype(np.float32)
    X[:, 6:8] = rng.uniform(0, 1, (B, 2))  # abundance-like columns
    return X


def _make(torch, seed, theta=None, m=None, v=None, step=0, norm=None):
    from paper_2210_08024_amd import ism
    s = ism.Surrogate(seed=seed)
    if theta is not None:
        norm = norm or {}
        s.set_params(ism.Surrogate.state(theta, m, v, step, **norm))
    return s


@pytest.mark.parametrize("B", [1, 17, 1000, 4133])
def test_forward_matches_reference(torch_dev, B):
    torch = torch_dev
    theta = mlp.init_params(11)
    X = _inputs(B, B)
    s = _make(torch, 0, theta)
    Y = s.forward(torch.from_numpy(X).cuda()).cpu().numpy().astype(np.float64)
    Yr, _ = mlp.forward(theta, X)
    scale = _abs_scale_out(theta, X)
    err = np.abs(Y - Yr) / scale
    assert err.max() < 1e-3, err.max()
    assert np.median(err) < 1e-5


def test_forward_standardisation(torch_dev):
    """Inputs standardised inside the library and outputs mapped back."""
    torch = torch_dev
    rng = np.random.default_rng(5)
    B = 777
    mu_x = rng.normal(0, 3, 10)
    sd_x = rng.uniform(0.5, 4, 10)
    mu_y = rng.normal(0, 2, 3)
    sd_y = rng.uniform(0.2, 3, 3)
    theta = mlp.init_params(3)
    X = (mu_x + sd_x * rng.normal(0, 1, (B, 10))).astype(np.float32)
    s = _make(torch, 0, theta, norm=dict(mu_x=mu_x, sd_x=sd_x, mu_y=mu_y, sd_y=sd_y))
    Y = s.forward(torch.from_numpy(X).cuda()).cpu().numpy().astype(np.float64)
    mux32, isd32 = mu_x.astype(np.float32), (1.0 / sd_x).astype(np.float32)
    Xs = (X - mux32) * isd32                     # the library standardises in FP32
    Ys, _ = mlp.forward(theta, Xs)
    Yr = Ys * sd_y.astype(np.float32) + mu_y.astype(np.float32)
    scale = _abs_scale_out(theta, Xs) * sd_y
    assert (np.abs(Y - Yr) / scale).max() < 1e-3


def test_forward_empty_batch(torch_dev):
    torch = torch_dev
    s = _make(torch, 0)
    Y = s.forward(torch.empty((0, 10), dtype=torch.float32, device="cuda"))
    assert Y.shape == (0, 3)


def _oracle_grad_for_dY(theta, X, dY):
    """Reference gradient of sum(dY * y): the MSE gradient with targets y - dY (3B)/2."""
    Yh, _ = mlp.forward(theta, X)
    B = X.shape[0]
    _, g = mlp.loss_and_grad(theta, X, Yh - dY * (3 * B) / 2.0)
    return g


def _check_grad(g, gr, label):
    for k, (W, b) in enumerate(zip(mlp.unflatten(g), mlp.unflatten(gr))):
        for name, a, r in (("W", W[0], b[0]), ("b", W[1], b[1])):
            d = np.abs(a - r)
            nr = np.linalg.norm(r)
            assert np.linalg.norm(d) <= 1e-3 * nr + 1e-12, f"{label} layer {k + 1} {name}: {np.linalg.norm(d) / nr:.2e}"
            assert d.max() <= 2e-3 * np.abs(r).max() + 1e-12, f"{label} layer {k + 1} {name} max"


@pytest.mark.parametrize("B", [1, 300, 5000])
def test_backward_matches_reference(torch_dev, B):
    torch = torch_dev
    theta = mlp.init_params(21)
    X = _inputs(B, 100 + B)
    dY = np.random.default_rng(B).normal(0, 1.0 / B, (B, 3)).astype(np.float32)
    s = _make(torch, 0, theta)
    g = s.backward(torch.from_numpy(X).cuda(), torch.from_numpy(dY).cuda()).cpu().numpy().astype(np.float64)
    gr = _oracle_grad_for_dY(theta, X, dY.astype(np.float64))
    _check_grad(g, gr, f"B={B}")


def test_backward_is_deterministic(torch_dev):
    torch = torch_dev
    theta = mlp.init_params(4)
    X = torch.from_numpy(_inputs(3000, 9)).cuda()
    dY = torch.randn(3000, 3, device="cuda", dtype=torch.float32, generator=torch.Generator("cuda").manual_seed(1))
    s = _make(torch, 0, theta)
    g1 = s.backward(X, dY).clone()
    g2 = s.backward(X, dY).clone()
    assert torch.equal(g1, g2)


def test_train_step_loss_and_adam(torch_dev):
    torch = torch_dev
    rng = np.random.default_rng(8)
    B = 2500
    theta = mlp.init_params(31)
    X = _inputs(B, 77)
    Yt = rng.normal(0, 1, (B, 3)).astype(np.float32)
    # an Adam history so that the step is not just lr * sign(g)
    _, g0 = mlp.loss_and_grad(theta, X, Yt)
    m0 = (g0 * rng.uniform(0.5, 1.5, g0.size)).astype(np.float32)
    v0 = (g0 ** 2 * rng.uniform(1.0, 2.0, g0.size) + 1e-12).astype(np.float32)
    s = _make(torch, 0, theta, m0, v0, step=9)
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    lr = 1e-3
    s.train_step(torch.from_numpy(X).cuda(), torch.from_numpy(Yt).cuda(), lr, loss)
    st = s.get_params().astype(np.float64)
    N = mlp.n_params()
    th1, m1, v1, step = st[:N], st[N:2 * N], st[2 * N:3 * N], st[3 * N]
    L, g = mlp.loss_and_grad(theta, X, Yt)
    th_r, m_r, v_r = mlp.adam(theta.astype(np.float64), m0.astype(np.float64), v0.astype(np.float64), g, 10, lr)
    assert step == 10
    assert abs(loss.item() - L) <= 1e-4 * L
    gs = np.abs(g).max()
    assert np.abs(m1 - m_r).max() <= 2e-4 * gs
    assert np.abs(v1 - v_r).max() <= 4e-4 * gs * gs
    assert np.all(np.abs(th1 - th_r) <= 3e-7 * np.abs(th_r) + 2e-3 * lr)


def test_checkpoint_round_trip(torch_dev):
    torch = torch_dev
    from paper_2210_08024_amd import ism
    X = torch.from_numpy(_inputs(600, 3)).cuda()
    Yt = torch.randn(600, 3, device="cuda", generator=torch.Generator("cuda").manual_seed(2))
    a = ism.Surrogate(seed=123)
    for _ in range(3):
        a.train_step(X, Yt, 1e-3)
    st = a.get_params()
    b = ism.Surrogate(seed=999)
    b.set_params(st)
    assert np.array_equal(b.get_params(), st)
    assert torch.equal(a.forward(X), b.forward(X))
    a.train_step(X, Yt, 1e-3)
    b.train_step(X, Yt, 1e-3)
    assert np.array_equal(a.get_params(), b.get_params())


def test_training_fits_a_smooth_map(torch_dev):
    """End to end: the training kernels drive the loss down on a smooth 10 -> 3 map."""
    torch = torch_dev
    from paper_2210_08024_amd import ism
    g = torch.Generator("cuda").manual_seed(0)
    B = 8192
    X = torch.randn(B, 10, device="cuda", generator=g)
    A = torch.randn(10, 3, device="cuda", generator=g) / 3
    Y = torch.tanh(X @ A) + 0.1 * (X[:, :3] ** 2)
    s = ism.Surrogate(seed=1)
    loss = torch.zeros(1, device="cuda")
    s.train_step(X, Y, 1e-3, loss)
    l0 = loss.item()
    for _ in range(300):
        s.train_step(X, Y, 2e-3, loss)
    assert loss.item() < 0.05 * l0, (l0, loss.item())
