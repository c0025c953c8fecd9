"""GPU parity of the cost-model MLP kernels (forward, backward, Adam)
against the FP64 NumPy oracle."""
import numpy as np
import pytest

from oracle import mlp as ref
from workloads import mlp_init

pytestmark = pytest.mark.gpu

cm = pytest.importorskip("paper_2212_14201_amd.costmodel")


@pytest.fixture(autouse=True)
def _gpu(require_gpu):
    pass


def setup(B=300, d=20, H=128, seed=0):
    import torch
    rng = np.random.default_rng(seed)
    params = mlp_init(d, H, seed + 10)
    for p in params[1::2]:
        p += 0.05 * rng.standard_normal(p.shape)
    X = rng.standard_normal((B, d))
    t = rng.standard_normal(B)
    net = cm.CostMLP(d, H, init=params)
    Xd = torch.tensor(X, dtype=torch.float32, device="cuda")
    td = torch.tensor(t, dtype=torch.float32, device="cuda")
    # the oracle sees the same FP32-rounded weights and inputs
    p32 = [np.asarray(p, dtype=np.float32).astype(np.float64) for p in params]
    return net, Xd, td, p32, X.astype(np.float32).astype(np.float64), t.astype(np.float32).astype(np.float64)


@pytest.mark.parametrize("B", [1, 37, 300])
def test_forward_backward_match_oracle(B):
    net, Xd, td, p, X, t = setup(B=B)
    y, act = net.forward(Xd)
    y_ref, _ = ref.forward(p, X)
    scale = 1 + np.max(np.abs(y_ref))
    assert np.max(np.abs(y.cpu().numpy() - y_ref)) <= 2e-5 * scale
    loss = net.backward(Xd, td, act, y)
    L_ref, g_ref = ref.backward(p, X, t)
    assert abs(float(loss.cpu()) - L_ref) <= 1e-5 * (1 + L_ref)
    for g, gr in zip(net.get_grads(), g_ref):
        assert np.max(np.abs(g - gr)) <= 1e-4 * (1e-3 + np.max(np.abs(gr))), (np.max(np.abs(g - gr)), np.max(np.abs(gr)))


def test_adam_matches_oracle():
    net, Xd, td, p, X, t = setup(B=64)
    y, act = net.forward(Xd)
    net.backward(Xd, td, act, y)
    g = net.get_grads()
    p0 = net.get_params()
    m = [np.zeros_like(a) for a in p0]
    v = [np.zeros_like(a) for a in p0]
    for step in (1, 2, 3):
        net.adam(1e-3)
        ref.adam_step(p0, g, m, v, step, 1e-3)
    for a, b in zip(net.get_params(), p0):
        assert np.max(np.abs(a - b)) <= 1e-6 * (1 + np.max(np.abs(b)))


def test_training_reduces_loss():
    import torch
    rng = np.random.default_rng(4)
    d, B = 12, 512
    X = rng.standard_normal((B, d))
    w = rng.standard_normal(d)
    t = np.sin(X @ w) + 0.5 * X[:, 0] ** 2
    net = cm.CostMLP(d, 128, init=mlp_init(d, 128, 5))
    Xd = torch.tensor(X, dtype=torch.float32, device="cuda")
    td = torch.tensor(t, dtype=torch.float32, device="cuda")
    first = float(net.train_step(Xd, td, 3e-3).cpu())
    for _ in range(400):
        last = net.train_step(Xd, td, 3e-3)
    assert float(last.cpu()) < 0.1 * first
