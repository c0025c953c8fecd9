"""GPU parity of the batched adjoint gradient against the FP64 oracle's
adjoint, central finite differences and torch autograd."""
import math

import numpy as np
import pytest

import oracle
from tests.util import c64_bound
from workloads import Gate, hardware_efficient_ansatz, random_pauli_sum

pytestmark = pytest.mark.gpu

adj = pytest.importorskip("paper_2212_14201_amd.adjoint")


@pytest.fixture(autouse=True)
def _gpu(require_gpu):
    pass


def problem(n, layers, terms, seed):
    gates, P = hardware_efficient_ansatz(n, layers)
    xs, zs, cs, _ = random_pauli_sum(n, terms, seed + 1)
    return gates, P, xs, zs, cs


def c64_tol(gates, cs):
    """The stated complex64 gradient bound 2 tau sum|c|: each gate is one
    pass of k = 1 in the forward sweep and two (psi and lambda) in the
    reverse sweep, the Pauli sum one pass per term; lambda carries
    sum |c|."""
    tau = c64_bound([1] * (3 * len(gates)) + [2] * len(cs))
    return 2 * tau * float(np.sum(np.abs(cs)))


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_adjoint_matches_oracle(dtype):
    n, B = 6, 5
    gates, P, xs, zs, cs = problem(n, 3, 8, 11)
    theta = np.random.default_rng(3).uniform(0, 2 * math.pi, (B, P))
    prob = adj.AdjointProblem(n, gates, P, xs, zs, cs, B, dtype)
    f, g = prob.run(theta)
    tol = 1e-12 * (1 + np.sum(np.abs(cs))) if dtype == "c128" else c64_tol(gates, cs)
    for b in range(B):
        fo, go = oracle.adjoint(n, gates, theta[b], xs, zs, cs)
        assert abs(f[b] - fo) <= tol
        assert np.max(np.abs(g[b] - go)) <= tol, (b, np.max(np.abs(g[b] - go)), tol)


def test_adjoint_controlled_and_fixed_gates():
    n, B = 5, 3
    gates = [Gate("h", (0,)), Gate("h", (3,)), Gate("ry", (2,), (0,), (0.0,), pidx=0),
             Gate("x", (4,), (2,)), Gate("rx", (1,), (2, 3), (0.0,), pidx=1),
             Gate("rz", (4,), (), (0.0,), pidx=2), Gate("u3", (1,), (4,), (0.3, 1.1, -0.4)),
             Gate("ry", (3,), (), (0.0,), pidx=0)]          # parameter shared by two gates
    xs, zs, cs, _ = random_pauli_sum(n, 6, 7, wmin=1, wmax=3)
    theta = np.random.default_rng(5).uniform(-3, 3, (B, 3))
    prob = adj.AdjointProblem(n, gates, 3, xs, zs, cs, B, "c128")
    f, g = prob.run(theta)
    for b in range(B):
        fo, go = oracle.adjoint(n, gates, theta[b], xs, zs, cs)
        assert abs(f[b] - fo) < 1e-12 * (1 + np.sum(np.abs(cs)))
        assert np.max(np.abs(g[b] - go)) < 1e-12 * (1 + np.sum(np.abs(cs)))


def test_adjoint_matches_central_differences():
    """Along one coordinate f = A cos t + B sin t + C, so the central
    difference with h = 1e-3 equals f'(t) sin(h)/h; checked on the GPU's own
    complex128 expectation values."""
    n, B = 8, 1
    gates, P, xs, zs, cs = problem(n, 4, 12, 21)
    theta = np.random.default_rng(9).uniform(0, 2 * math.pi, (1, P))
    prob = adj.AdjointProblem(n, gates, P, xs, zs, cs, B, "c128")
    _, g = prob.run(theta)
    h = 1e-3
    for p in range(0, P, 5):
        tp, tm = theta.copy(), theta.copy()
        tp[0, p] += h
        tm[0, p] -= h
        fp, _ = prob.run(tp, want_grad=False)
        fm, _ = prob.run(tm, want_grad=False)
        fd = (fp[0] - fm[0]) / (2 * h) / (math.sin(h) / h)
        assert abs(fd - g[0, p]) <= 1e-9 * np.sum(np.abs(cs)), p


def test_autograd_function():
    import torch
    n, B = 6, 4
    gates, P, xs, zs, cs = problem(n, 2, 6, 31)
    prob = adj.AdjointProblem(n, gates, P, xs, zs, cs, B, "c128")
    theta = torch.tensor(np.random.default_rng(2).uniform(0, 6, (B, P)), dtype=torch.float64,
                         requires_grad=True)
    f = adj.adjoint_expectation(theta, prob)
    w = torch.linspace(0.5, 2.0, B, dtype=torch.float64)
    (gt,) = torch.autograd.grad((w * f).sum(), theta)
    _, g = prob.run(theta.detach().numpy())
    assert np.allclose(gt.numpy(), w.numpy()[:, None] * g, atol=1e-14)


def _batch20(dtype):
    n, B = 20, 64
    gates, P, xs, zs, cs = problem(n, 16, 40, 2001)
    assert P == 640 and len(gates) == 944
    theta = np.random.default_rng(2002).uniform(0, 2 * math.pi, (B, P))
    prob = adj.AdjointProblem(n, gates, P, xs, zs, cs, B, dtype)
    f, g = prob.run(theta)
    return n, gates, theta, xs, zs, cs, f, g


def test_adjoint_20_qubits_batch_64_sampled_against_oracle():
    """20 qubits, complex64, 16 layers (640 parameters), 40 Pauli terms of
    weight 2-4, a batch of 64: four batch elements checked in full against
    the oracle's adjoint, within the stated bound 2 tau sum|c| and within
    1e-3 of the largest oracle gradient and of |f| (the stated bound alone
    is larger than many gradients at this size; the relative bar is what
    a zero or a wrong-sign output fails)."""
    n, gates, theta, xs, zs, cs, f, g = _batch20("c64")
    tol = c64_tol(gates, cs)
    for b in (0, 17, 40, 63):
        fo, go = oracle.adjoint(n, gates, theta[b], xs, zs, cs)
        gmax = float(np.max(np.abs(go)))
        err = float(np.max(np.abs(g[b] - go)))
        ferr = abs(f[b] - fo)
        print(f"b={b} f {fo:.4e} err {ferr:.2e}; max|g| {gmax:.3e} grad err {err:.2e}; "
              f"stated bound {tol:.2e}", flush=True)
        assert ferr <= min(tol, 1e-3 * abs(fo))
        assert err <= min(tol, 1e-3 * gmax)


def test_adjoint_20_qubits_batch_64_complex128():
    """The same 20-qubit batch in complex128: four elements (other than the
    complex64 test's) against the oracle's adjoint at 1e-12 (1 + sum|c|),
    every element's value and gradient finite."""
    n, gates, theta, xs, zs, cs, f, g = _batch20("c128")
    tol = 1e-12 * (1 + float(np.sum(np.abs(cs))))
    assert np.all(np.isfinite(f)) and np.all(np.isfinite(g))
    for b in (3, 29, 51, 62):
        fo, go = oracle.adjoint(n, gates, theta[b], xs, zs, cs)
        err = float(np.max(np.abs(g[b] - go)))
        print(f"b={b} f err {abs(f[b] - fo):.2e} grad err {err:.2e} tol {tol:.2e}", flush=True)
        assert abs(f[b] - fo) <= tol
        assert err <= tol
