"""The adjoint entry point without a workspace argument
(qvm_adjoint_expect_grad_static): its results against the entry point with
a caller workspace, on two calls in a row (the second smaller), and its
size limit."""
import math

import numpy as np
import pytest

import oracle
from workloads import hardware_efficient_ansatz, random_pauli_sum

pytestmark = pytest.mark.gpu

adj = pytest.importorskip("paper_2212_14201_amd.adjoint")


@pytest.fixture(autouse=True)
def _gpu(require_gpu):
    pass


def _case(n, layers, terms, batch, seed, dtype):
    gates, P = hardware_efficient_ansatz(n, layers)
    xs, zs, cs, _ = random_pauli_sum(n, terms, seed + 1)
    theta = np.random.default_rng(seed).uniform(0, 2 * math.pi, (batch, P))
    return gates, P, xs, zs, cs, theta


@pytest.mark.parametrize("dtype", ["c64", "c128"])
def test_static_workspace_matches_caller_workspace(dtype):
    """Two calls in a row on the static workspace (20 qubits, batch 64 at
    the full 944-gate ansatz, then 12 qubits, batch 5, 4 layers), each
    bit-identical to the caller-workspace entry point (same kernels, same
    reduction order) and, for sampled elements, within the stated bound
    of the oracle's adjoint."""
    for (n, layers, terms, batch, seed) in ((20, 16, 40, 64, 2001), (12, 4, 10, 5, 77)):
        gates, P, xs, zs, cs, theta = _case(n, layers, terms, batch, seed, dtype)
        print(f"static workspace: {dtype} n={n} batch={batch} gates={len(gates)}", flush=True)
        ref = adj.AdjointProblem(n, gates, P, xs, zs, cs, batch, dtype)
        f_ref, g_ref = ref.run(theta)
        del ref
        st = adj.AdjointProblem(n, gates, P, xs, zs, cs, batch, dtype, static_workspace=True)
        assert st.work is None
        f, g = st.run(theta)
        assert np.array_equal(f, f_ref) and np.array_equal(g, g_ref)
        fo, go = oracle.adjoint(n, gates, theta[batch - 1], xs, zs, cs)
        if dtype == "c128":
            tol = 1e-12 * (1 + float(np.sum(np.abs(cs))))
        else:
            tol = 1e-3 * max(abs(fo), float(np.max(np.abs(go))))
        assert abs(f[batch - 1] - fo) <= tol
        assert float(np.max(np.abs(g[batch - 1] - go))) <= tol
        del st


def test_static_workspace_rejects_oversized_problem():
    """A problem whose workspace exceeds the static array fails with
    QVM_ENOMEM before anything runs; a later call still works."""
    from paper_2212_14201_amd.qvm import QvmError
    gates, P, xs, zs, cs, theta = _case(4, 200, 6, 300, 5, "c64")   # 2 x 2,200 gates x 300 x 64 B > 64 MiB
    big = adj.AdjointProblem(4, gates, P, xs, zs, cs, 300, "c64", static_workspace=True)
    with pytest.raises(QvmError) as ei:
        big.run(theta)
    assert ei.value.status == -3 and "static" in str(ei.value)
    gates, P, xs, zs, cs, theta = _case(5, 2, 4, 3, 6, "c128")
    f, g = adj.AdjointProblem(5, gates, P, xs, zs, cs, 3, "c128", static_workspace=True).run(theta)
    f_ref, g_ref = adj.AdjointProblem(5, gates, P, xs, zs, cs, 3, "c128").run(theta)
    assert np.array_equal(f, f_ref) and np.array_equal(g, g_ref)
