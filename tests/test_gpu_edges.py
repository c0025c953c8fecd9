"""Edge cases on the GPU: empty gate lists on both paths, the smallest
states (1 and 2 qubits on the plain path, 3 on the fused path), readouts and
a Kraus branching on one qubit, and zero samples; against the FP64 oracle."""
import numpy as np
import pytest

import oracle
from oracle import noise as onoise
from tests.util import C128_TOL
from workloads import Gate, random_mixed_circuit

pytestmark = pytest.mark.gpu

qvm = pytest.importorskip("paper_2212_14201_amd.qvm")


@pytest.fixture(autouse=True)
def _gpu(require_gpu):
    pass


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_empty_gate_lists(dtype):
    n = 10
    sv = qvm.StateVector(n, dtype, init=37)
    sv.run([])
    plan = qvm.Plan([], n, dtype, k_max=3, tile_qubits=8)
    assert plan.stats()["passes"] == 0
    plan.run(sv)
    a = sv.amplitudes()
    want = np.zeros(1 << n, complex)
    want[37] = 1
    assert np.array_equal(a, want)
    assert sv.sample(np.zeros(0)).size == 0


@pytest.mark.parametrize("n", [1, 2])
def test_smallest_states_plain_path(n):
    gates = random_mixed_circuit(n, 25, 60 + n, kmax=n, max_ctrl=0 if n == 1 else 1)
    sv = qvm.StateVector(n, "c128", init=n - 1)
    sv.run(gates)
    want = oracle.simulate(n, gates, init=n - 1)
    assert np.max(np.abs(sv.amplitudes() - want)) <= C128_TOL
    p = sv.probabilities()
    assert np.max(np.abs(p - np.abs(want) ** 2)) < 1e-13
    z = sv.expect_z_all()
    assert abs(z[0] - oracle.expect_z_all(want)[0]) < 1e-13
    s = sv.sample([0.0, 0.999999])
    assert all(0 <= int(v) < (1 << n) for v in s)
    with pytest.raises(qvm.QvmError):
        qvm.Plan(gates, n, "c128", k_max=n, tile_qubits=0)     # fused plans need n >= 3


def test_smallest_fused_state():
    n = 3
    gates = random_mixed_circuit(n, 30, 63, kmax=3, max_ctrl=0)
    for dtype, tol in (("c128", C128_TOL), ("c64", 5e-6)):
        for k_max, tile in ((3, 3), (3, 0), (2, 0)):
            if k_max < 3 and any(len(g.qubits()) > k_max for g in gates):
                continue
            sv = qvm.StateVector(n, dtype, init=6)
            qvm.Plan(gates, n, dtype, k_max=k_max, tile_qubits=tile).run(sv)
            err = np.max(np.abs(sv.amplitudes() - oracle.simulate(n, gates, init=6)))
            assert err <= tol, (dtype, k_max, tile, err)


def test_one_qubit_kraus_branching():
    sv = qvm.StateVector(1, "c128")
    sv.apply(Gate("ry", (0,), (), (1.1,)))
    psi = sv.amplitudes()
    ops = onoise.kraus("damping", p=0.4)
    for u in (0.05, 0.95):
        sv2 = qvm.StateVector(1, "c128")
        sv2.apply(Gate("ry", (0,), (), (1.1,)))
        j, probs = sv2.apply_kraus(0, ops, u)
        want, jj, _ = onoise.trajectory_step(psi, 1, 0, ops, u)
        assert j == jj
        assert np.max(np.abs(sv2.amplitudes() - want)) <= C128_TOL
