"""GPU parity of the paper's own benchmark shapes against the FP64 oracle:
the random circuit of "Compared with existing libs" (a rotation layer of RX,
RY, RZ on every qubit, then CNOT with target i and control (i+1) mod n,
repeated from |0>) through the plain path in both dtypes and through the
fused path with the greedy fallback and with the shipped learned planner;
and every gate kind of the per-gate sweep ("Performance of basic gates":
RX, RY, CNOT, Toffoli, random 1-, 2- and 3-qubit unitaries) once each."""
import numpy as np
import pytest

import oracle
from tests.util import C128_TOL, U32, c64_bound, gate_ks
from workloads import rotation_cnot_circuit

pytestmark = pytest.mark.gpu

qvm = pytest.importorskip("paper_2212_14201_amd.qvm")


@pytest.fixture(autouse=True)
def _gpu(require_gpu):
    pass


def plan_tau(plan):
    st = plan.stats()
    s = sum((1 << plan.block(b)["k"]) + 4 for b in range(st["blocks"])) + 5 * st["diag_ops"]
    return 10.0 * np.sqrt(s) * U32


def rel2(got, want):
    return float(np.linalg.norm(got - want) / np.linalg.norm(want))


@pytest.mark.parametrize("n", [16, 20])
def test_rotation_cnot_circuit(n):
    layers = 6
    gates = rotation_cnot_circuit(n, layers, 8200 + n)
    assert len(gates) == layers * 4 * n
    want = oracle.run_packed(n, gates)
    results = {}
    for dtype in ("c128", "c64"):
        sv = qvm.StateVector(n, dtype, init=0)
        sv.run(gates)
        got = sv.amplitudes()
        results["plain_" + dtype] = (got, C128_TOL if dtype == "c128" else c64_bound(gate_ks(gates)))
    for dtype in ("c128", "c64"):
        plan = qvm.Plan(gates, n, dtype, k_max=4, tile_qubits=13 if dtype == "c64" else 12)
        sv = qvm.StateVector(n, dtype, init=0)
        plan.run(sv)
        results["greedy_" + dtype] = (sv.amplitudes(), C128_TOL if dtype == "c128" else plan_tau(plan))
    from paper_2212_14201_amd import learned_planner
    planner = learned_planner.load_default()
    if planner is not None:
        cand, plan, _ = planner.choose(qvm.GateArray(gates), n, "c64")
        sv = qvm.StateVector(n, "c64", init=0)
        plan.run(sv)
        results[f"learned_c64 {cand}"] = (sv.amplitudes(), plan_tau(plan))
    for name, (got, tol) in results.items():
        err = float(np.max(np.abs(got - want)))
        r2 = rel2(got, want)
        print(f"n={n} {name}: max-abs {err:.2e}, relative 2-norm {r2:.2e}, tol {tol:.1e}", flush=True)
        if "c128" in name:
            assert err <= tol
        else:
            assert r2 <= tol and err <= tol
    pz = oracle.expect_z_all(want)
    sv = qvm.StateVector(n, "c128", init=0)
    sv.run(gates)
    assert np.max(np.abs(sv.expect_z_all() - pz)) <= 1e-12


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_sweep_gate_kinds(dtype):
    """Each gate kind of the per-gate sweep, as the sweep generates it (32
    gates on seeded random qubits), on a random 16-qubit start state built
    from a rotation + CNOT circuit, against the oracle."""
    from paper_2212_14201_amd.sweeps import GATE_KINDS, gate_list
    n = 16
    prep = rotation_cnot_circuit(n, 2, 8300)
    for kind in GATE_KINDS:
        gates = prep + gate_list(kind, n, 32, 7)
        want = oracle.run_packed(n, gates)
        sv = qvm.StateVector(n, dtype, init=0)
        sv.run(gates)
        err = float(np.max(np.abs(sv.amplitudes() - want)))
        tol = C128_TOL if dtype == "c128" else c64_bound(gate_ks(gates))
        print(f"{kind} {dtype}: max-abs {err:.2e} tol {tol:.1e}", flush=True)
        assert err <= tol, kind
