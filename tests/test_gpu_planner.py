"""The learned planner end to end at small size: pass timings collected on
the GPU, the HIP MLP trained on them, a candidate chosen for a held-out
circuit, and the chosen plan's result checked against the oracle."""
import math

import numpy as np
import pytest

import oracle
from tests.util import U32
from workloads import random_planner_circuit

pytestmark = pytest.mark.gpu

lp = pytest.importorskip("paper_2212_14201_amd.learned_planner")


@pytest.fixture(autouse=True)
def _gpu(require_gpu):
    pass


def test_collect_train_choose(tmp_path):
    path = str(tmp_path / "rows.npz")
    rows = lp.collect(0, 40, path, n_range=(13, 16), g_range=(60, 120), mix=False)
    assert rows > 40
    F, T = lp.load_rows(path)
    assert F.shape[1] == lp.NFEAT and np.all(T > 0)
    planner, hist = lp.train(F, T, epochs=40, batch=256, log=False)
    assert hist[-1] < hist[0]
    n, gates = random_planner_circuit(10_000, n_range=(14, 14), g_range=(150, 150))
    from paper_2212_14201_amd import qvm
    ga = qvm.GateArray(gates)
    cand, plan, pred = planner.choose(ga, n, "c64")
    assert pred > 0
    sv = qvm.StateVector(n, "c64", init=0)
    plan.run(sv)
    want = oracle.simulate(n, gates)
    st = plan.stats()
    tau = 10 * math.sqrt(sum((1 << plan.block(b)["k"]) + 4 for b in range(st["blocks"]))
                         + 5 * st["diag_ops"]) * U32
    assert np.max(np.abs(sv.amplitudes() - want)) <= tau
    recs = lp.evaluate(planner, 20_000, 4, n_range=(13, 15), g_range=(60, 100), log=False)
    summ = lp.summarize(recs)
    assert summ["circuits"] == 4 and summ["amplitude_checks"] == 4
    assert summ["max_abs_err_vs_c128"] < 1e-5


def plan_tau(plan):
    st = plan.stats()
    return 10 * math.sqrt(sum((1 << plan.block(b)["k"]) + 4 for b in range(st["blocks"]))
                          + 5 * st["diag_ops"]) * U32


def test_trained_model_against_the_fallback():
    """The shipped model on held-out circuits of the planner workload (26-28
    qubits, 100-500 gates) against the greedy planner without it (its
    fallback setting, 3-qubit blocks in 13-qubit tiles): the measured total
    of the learned choices must not exceed the fallback's by more than 2%
    (the gain is printed), and the learned plan's whole state must agree
    with the plain complex128 path within 1e-5."""
    from paper_2212_14201_amd import qvm
    planner = lp.load_default()
    if planner is None:
        pytest.skip("no trained model shipped")
    recs = lp.evaluate(planner, 100_000, 6, n_range=(26, 28), g_range=(100, 500), log=False)
    for r in recs:
        print(f"seed {r['seed']} n={r['n']} gates={r['gates']} choice={r['choice']}: learned "
              f"{r['learned_ms']:.2f} ms, fallback {r['all_ms'][lp.cand_name(lp.FALLBACK)]:.2f} ms, "
              f"error vs complex128 {r['max_abs_err_vs_c128']:.1e}")
    summ = lp.summarize(recs)
    print("summary:", summ)
    fb = summ["vs_fallback"]
    assert summ["learned_total_ms"] <= 1.02 * fb["total_ms"]
    assert summ["within_1e-5"] == len(recs)


def test_adaptive_plan_on_gpu():
    """A plan whose passes each take their own block width (3..5) runs on
    the GPU and reproduces the oracle in both dtypes."""
    from paper_2212_14201_amd import qvm
    n, gates = random_planner_circuit(100_321, n_range=(15, 15), g_range=(200, 200))
    want = oracle.simulate(n, gates, init=5)
    for dtype, tile in (("c64", 12), ("c128", 11)):
        npass = qvm.Plan(gates, n, dtype, k_max=3, tile_qubits=tile, image=False).stats()["passes"]
        ks = np.random.default_rng(7).integers(3, 6, npass)
        plan = qvm.Plan(gates, n, dtype, tile_qubits=tile, k_of_pass=ks)
        sv = qvm.StateVector(n, dtype, init=5)
        plan.run(sv)
        err = float(np.max(np.abs(sv.amplitudes() - want)))
        tol = plan_tau(plan) if dtype == "c64" else 1e-12
        print(f"{dtype}: widths {ks.tolist()}, error {err:.1e} (bound {tol:.1e})")
        assert err <= tol


def test_plan_front_end_with_the_learned_planner():
    """qvm.plan(circuit, planner="learned") builds the shipped model's choice
    and the plan reproduces the oracle."""
    from paper_2212_14201_amd import qvm
    if lp.load_default() is None:
        pytest.skip("no trained model shipped")
    n, gates = random_planner_circuit(100_123, n_range=(14, 14), g_range=(120, 120))
    c = qvm.Circuit(n, gates)
    plan = qvm.plan(c, planner="learned")
    sv = qvm.StateVector(n, "c64", init=3)
    plan.run(sv)
    want = oracle.simulate(n, gates, init=3)
    assert np.max(np.abs(sv.amplitudes() - want)) <= plan_tau(plan)
