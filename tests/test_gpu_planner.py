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
    recs, checks = lp.evaluate(planner, 20_000, 4, all_cands=2, check_amplitudes=2,
                               n_range=(13, 15), g_range=(60, 100))
    summ = lp.summarize(recs, checks)
    assert summ["circuits"] == 4 and summ["max_abs_err_vs_c128"] < 1e-5


def test_trained_model_gains_over_greedy():
    """The shipped model against the greedy planner's classic setting (one
    5-qubit block per pass) on held-out circuits from the training
    distribution (26-28 qubits, 100-500 gates): measured total time of the
    learned choices must not exceed the greedy total, and the learned plan's
    amplitudes must agree with the plain complex128 path."""
    from paper_2212_14201_amd import qvm
    planner = lp.load_default()
    if planner is None:
        pytest.skip("no trained model shipped")
    pool = lp.StatePool()
    learned = greedy = 0.0
    for s in range(100_000, 100_006):
        n, gates = random_planner_circuit(s, n_range=(26, 28), g_range=(100, 500))
        ga = qvm.GateArray(gates)
        cand, plan, _ = planner.choose(ga, n, "c64")
        sv = pool.get(n, "c64")
        lp.time_plan(sv, plan)                        # warm-up
        lms = lp.time_plan(sv, plan)[0]
        gms = lp.time_plan(sv, lp.build_plan(ga, n, "c64", lp.GREEDY))[0]
        print(f"seed {s} n={n} gates={len(gates)} choice={cand}: learned {lms:.2f} ms, greedy {gms:.2f} ms")
        learned += lms
        greedy += gms
    print(f"gain over greedy: {greedy / learned:.2f}x")
    assert learned <= greedy
    # the last circuit's learned plan against the plain complex128 path
    sv.init_basis(0)
    plan.run(sv)
    del pool
    plain = qvm.StateVector(n, "c128", init=0)
    plain.run(ga)
    idx = np.random.default_rng(s).integers(0, 1 << n, 4096, dtype=np.uint64)
    st = plan.stats()
    tau = 10 * math.sqrt(sum((1 << plan.block(b)["k"]) + 4 for b in range(st["blocks"]))
                         + 5 * st["diag_ops"]) * U32
    assert np.max(np.abs(sv.gather(idx) - plain.gather(idx))) <= tau


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
    st = plan.stats()
    tau = 10 * math.sqrt(sum((1 << plan.block(b)["k"]) + 4 for b in range(st["blocks"]))
                         + 5 * st["diag_ops"]) * U32
    assert np.max(np.abs(sv.amplitudes() - want)) <= tau
