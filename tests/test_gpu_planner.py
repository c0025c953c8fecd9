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
    rows = lp.collect(0, 40, path, n_range=(13, 16), g_range=(60, 120))
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
