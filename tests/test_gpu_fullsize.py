"""Full-size parity: the 28-qubit layered workload and the 30-qubit
QFT + brick workload (in the configuration bench.py times) against values
the FP64 oracle stored in tests/golden/ (written by make_golden.py)."""
import json
import math
import os

import numpy as np
import pytest

from tests.util import C128_TOL, U32, c64_bound, gate_ks
from workloads import config_circuit

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

qvm = pytest.importorskip("paper_2212_14201_amd.qvm")
HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(autouse=True)
def _gpu(require_gpu):
    pass


def golden(name):
    with open(os.path.join(HERE, "golden", name + ".json")) as fh:
        return json.load(fh)


def plan_bound(plan):
    st = plan.stats()
    s = sum((1 << plan.block(b)["k"]) + 4 for b in range(st["blocks"])) + 5 * st["diag_ops"]
    return 10.0 * math.sqrt(s) * U32


def check_samples(got, g, dtype):
    """complex128: the oracle's bin except where the target lies within
    1e-12 of a CDF boundary (then a neighbour).  complex64: at 2^28 bins of
    ~4e-9 probability each, a CDF perturbation of the state's rounding size
    (~1e-6) moves a sample by up to a few hundred bins, so only closeness is
    required (within 2^16 bins) and the rest is reported."""
    want = np.asarray(g["samples"], dtype=np.int64)
    got = got.astype(np.int64)
    if dtype == "c128":
        close = np.asarray(g["sample_margin"]) <= 1e-12
        assert np.array_equal(got[~close], want[~close])
        assert np.all(np.abs(got[close] - want[close]) <= 1)
        return f"{int(close.sum())} on a CDF boundary"
    d = np.abs(got - want)
    assert np.all(d <= 1 << 16)
    return f"bin distance median {int(np.median(d))}, max {int(d.max())}, exact {int(np.sum(d == 0))}"


@pytest.mark.parametrize("path", ["plain_c128", "plain_c64", "fused_c64"])
def test_layered_28_qubits(path):
    g = golden("layered28")
    cfg = config_circuit("layered28")
    n, gates = cfg["n"], cfg["gates"]
    dtype = "c128" if path.endswith("c128") else "c64"
    sv = qvm.StateVector(n, dtype, init=0)
    if path.startswith("plain"):
        sv.run(gates)
        tol = C128_TOL if dtype == "c128" else c64_bound(gate_ks(gates))
    else:
        plan = qvm.Plan(gates, n, dtype, k_max=4, tile_qubits=13)
        plan.run(sv)
        tol = plan_bound(plan)
    idx = np.asarray(g["amp_index"], dtype=np.uint64)
    want = np.asarray(g["amp_re"]) + 1j * np.asarray(g["amp_im"])
    err = float(np.max(np.abs(sv.gather(idx) - want)))
    ptol = 1e-13 if dtype == "c128" else 2 * tol + tol * tol
    z = sv.expect_z_all()
    zz, _ = sv.expect_pauli(np.zeros(n - 1, np.uint64),
                            np.array([(1 << q) | (1 << (q + 1)) for q in range(n - 1)], np.uint64))
    zerr = float(np.max(np.abs(z - g["z"])))
    zzerr = float(np.max(np.abs(zz - g["zz"])))
    samp = check_samples(sv.sample(cfg["uniforms"]), g, dtype)
    print(f"{path}: amp err {err:.2e} (tol {tol:.1e}), <Z> err {zerr:.2e}, <ZZ> err {zzerr:.2e}, "
          f"samples: {samp}")
    assert err <= tol
    assert zerr <= ptol and zzerr <= ptol


def bench_plan(gates, n):
    """The plan bench.py times: the shipped learned planner's choice, or the
    greedy planner with 4-qubit blocks in 13-qubit tiles without a model."""
    from paper_2212_14201_amd import learned_planner
    planner = learned_planner.load_default()
    ga = qvm.GateArray(gates)
    if planner is None:
        return qvm.Plan(ga, n, "c64", k_max=4, tile_qubits=13)
    return planner.choose(ga, n, "c64")[1]


def test_qft_brick_30_qubits_bench_configuration():
    """The bench's fused complex64 plan and the plain complex128 path on the
    30-qubit workload."""
    g = golden("qft30")
    cfg = config_circuit("qft30")
    n, x, gates = cfg["n"], cfg["init"], cfg["gates"]
    assert x == g["x"]
    idx = np.asarray(g["amp_index"], dtype=np.uint64)
    want = np.asarray(g["amp_re"]) + 1j * np.asarray(g["amp_im"])
    fused = qvm.StateVector(n, "c64", init=x)
    plan = bench_plan(gates, n)
    plan.run(fused)
    ferr = float(np.max(np.abs(fused.gather(idx) - want)))
    fz = float(np.max(np.abs(fused.expect_z_all() - g["z"])))
    del fused
    plain = qvm.StateVector(n, "c128", init=x)
    plain.run(gates)
    perr = float(np.max(np.abs(plain.gather(idx) - want)))
    pz = float(np.max(np.abs(plain.expect_z_all() - g["z"])))
    tol = plan_bound(plan)
    print(f"fused c64 amp err {ferr:.2e} (tol {tol:.1e}) <Z> {fz:.2e}; plain c128 amp err {perr:.2e} <Z> {pz:.2e}")
    assert perr <= C128_TOL and pz <= 1e-12
    assert ferr <= tol and fz <= 2 * tol + tol * tol
