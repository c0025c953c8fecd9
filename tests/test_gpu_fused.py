"""GPU parity of the fused path (tile passes with MFMA blocks, phase and
diagonal ops, tile-bit remapping) against the FP64 oracle."""
import math

import numpy as np
import pytest

import oracle
from tests.util import C128_TOL, U32, blocks_and_diagonals, epilogue_runs, long_phase_run
from workloads import (Gate, config_circuit, layered_u3_cz, qft_circuit, qft_then_brick,
                       random_mixed_circuit, random_planner_circuit, random_pauli_sum)

pytestmark = pytest.mark.gpu

qvm = pytest.importorskip("paper_2212_14201_amd.qvm")


@pytest.fixture(autouse=True)
def _gpu(require_gpu):
    pass


def plan_bound(plan):
    """Stated complex64 bound for a plan: each block of 2^k columns and each
    diagonal op counts as one pass in the rounding model."""
    st = plan.stats()
    s = 0
    for b in range(st["blocks"]):
        s += (1 << plan.block(b)["k"]) + 4
    s += 5 * st["diag_ops"]
    return 10.0 * math.sqrt(max(s, 1)) * U32


def run_fused(n, gates, dtype, k_max, tile, init=0):
    plan = qvm.Plan(gates, n, dtype, k_max=k_max, tile_qubits=tile)
    sv = qvm.StateVector(n, dtype, init=init)
    plan.run(sv)
    return sv, plan


CASES = [  # n, k_max, tile
    (9, 3, 0), (9, 5, 0), (10, 4, 0), (12, 5, 0), (12, 6, 0), (14, 3, 10), (14, 5, 10),
    (15, 4, 12), (16, 5, 12), (13, 2, 8), (16, 3, 11), (17, 4, 11),
]


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("n,k_max,tile", CASES)
def test_fused_random_circuits(n, k_max, tile, dtype):
    if dtype == "c128" and tile > 12:
        pytest.skip("complex128 tiles hold at most 12 qubits")
    gates = random_mixed_circuit(n, 90, 500 + n + k_max, kmax=min(3, k_max),
                                 max_ctrl=max(0, min(2, k_max - 3)))
    init = (37 * n) % (1 << n)
    sv, plan = run_fused(n, gates, dtype, k_max, tile, init)
    want = oracle.simulate(n, gates, init=init)
    got = sv.amplitudes()
    err = float(np.max(np.abs(got - want)))
    tol = C128_TOL if dtype == "c128" else plan_bound(plan)
    print(f"n={n} k={k_max} tile={tile} {dtype} {plan.stats()} err={err:.2e} tol={tol:.2e}")
    assert err <= tol


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_fused_layered_12(dtype):
    n = 12
    gates = layered_u3_cz(n, 20, 1201)
    want = oracle.simulate(n, gates)
    for k, tile in ((5, 0), (4, 10), (3, 12)):
        sv, plan = run_fused(n, gates, dtype, k, tile)
        tol = C128_TOL if dtype == "c128" else plan_bound(plan)
        assert np.max(np.abs(sv.amplitudes() - want)) <= tol
        assert np.max(np.abs(sv.expect_z_all() - oracle.expect_z_all(want))) <= 4 * tol


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_fused_qft_closed_form_16(dtype):
    """Closed-form QFT amplitudes at 16 qubits through the fused path; the
    final swaps become relabelings, so the layout is permuted afterwards."""
    n, x = 16, 40503
    y = np.arange(1 << n)
    want = np.exp(2j * np.pi * ((x * y) % (1 << n)) / (1 << n)) / math.sqrt(1 << n)
    for k, tile in ((5, 0), (5, 12), (4, 12)):
        sv, plan = run_fused(n, qft_circuit(n), dtype, k, tile, init=x)
        tol = 1e-12 if dtype == "c128" else plan_bound(plan)
        # the final swaps are relabelings: the state is left in the plan's
        # final layout, which is not the identity
        assert np.array_equal(sv.layout(), plan.final_layout())
        assert not np.array_equal(sv.layout(), np.arange(n))
        assert np.max(np.abs(sv.amplitudes() - want)) <= tol
        # layout reset physically restores the identity order
        sv.reset_layout()
        assert np.array_equal(sv.layout(), np.arange(n))
        assert np.max(np.abs(sv.amplitudes() - want)) <= tol


def test_fused_readouts_with_permuted_layout():
    n = 14
    x, gates = qft_then_brick(n, 6, 77)
    want = oracle.simulate(n, gates, init=x)
    sv, plan = run_fused(n, gates, "c128", 5, 12, init=x)
    assert not np.array_equal(plan.final_layout(), np.arange(n))
    assert np.max(np.abs(sv.probabilities() - oracle.probabilities(want))) < 1e-13
    qs = [3, 11, 0, 7]
    assert np.max(np.abs(sv.probabilities(qs) - oracle.marginal(want, qs))) < 1e-13
    assert np.max(np.abs(sv.expect_z_all() - oracle.expect_z_all(want))) < 1e-12
    xs, zs, cs, _ = random_pauli_sum(n, 20, 8, wmin=1, wmax=4)
    terms, _ = sv.expect_pauli(xs, zs)
    ref = [oracle.expect_pauli(want, int(a), int(b))[0] for a, b in zip(xs, zs)]
    assert np.max(np.abs(terms - ref)) < 1e-12
    u = np.random.default_rng(3).random(500)
    got = sv.sample(u).astype(np.int64)
    ref, margin = oracle.sample(want, u)
    close = margin < 1e-12
    assert np.array_equal(got[~close], ref.astype(np.int64)[~close])
    with pytest.raises(qvm.QvmError):
        plan.run(sv)                    # needs the identity layout


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_fused_planner_gate_set(dtype):
    n, gates = random_planner_circuit(4, n_range=(13, 13), g_range=(150, 150))
    want = oracle.simulate(n, gates)
    for k, tile in ((3, 0), (4, 0), (6, 0), (5, 11)):
        sv, plan = run_fused(n, gates, dtype, k, tile)
        tol = C128_TOL if dtype == "c128" else plan_bound(plan)
        assert np.max(np.abs(sv.amplitudes() - want)) <= tol


def test_partition_plan_on_gpu():
    n = 11
    gates = random_mixed_circuit(n, 50, 8, kmax=2, max_ctrl=1)
    part = np.arange(len(gates), dtype=np.uint32) // 3
    try:
        plan = qvm.Plan(gates, n, "c128", k_max=6, partition=part)
    except qvm.QvmError:
        part = np.arange(len(gates), dtype=np.uint32)
        plan = qvm.Plan(gates, n, "c128", k_max=6, partition=part)
    sv = qvm.StateVector(n, "c128")
    plan.run(sv)
    assert np.max(np.abs(sv.amplitudes() - oracle.simulate(n, gates))) <= C128_TOL


def test_fused_c64_against_plain_c128_at_20_qubits():
    """Larger state: the fused complex64 result against the plain complex128
    path and against oracle amplitudes at sampled indices."""
    n = 20
    x, gates = qft_then_brick(n, 8, 3001)
    plain = qvm.StateVector(n, "c128", init=x)
    plain.run(gates)
    sv, plan = run_fused(n, gates, "c64", 5, 13, init=x)
    idx = np.random.default_rng(0).integers(0, 1 << n, 4096, dtype=np.uint64)
    a = sv.gather(idx)
    b = plain.gather(idx)
    want = oracle.simulate(n, gates, init=x)[idx.astype(np.int64)]
    assert np.max(np.abs(b - want)) <= C128_TOL
    assert np.max(np.abs(a - want)) <= plan_bound(plan)


def diagonal_heavy_circuit(n, seed):
    """H on every qubit, then long runs of diagonal gates between sparse
    dense layers: random-angle RZ, RZZ and controlled phases, T, S, CZ-only
    stretches (sign-only runs) and multi-controlled phases, so that runs take
    both the term-by-term and the angle-accumulating path of the tile kernel,
    with conditions on tile bits below and above the thread bits and on
    outer bits."""
    rng = np.random.Generator(np.random.PCG64(seed))
    gates = [Gate("h", (q,)) for q in range(n)]
    for layer in range(6):
        for _ in range(int(rng.integers(3, 25))):
            kind = int(rng.integers(0, 7))
            a, b, c = (int(v) for v in rng.choice(n, 3, replace=False))
            th = float(rng.uniform(0, 2 * math.pi))
            gates.append([Gate("rz", (a,), (), (th,)), Gate("rzz", (a, b), (), (th,)),
                          Gate("p", (a,), (b,), (th,)), Gate("t", (a,)), Gate("s", (a,)),
                          Gate("z", (a,), (b,)), Gate("p", (a,), (b, c), (th,))][kind])
        if layer % 2:
            gates += [Gate("z", (q + 1,), (q,)) for q in range(layer % 2, n - 1, 2)] * 2
            gates += [Gate("z", (q,), (int(rng.integers(0, q)),)) for q in range(1, n)]
        q = int(rng.integers(0, n))
        gates.append(Gate("u3", (q,), (), tuple(float(v) for v in rng.uniform(0, 2 * math.pi, 3))))
    return gates


@pytest.mark.parametrize("dtype,n,k_max,tile", [("c64", 9, 4, 5), ("c64", 10, 4, 6), ("c128", 9, 4, 4),
                                               ("c128", 10, 4, 5), ("c128", 8, 4, 6)])
def test_fused_narrow_tiles(dtype, n, k_max, tile):
    """Tiles with few slots beside the always-local low bits: the plan
    includes passes that only remap, to bring a blocked gate's wires in."""
    gates = random_mixed_circuit(n, 60, 910 + n + tile, kmax=3, max_ctrl=1)
    sv, plan = run_fused(n, gates, dtype, k_max, tile, init=5)
    want = oracle.simulate(n, gates, init=5)
    err = float(np.max(np.abs(sv.amplitudes() - want)))
    tol = C128_TOL if dtype == "c128" else plan_bound(plan)
    print(f"n={n} k={k_max} tile={tile} {dtype} {plan.stats()} err={err:.2e} tol={tol:.2e}")
    assert err <= tol


@pytest.mark.parametrize("dtype,n,tile", [(d, n, t) for d in ("c128", "c64")
                                          for n, t in ((14, 10), (16, 12), (12, 12))]
                         + [("c64", 13, 13), ("c64", 18, 13), ("c64", 8, 8)])
def test_fused_long_diagonal_runs(n, tile, dtype):
    gates = diagonal_heavy_circuit(n, 900 + n + tile)
    sv, plan = run_fused(n, gates, dtype, 3, tile, init=0)
    want = oracle.simulate(n, gates)
    err = float(np.max(np.abs(sv.amplitudes() - want)))
    tol = C128_TOL if dtype == "c128" else plan_bound(plan)
    print(f"n={n} tile={tile} {dtype} {plan.stats()} err={err:.2e} tol={tol:.2e}")
    assert err <= tol


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_simplified_circuit_on_gpu(dtype):
    """Peephole pre-pass then fused plan on the GPU, against the oracle on
    the original circuit."""
    from tests.test_simplify_cpu import redundant_circuit
    n = 12
    gates = redundant_circuit(n, 400, 4200)
    ga = qvm.simplify(gates, n)
    assert ga.n < len(gates)
    plan = qvm.Plan(ga, n, dtype, k_max=4, tile_qubits=10)
    sv = qvm.StateVector(n, dtype, init=5)
    plan.run(sv)
    err = float(np.max(np.abs(sv.amplitudes() - oracle.simulate(n, gates, init=5))))
    tol = C128_TOL if dtype == "c128" else plan_bound(plan)
    print(f"{dtype}: {len(gates)} -> {ga.n} gates, err {err:.2e} tol {tol:.2e}")
    assert err <= tol


@pytest.mark.parametrize("n,k_max", [(13, 3), (13, 4), (18, 3), (20, 4)])
def test_fused_epilogue_runs(n, k_max):
    """complex64 in 13-qubit tiles: diagonal runs right after a 3- or
    4-qubit block are applied by that block's epilogue (terms over its
    output layout, with conditions on outer bits across many tiles)."""
    gates = blocks_and_diagonals(n, 4300 + n + k_max, layers=20)
    init = (91 * n) % (1 << n)
    sv, plan = run_fused(n, gates, "c64", k_max, 13, init)
    ne = epilogue_runs(plan)
    want = oracle.simulate(n, gates, init=init)
    err = float(np.max(np.abs(sv.amplitudes() - want)))
    tol = plan_bound(plan)
    print(f"n={n} k={k_max} {plan.stats()} epilogue runs {ne} err={err:.2e} tol={tol:.2e}")
    assert ne >= 5
    assert err <= tol


@pytest.mark.parametrize("n,k_max", [(13, 3), (19, 4)])
def test_fused_epilogue_sign_runs(n, k_max):
    """Runs of CZ and Z gates only: the block epilogues flip signs (the sign
    bit of each output) instead of taking a phase factor."""
    gates = blocks_and_diagonals(n, 4400 + n + k_max, layers=20, signs_only=True)
    init = (57 * n) % (1 << n)
    sv, plan = run_fused(n, gates, "c64", k_max, 13, init)
    ns = epilogue_runs(plan, signs=True)
    want = oracle.simulate(n, gates, init=init)
    err = float(np.max(np.abs(sv.amplitudes() - want)))
    tol = plan_bound(plan)
    print(f"n={n} k={k_max} {plan.stats()} epilogue sign runs {ns} err={err:.2e} tol={tol:.2e}")
    assert ns >= 5
    assert err <= tol


@pytest.mark.parametrize("case,n,k_max,tile,dtype", [
    ("qftbrick", 16, 3, 11, "c64"), ("qftbrick", 16, 3, 11, "c128"), ("qftbrick", 20, 3, 13, "c64"),
    ("qftbrick", 22, 4, 13, "c64"), ("mixed", 14, 3, 10, "c64"), ("mixed", 14, 4, 10, "c128")])
def test_fused_defer_narrow(case, n, k_max, tile, dtype):
    """Plans whose tile passes leave narrow trailing blocks to a later pass
    (the learned planner's "tiled" candidates) against the oracle; each case
    is one where the deferral changes the plan."""
    if case == "qftbrick":
        init, gates = qft_then_brick(n, 12, 600 + n)
    else:
        init, gates = (29 * n) % (1 << n), random_mixed_circuit(n, 200, 700 + n, kmax=3, max_ctrl=0)
    plan = qvm.Plan(gates, n, dtype, k_max=k_max, tile_qubits=tile, defer_narrow=True)
    base = qvm.Plan(gates, n, dtype, k_max=k_max, tile_qubits=tile, image=False).stats()
    st = plan.stats()
    assert (st["blocks"], st["passes"], st["blocks_by_k"]) != (base["blocks"], base["passes"], base["blocks_by_k"])
    sv = qvm.StateVector(n, dtype, init=init)
    plan.run(sv)
    want = oracle.simulate(n, gates, init=init)
    err = float(np.max(np.abs(sv.amplitudes() - want)))
    tol = C128_TOL if dtype == "c128" else plan_bound(plan)
    print(f"{case} n={n} k={k_max} tile={tile} {dtype} {st} (without: {base['passes']} passes, "
          f"{base['blocks']} blocks) err={err:.2e} tol={tol:.2e}")
    assert err <= tol


@pytest.mark.parametrize("count", [200, 1100])
def test_fused_long_phase_run_after_a_block(count):
    """complex64, 13 qubits: a run of controlled phases after a block, in the
    block's epilogue through the pass's phase sums (200 gates) or on its own
    once its bound passes the phase-sum area (1,100 gates), against the
    oracle."""
    n = 13
    gates = long_phase_run(n, count, 5100 + count)
    init = 77
    sv, plan = run_fused(n, gates, "c64", 3, 13, init)
    want = oracle.simulate(n, gates, init=init)
    err = float(np.max(np.abs(sv.amplitudes() - want)))
    tol = plan_bound(plan)
    print(f"{count} phases: {plan.stats()} epilogue runs {epilogue_runs(plan)} err={err:.2e} tol={tol:.2e}")
    assert (epilogue_runs(plan) > 0) == (count < 1024)
    assert err <= tol
