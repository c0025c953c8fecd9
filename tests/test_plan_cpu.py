"""Host-side checks of the fusion planner: plan validity and block matrices.

Block matrices built by the library (FP64) are compared with the oracle's
block construction over the same gates and qubits; the execution order the
plan reports is checked with the oracle's plan validator.
"""
import numpy as np
import pytest

import oracle
from workloads import (Gate, config_circuit, layered_u3_cz, qft_circuit,
                       random_mixed_circuit, random_planner_circuit)

qvm = pytest.importorskip("paper_2212_14201_amd.qvm")


def units_in_order(plan, ngates):
    pos, unit = plan.schedule()
    groups = {}
    for i in range(ngates):
        if unit[i] >= 0:
            groups.setdefault(unit[i], []).append((pos[i], i))
    return [[i for _, i in sorted(groups[u])] for u in sorted(groups)]


def on_wires(gates):
    """Rewrite gates onto wires: an uncontrolled SWAP exchanges the wires of
    its two qubits and is dropped (the relabeling the planner performs)."""
    w = list(range(64))
    out = {}
    for i, g in enumerate(gates):
        if g.name == "swap" and not g.controls:
            a, b = g.targets
            w[a], w[b] = w[b], w[a]
            continue
        out[i] = Gate(g.name, tuple(w[t] for t in g.targets), tuple(w[c] for c in g.controls),
                      g.params, g.pidx, g.matrix)
    return out


def check_plan(gates, n, k_max, tile, dtype="c64", relabeled_swaps=None):
    plan = qvm.Plan(gates, n, dtype, k_max=k_max, tile_qubits=tile)
    st = plan.stats()
    units = units_in_order(plan, len(gates))
    wg = on_wires(gates)
    kept = sorted(wg)
    sub = [wg[i] for i in kept]
    remap = {g: j for j, g in enumerate(kept)}
    ok, why = oracle.validate_plan(sub, [[remap[i] for i in u] for u in units], n)
    assert ok, why
    for b in range(st["blocks"]):
        blk = plan.block(b)
        assert blk["k_true"] <= k_max
        assert set(q for gi in blk["gates"] for q in wg[gi].qubits()) <= set(blk["qubits"])
        want = oracle.block_matrix([wg[i] for i in blk["gates"]], blk["qubits"])
        assert np.max(np.abs(blk["matrix"] - want)) < 1e-13
    return plan, st


@pytest.mark.parametrize("k_max", [1, 2, 3, 4, 5, 6])
@pytest.mark.parametrize("tile", [0, 8])
def test_random_circuits_plans_valid(k_max, tile):
    n = 10
    if tile and tile < k_max:
        pytest.skip("tile narrower than a block")
    gates = random_mixed_circuit(n, 120, 100 + k_max, kmax=min(3, k_max), max_ctrl=max(0, k_max - 3))
    check_plan(gates, n, k_max, tile)


def test_layered_and_qft_plans():
    check_plan(layered_u3_cz(12, 20, 1201), 12, 5, 0, "c128")
    check_plan(layered_u3_cz(12, 20, 1201), 12, 4, 10, "c128")
    plan, st = check_plan(qft_circuit(9), 9, 4, 0, "c64", relabeled_swaps=True)
    # the uncontrolled SWAPs are relabelings: nothing executes them
    pos, unit = plan.schedule()
    assert all(unit[i] == -1 for i, g in enumerate(qft_circuit(9)) if g.name == "swap")


def test_thirty_qubit_workload_plans():
    cfg = config_circuit("qft30")
    for k, tile in ((5, 0), (5, 13), (3, 13)):
        plan = qvm.Plan(cfg["gates"], 30, "c64", k_max=k, tile_qubits=tile)
        st = plan.stats()
        assert st["blocks"] > 0 and st["passes"] > 0
        if tile:
            assert st["passes"] < 40
        # every non-relabeled gate is scheduled exactly once
        pos, unit = plan.schedule()
        live = pos[pos >= 0]
        assert np.array_equal(np.sort(live), np.arange(live.size))


def test_planner_workload_plans_valid():
    for seed in range(3):
        n, gates = random_planner_circuit(seed, n_range=(10, 12), g_range=(60, 120))
        for k in (3, 4, 6):
            check_plan(gates, n, k, 0)


def test_partition_plan():
    n = 6
    gates = random_mixed_circuit(n, 30, 5, kmax=2, max_ctrl=0)
    # one block per gate is always a valid partition
    part = np.arange(len(gates), dtype=np.uint32)
    plan = qvm.Plan(gates, n, "c128", k_max=2, partition=part)
    assert plan.stats()["blocks"] == len(gates)
    # reversing two dependent gates must be rejected
    bad = part.copy()
    i = next(i for i in range(1, len(gates))
             if set(gates[i].qubits()) & set(gates[i - 1].qubits()))
    bad[i], bad[i - 1] = bad[i - 1], bad[i]
    with pytest.raises(qvm.QvmError):
        qvm.Plan(gates, n, "c128", k_max=2, partition=bad)


def test_plan_argument_errors():
    g = [Gate("h", (0,)), Gate("x", (2,), (0, 1))]
    with pytest.raises(qvm.QvmError):
        qvm.Plan(g, 3, "c64", k_max=2)          # Toffoli spans 3 > k_max
    with pytest.raises(qvm.QvmError):
        qvm.Plan(g, 3, "c64", k_max=7)
    with pytest.raises(qvm.QvmError):
        qvm.Plan(g, 20, "c64", k_max=5, tile_qubits=14)
    with pytest.raises(qvm.QvmError):
        qvm.Plan([Gate("h", (5,))], 3, "c64", k_max=3)


def test_pass_features():
    lp = pytest.importorskip("paper_2212_14201_amd.learned_planner")
    cfg = config_circuit("qft30")
    for k, tile in ((5, 0), (4, 13)):
        plan = qvm.Plan(cfg["gates"], 30, "c64", k_max=k, tile_qubits=tile)
        F = lp.plan_features(plan)
        st = plan.stats()
        assert F.shape == (st["passes"], lp.NFEAT)
        assert np.all(F[:, 0] == 30) and np.all(F[:, 1] == 0) and np.all(F[:, 2] == 13)
        assert F[:, 3:7].sum() == st["blocks"]
        assert F[:, 10].sum() == len(cfg["gates"]) - 15        # swaps are relabelings
        assert np.all(F[:, 18] == 33) and np.all(F[:, 19] == 17)
        # angle-accumulating runs are a subset of all runs and terms
        assert np.all(F[:, 20] <= F[:, 8]) and np.all(F[:, 21] <= F[:, 9])
        assert np.all((F[:, 20] == 0) == (F[:, 21] == 0))


def test_sweep_gate_lists():
    """The paper-shaped sweep builds valid gates of every kind (checked by
    the library's own validation when packed) with the stated touched
    fractions."""
    sweeps = pytest.importorskip("paper_2212_14201_amd.sweeps")
    for kind in sweeps.GATE_KINDS:
        gates = sweeps.gate_list(kind, 12, 16, 5)
        ga = qvm.GateArray(gates)
        plan = qvm.Plan(ga, 12, "c64", k_max=3)
        assert plan.stats()["passes"] >= 1
        for g in gates:
            if g.name == "unitary":
                u = np.asarray(g.matrix)
                assert np.allclose(u @ u.conj().T, np.eye(u.shape[0]), atol=1e-12)
    assert sweeps.touched_fraction("toffoli") == 0.25


def test_scoring_only_plans_match_full_plans():
    """A plan built without its image carries the same schedule, statistics
    (apart from the device bytes) and pass features as the full plan, and
    refuses to hand out block matrices."""
    lp = pytest.importorskip("paper_2212_14201_amd.learned_planner")
    cfg = config_circuit("qft30")
    for k, tile in ((5, 0), (3, 13), (4, 12)):
        full = qvm.Plan(cfg["gates"], 30, "c64", k_max=k, tile_qubits=tile)
        lean = qvm.Plan(cfg["gates"], 30, "c64", k_max=k, tile_qubits=tile, image=False)
        sf, sl = full.stats(), lean.stats()
        assert sl["device_bytes"] < sf["device_bytes"]
        sf.pop("device_bytes"), sl.pop("device_bytes")
        assert sf == sl
        assert np.array_equal(lp.plan_features(full), lp.plan_features(lean))
        for a, b in zip(full.schedule(), lean.schedule()):
            assert np.array_equal(a, b)
        assert np.array_equal(full.final_layout(), lean.final_layout())
        with pytest.raises(qvm.QvmError):
            lean.block(0)
    with pytest.raises(ValueError):
        qvm.Plan(cfg["gates"], 30, "c64", k_max=2, partition=np.zeros(len(cfg["gates"])), image=False)


def test_plan_flags_rejected():
    qvm.Plan([Gate("h", (0,))], 3, "c64", k_max=3)
    L = qvm.lib()
    ga = qvm.GateArray([Gate("h", (0,))])
    h = qvm.ctypes.c_void_p()
    st = L.qvm_plan_greedy_ex(ga.ptr(), ga.n, 3, 3, 0, qvm.QVM_C64, 2, qvm.ctypes.byref(h))
    assert qvm.STATUS[st] == "QVM_EARG" and not h.value


# Device-image records of the tile kernel (layouts in csrc/tile.hpp).
_PD = np.dtype([("L", "<i4"), ("c", "<i4"), ("nops", "<i4"), ("remap", "<i4"), ("kmax", "<i4"),
                ("first_block", "<i4"), ("qmask", "<u8"), ("ops", "<u8"), ("ldoff", "<u8"),
                ("rmhi", "<u8"), ("rmlo", "<u8")])
_TOP = np.dtype([("type", "<i4"), ("k", "<i4"), ("lb", "<i4", 6), ("data", "<u8"),
                 ("next_block", "<i4"), ("flags", "<i4"), ("tab", "<u8")])
_DSUB = np.dtype([("lmask", "<u4"), ("lval", "<u4"), ("neg", "<i4"), ("rows", "<u4"), ("omask", "<u8"),
                  ("oval", "<u8"), ("pr", "<f8"), ("pi", "<f8"), ("turns", "<u8"), ("pad", "<u8")])
_DTERM = np.dtype([("omask", "<u8"), ("oval", "<u8"), ("turns", "<u8"), ("lmask", "<u4"), ("lval", "<u4")])


def plan_image(plan):
    import ctypes
    L = qvm.lib()
    L.qvm_plan_image.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t,
                                 ctypes.POINTER(ctypes.c_size_t), ctypes.POINTER(ctypes.c_uint64),
                                 ctypes.POINTER(ctypes.c_int32)]
    nb, pt, npass = ctypes.c_size_t(), ctypes.c_uint64(), ctypes.c_int32()
    qvm.check(L.qvm_plan_image(plan._h, None, 0, ctypes.byref(nb), ctypes.byref(pt), ctypes.byref(npass)))
    buf = np.zeros(nb.value, np.uint8)
    qvm.check(L.qvm_plan_image(plan._h, buf.ctypes.data, nb.value, None, None, None))
    rec = lambda off, dt, cnt: np.frombuffer(buf[off: off + cnt * dt.itemsize].tobytes(), dt)
    return rec, rec(pt.value, _PD, npass.value)


def emulate_diagonal_pass(plan, n, width):
    """Phase of every basis index after the single pass of a plan over a
    diagonal-only circuit, from the image's diagonal runs: term-by-term
    factors for short runs; grouped angle sums and the subset-sum over the
    element bits for angle-path runs."""
    rec, passes = plan_image(plan)
    assert len(passes) == 1 and passes[0]["L"] == n
    pd = passes[0]
    L, c = n, int(pd["c"])
    ldoff = rec(int(pd["ldoff"]), np.dtype("<u8"), 1 << (L - c))
    e = np.arange(1 << L, dtype=np.uint64)
    phys = (e & np.uint64((1 << c) - 1)) | ldoff[(e >> np.uint64(c)).astype(np.int64)]
    nt = 512
    nhb = max(L - 9, 0)
    t = np.arange(min(nt, 1 << L), dtype=np.uint64)
    wmask = np.uint64((1 << width) - 1) if width < 64 else np.uint64(~np.uint64(0))
    phase = np.ones(1 << L, np.complex128)
    n_turns = 0
    for op in rec(int(pd["ops"]), _TOP, int(pd["nops"])):
        assert op["type"] == 2
        if op["flags"] & 1:
            n_turns += 1
            terms = rec(int(op["data"]), _DTERM, int(op["k"]))
            off = rec(int(op["tab"]), np.dtype("<u4"), (1 << nhb) + 1)
            assert off[-1] == len(terms) and np.all(np.diff(off.astype(np.int64)) >= 0)
            acc = np.zeros((1 << nhb, len(t)), np.uint64)
            for g in range(1 << nhb):
                for d in terms[off[g]: off[g + 1]]:
                    assert d["oval"] == 0 and d["lmask"] < nt and d["lval"] & ~d["lmask"] == 0
                    hit = (t & np.uint64(d["lmask"])) == np.uint64(d["lval"])
                    acc[g] = (acc[g] + np.where(hit, d["turns"], np.uint64(0))) & wmask
            for b in range(nhb):
                for i in range(1 << nhb):
                    if (i >> b) & 1:
                        acc[i] = (acc[i] + acc[i ^ (1 << b)]) & wmask
            ang = acc.reshape(-1)              # element t + 512 i at i * len(t) + t
            if op["flags"] & 2:
                phase *= np.where(ang >> np.uint64(width - 1), -1.0, 1.0)
            else:
                phase *= np.exp(2j * np.pi * (ang.astype(np.float64) / 2.0 ** width))
        else:
            for d in rec(int(op["data"]), _DSUB, int(op["k"])):
                hit = (e & np.uint64(d["lmask"])) == np.uint64(d["lval"])
                f = -1.0 if d["neg"] else d["pr"] + 1j * d["pi"]
                phase = np.where(hit, phase * f, phase)
    out = np.zeros(1 << n, np.complex128)
    out[phys.astype(np.int64)] = phase
    return out, n_turns


@pytest.mark.parametrize("dtype,n", [("c64", 13), ("c64", 11), ("c128", 12), ("c64", 8)])
def test_angle_path_encoding_reproduces_diagonal(dtype, n):
    """Pins the planner's encoding of long diagonal runs (element-bit zeros
    rewritten as 1 - h, merged terms, grouped sums, subset sums) against
    the oracle: on a diagonal-only circuit the state from the uniform
    superposition carries exactly the circuit's diagonal."""
    rng = np.random.Generator(np.random.PCG64(77 + n))
    gates = []
    for _ in range(60):
        kind = int(rng.integers(0, 7))
        a, b, cq = (int(v) for v in rng.choice(n, 3, replace=False))
        th = float(rng.uniform(0, 2 * np.pi))
        gates.append([Gate("rz", (a,), (), (th,)), Gate("rzz", (a, b), (), (th,)),
                      Gate("p", (a,), (b,), (th,)), Gate("t", (a,)), Gate("sdg", (a,)),
                      Gate("p", (a,), (b, cq), (th,)), Gate("rz", (a,), (b,), (th,))][kind])
    signs = [Gate("z", (int(q),), (int(r),)) for q, r in rng.integers(0, n, (12, 2)) if q != r]
    for gl, only_signs in ((gates, False), (signs, True)):
        plan = qvm.Plan(gl, n, dtype, k_max=3, tile_qubits=n)
        got, n_turns = emulate_diagonal_pass(plan, n, 32 if dtype == "c64" else 64)
        assert n_turns >= 1
        psi = np.full(1 << n, 2.0 ** (-n / 2), np.complex128)
        want = oracle.apply_gates(psi, n, gl) * 2.0 ** (n / 2)
        tol = 1e-7 if dtype == "c64" else 1e-12
        assert np.max(np.abs(got - want)) < tol, (only_signs, np.max(np.abs(got - want)))


@pytest.mark.parametrize("dtype,c", [("c64", 4), ("c128", 3)])
def test_narrow_tiles_plan_and_validate(dtype, c):
    """Tiles with one to three slots beside the low bits every tile holds:
    the scheduler inserts passes without ops whose remap brings a blocked
    gate's wires onto the low bits; the plans are valid and their blocks
    match the oracle.  A tile no wider than those low bits is rejected."""
    for n in (6, 8, 9):
        gates = random_mixed_circuit(n, 40, 900 + n, kmax=3, max_ctrl=1)
        for free in (1, 2, 3):
            for k in (3, 4):
                tile = c + free
                if tile < k or tile >= n:
                    continue
                plan, st = check_plan(gates, n, k, tile, dtype)
                assert st["passes"] >= 1
        with pytest.raises(qvm.QvmError, match="tile_qubits must exceed"):
            qvm.Plan(gates, n, dtype, k_max=3, tile_qubits=c)


def test_python_layer_names():
    """Circuit, plan(..., planner=...) and AdjointExpectation, the names the
    Python layer offers over the C calls (host side: no GPU needed)."""
    c = qvm.Circuit(5)
    c.add(Gate("h", (0,))).add(Gate("x", (1,), (0,))).add(Gate("rz", (4,), (), (0.3,)))
    assert len(c) == 3 and c.array().n == 3
    with pytest.raises(ValueError):
        c.add(Gate("h", (5,)))
    p = qvm.plan(c, planner="greedy", k_max=3, tile_qubits=5)
    assert p.stats()["passes"] >= 1
    with pytest.raises(ValueError):
        qvm.plan(c, planner="dynamic")
    with pytest.raises(ValueError):
        qvm.plan(list(c), planner="greedy")
    adj = pytest.importorskip("paper_2212_14201_amd.adjoint")
    assert qvm.AdjointExpectation is adj._function()
