"""Host-side checks of the fusion planner: plan validity and block matrices.

Block matrices built by the library (FP64) are compared with the oracle's
block construction over the same gates and qubits; the execution order the
plan reports is checked with the oracle's plan validator.
"""
import numpy as np
import pytest

import oracle
from tests.util import (_DSUB, _DTERM, _ETERM, _PREC, _TOP, blocks_and_diagonals, long_phase_run, plan_image,
                        tile_blocks_outer_diagonals)
from workloads import (Gate, config_circuit, layered_u3_cz, qft_circuit, qft_then_brick,
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


def check_plan(gates, n, k_max, tile, dtype="c64", relabeled_swaps=None, defer_narrow=False):
    plan = qvm.Plan(gates, n, dtype, k_max=k_max, tile_qubits=tile, defer_narrow=defer_narrow)
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


@pytest.mark.parametrize("n,k_max,tile", [(10, 3, 8), (10, 4, 8), (12, 3, 9), (14, 3, 10), (14, 4, 10)])
def test_defer_narrow_plans_valid(n, k_max, tile):
    """Tile passes that leave narrow trailing blocks to a later pass: the
    plans stay valid (per-wire order, block matrices) on random circuits
    and on the QFT followed by a brick."""
    gates = random_mixed_circuit(n, 200, 700 + n + k_max, kmax=3, max_ctrl=max(0, k_max - 3))
    check_plan(gates, n, k_max, tile, defer_narrow=True)
    _, gates = qft_then_brick(n, 12, 600 + n)
    check_plan(gates, n, k_max, tile, defer_narrow=True)
    with pytest.raises(ValueError):
        qvm.Plan(gates, n, "c64", tile_qubits=tile, k_of_pass=[3], defer_narrow=True)


def test_defer_narrow_on_the_30_qubit_workload():
    """On the 30-qubit workload (QFT + 30 brick layers, 3-qubit blocks in
    13-qubit tiles) every narrow block but those of the last pass is left
    to a later pass, where it joins a 3-qubit block: 229 -> 220 blocks and
    18 -> 17 passes."""
    cfg = config_circuit("qft30")
    base = qvm.Plan(cfg["gates"], 30, "c64", k_max=3, tile_qubits=13, image=False)
    plan = qvm.Plan(cfg["gates"], 30, "c64", k_max=3, tile_qubits=13, defer_narrow=True)
    sb, sd = base.stats(), plan.stats()
    assert sb["blocks_by_k"][1] + sb["blocks_by_k"][2] > 0
    last = sd["passes"] - 1
    for b in range(sd["blocks"]):
        blk = plan.block(b)
        assert blk["k_true"] == 3 or blk["pass"] == last
    assert sd["blocks"] < sb["blocks"] and sd["passes"] <= sb["passes"]


@pytest.mark.parametrize("count,epilogue", [(200, True), (1100, False)])
def test_phase_sums_bounded(count, epilogue):
    """A phase run rides in the block epilogue only while the pass's phase
    sums stay within their LDS area (kPSumMax = 1024 combos, bounded before
    the layout is fixed); a longer run is applied on its own.  Both plans are
    valid (oracle validator, block matrices; tests/test_gpu_fused.py runs
    them against the oracle's state)."""
    n = 13
    gates = long_phase_run(n, count, 5100 + count)
    plan, _ = check_plan(gates, n, 3, 13)
    rec, passes = plan_image(plan)
    assert len(passes) == 1 and 0 <= int(passes[0]["npsum"]) <= 1024
    ops = rec(int(passes[0]["ops"]), _TOP, int(passes[0]["nops"]))
    runs = [op for op in ops if op["type"] == 2]
    assert runs and any(op["flags"] & 4 for op in runs) == epilogue
    assert (int(passes[0]["psum"]) != 0) == epilogue


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
    st = L.qvm_plan_greedy_ex(ga.ptr(), ga.n, 3, 3, 0, qvm.QVM_C64, 4, qvm.ctypes.byref(h))
    assert qvm.STATUS[st] == "QVM_EARG" and not h.value
    ks = np.array([3], np.int32)
    st = L.qvm_plan_tile_per_pass(ga.ptr(), ga.n, 3, 3, ks.ctypes.data_as(qvm._i32p), 1, qvm.QVM_C64,
                                  qvm.QVM_PLAN_DEFER_NARROW, qvm.ctypes.byref(h))
    assert qvm.STATUS[st] == "QVM_EARG" and not h.value


def run_angles(terms, off, t, nhb, wmask):
    """Angle-path sums: per element code i and thread code t, the total of
    every term group whose element-bit set is contained in i (terms whose
    outer-bit test holds for the tile: the caller passes only those)."""
    assert off[-1] == len(terms) and np.all(np.diff(off.astype(np.int64)) >= 0)
    acc = np.zeros((1 << nhb, len(t)), np.uint64)
    for g in range(1 << nhb):
        for d in terms[off[g]: off[g + 1]]:
            assert d["lmask"] < 512 and d["lval"] & ~d["lmask"] == 0
            hit = (t & np.uint64(d["lmask"])) == np.uint64(d["lval"])
            acc[g] = (acc[g] + np.where(hit, d["turns"], np.uint64(0))) & wmask
    for b in range(nhb):
        for i in range(1 << nhb):
            if (i >> b) & 1:
                acc[i] = (acc[i] + acc[i ^ (1 << b)]) & wmask
    return acc


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
            ang = run_angles(terms, off, t, nhb, wmask).reshape(-1)   # element t + 512 i at i * len(t) + t
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


_SWZ_IMG = (3, 5, 6, 9, 10, 12, 7, 11, 13)     # low-bit images of tile bits 4..12


def _swz(e):
    """The tile kernel's LDS swizzle (an involution: it is its own inverse)."""
    e = np.asarray(e, dtype=np.int64)
    x = np.zeros_like(e)
    for j, v in enumerate(_SWZ_IMG):
        x ^= np.where((e >> (4 + j)) & 1, v, 0)
    return e ^ x


def test_swizzle_is_a_linear_involution_and_spreads_banks():
    """The LDS slot map: an involution on every tile size, linear over
    GF(2), element pairs (2m, 2m + 1) on adjacent slots; and the column bits
    the planner gives the lanes of the 30-qubit workload's blocks put every
    16-lane column walk of complex64 on distinct LDS bank pairs (slot bits
    0..3) whenever the free bits allow it (they do for every block there)."""
    for L in range(3, 14):
        e = np.arange(1 << L)
        s = _swz(e)
        assert np.array_equal(np.sort(s), e) and np.array_equal(_swz(s), e)
        a, b = e[:, None], e[None, ::97]
        assert np.array_equal(_swz(a ^ b), _swz(a) ^ _swz(b))
        assert np.all((s[0::2] ^ s[1::2]) == 1)
    cfg = config_circuit("qft30")
    plan = qvm.Plan(cfg["gates"], 30, "c64", k_max=3, tile_qubits=13)
    rec, passes = plan_image(plan)
    nblk = 0
    for pd in passes:
        L = int(pd["L"])
        for op in rec(int(pd["ops"]), _TOP, int(pd["nops"])):
            if op["type"] != 1:
                continue
            k = int(op["k"])
            ntile, K = ((1 << (L - k)) + 15) >> 4, 2 << k
            off = ntile + K // 8 + 4 * (K // 16)
            lanew = rec(int(op["tab"]), np.dtype("<u4"), off + 4)[off:]
            slots = [0]
            for w in lanew:
                slots = slots + [x ^ (int(w) // 8) for x in slots]
            assert len({x & 15 for x in slots}) == 16, (k, lanew)
            nblk += 1
    assert nblk == plan.stats()["blocks"]


def _block_ct(k, L, c128):
    K = 2 << k
    RB = K // 16
    ct0 = 1 if RB >= 4 else (4 // RB if c128 else (8 if K == 16 else 4))
    ntile = ((1 << max(L - k, 0)) + 15) >> 4
    share = ntile // 8
    return ct0 if ct0 < share else (share if share >= 1 else 1)


def block_layout(rec, op, L, dtype):
    """Emulates how the tile kernel's block op forms its LDS addresses from
    the op's address table (col, brow, erow, lane words).  Lanes l, l + 16,
    l + 32, l + 48 of a wave share a column (l % 16) of each column tile the
    wave takes; each lane reads its share of the column's complex input rows
    and writes its share of the output rows.  Returns (inputs, outputs,
    wave, epi): inputs[col, row] / outputs[col, row] are the tile elements
    the column's row is read from / written to, wave[col] its wave, and epi
    the complex64 epilogue's outputs as rows (thread code, element code
    hh | ct << 1 | rb << (1 + log2 CT), tile element)."""
    k = int(op["k"])
    lb = [int(v) for v in op["lb"][:k]]
    c128 = dtype == "c128"
    es = 16 if c128 else 8
    K = 2 << k
    RB, KS = K // 16, K // 4
    ncol = 1 << (L - k)
    ntile = (ncol + 15) >> 4
    nb, ne = K // 8, 4 * RB
    CT = _block_ct(k, L, c128)
    LCT = CT.bit_length() - 1
    tab = rec(int(op["tab"]), np.dtype("<u4"), ntile + nb + ne + 4).astype(np.int64)
    col, brow, erow, lanew = tab[:ntile], tab[ntile:ntile + nb], tab[ntile + nb:ntile + nb + ne], tab[-4:]
    scat = lambda j: sum(((j >> q) & 1) << lb[q] for q in range(k))
    el = lambda slot: _swz(slot // es)
    # column items (wave, column tile, lane column), in the kernel's order
    w_, ti_, c_ = [], [], []
    for w in range(8):
        t0 = w * CT
        while t0 < ntile:
            for ct in range(CT):
                if t0 + ct < ntile:
                    for c16 in range(16):
                        if (t0 + ct) * 16 + c16 < ncol:
                            w_.append(w)
                            ti_.append(t0 + ct)
                            c_.append(c16)
            t0 += 8 * CT
    w_, ti_, c_ = np.array(w_), np.array(ti_), np.array(c_)
    ct_ = ti_ % CT
    swl = np.zeros(len(c_), np.int64)
    for i in range(4):
        swl ^= np.where((c_ >> i) & 1, lanew[i], 0)
    swe = swl ^ col[ti_]
    ins = np.full((len(c_), 1 << k), -1, np.int64)
    outs = np.full((len(c_), 1 << k), -1, np.int64)
    epi = []
    for g in range(4):
        swg = es * int(_swz(scat(g)))
        for t in range(KS // 2):
            ins[:, 4 * t + g] = el(swe ^ brow[t] ^ swg)
        if not c128:
            swo = es * int(_swz(scat(2 * g)))
            for rb in range(RB):
                for hh in range(2):
                    e = el(swe ^ swo ^ erow[4 * rb + hh])
                    outs[:, 8 * rb + 2 * g + hh] = e
                    epi.append(np.stack([w_ * 64 + 16 * g + c_, hh | ct_ << 1 | rb << (1 + LCT), e], 1))
        else:
            swo = es * int(_swz(scat(g >> 1)))
            for rb in range(RB):
                for r in range(4):
                    row = 8 * rb + 2 * r + (g >> 1)
                    e = el(swe ^ swo ^ erow[4 * rb + r])
                    assert np.all((outs[:, row] == -1) | (outs[:, row] == e))   # re, im from lanes g, g ^ 1
                    outs[:, row] = e
    epi = np.concatenate(epi) if epi else np.zeros((0, 3), np.int64)
    return ins, outs, w_, epi


def check_block_layouts(plan, dtype):
    """Every block op of every pass: each item reads and writes the same
    tile elements, row r of its column on the block's bit lb[r]; the items
    cover every tile element exactly once; and a block marked BLK_NOSYNC
    gives every wave exactly the elements it had in the block before (so no
    workgroup barrier is needed between them).  Returns the number of
    blocks and of BLK_NOSYNC blocks."""
    rec, passes = plan_image(plan)
    nblk = nsync = 0
    for pd in passes:
        L = int(pd["L"])
        prev = None
        for op in rec(int(pd["ops"]), _TOP, int(pd["nops"])):
            if op["type"] != 1:
                if not op["flags"] & 4:
                    prev = None
                continue
            nblk += 1
            k = int(op["k"])
            lb = [int(v) for v in op["lb"][:k]]
            ins, outs, waves, _ = block_layout(rec, op, L, dtype)
            assert np.array_equal(ins, outs) and np.all(ins >= 0)
            cols = ins
            rowbits = np.array([sum(((j >> q) & 1) << lb[q] for q in range(k)) for j in range(1 << k)])
            assert np.all((cols ^ cols[:, :1]) == rowbits[None, :])       # row r on the block's bits
            assert np.array_equal(np.sort(cols.reshape(-1)), np.arange(1 << L))
            owned = [frozenset(ins[waves == w].reshape(-1).tolist()) for w in range(8)]
            if op["flags"] & 2:
                nsync += 1
                assert prev is not None and owned == prev, "BLK_NOSYNC block changes the waves' elements"
            prev = owned
    return nblk, nsync


@pytest.mark.parametrize("k_max,tile,dtype", [(3, 13, "c64"), (4, 13, "c64"), (3, 12, "c64"), (4, 11, "c64"),
                                              (3, 12, "c128"), (4, 12, "c128")])
def test_block_layouts_and_wave_ownership(k_max, tile, dtype):
    """The block ops' address tables of the 30-qubit workload's plans (and
    of a random circuit): full coverage and the wave ownership that lets
    consecutive blocks skip the workgroup barrier; most blocks of the
    register-fragment passes do skip it."""
    cfg = config_circuit("qft30")
    plan = qvm.Plan(cfg["gates"], 30, dtype, k_max=k_max, tile_qubits=tile)
    nblk, nsync = check_block_layouts(plan, dtype)
    assert nsync >= nblk // 3, (nblk, nsync)
    n, gates = random_planner_circuit(31, n_range=(26, 26), g_range=(300, 300))
    check_block_layouts(qvm.Plan(gates, n, dtype, k_max=k_max, tile_qubits=tile), dtype)


def deposit(w, qmask):
    """Tile index w with a zero inserted at every tile bit (set bit of
    qmask): the tile's base physical index."""
    out, j = 0, 0
    for p in range(64):
        if (qmask >> p) & 1:
            continue
        out |= ((w >> j) & 1) << p
        j += 1
        if w >> j == 0:
            break
    return out


def epilogue_sign_factors(terms, off, w):
    """Factors of a sign run applied in a block's epilogue, per (element
    code, thread code), for tile index w: records matched on the tile index
    and the thread, parities over the element codes each record lists."""
    t = np.arange(512, dtype=np.int64)
    assert off[-1] == len(terms) and np.all(np.diff(off.astype(np.int64)) % 2 == 0)
    m = np.zeros(512, np.int64)
    for d in terms:
        hit = ((w & int(d["om"])) == int(d["ov"])) & ((t & int(d["lm"])) == int(d["lv"]))
        m ^= np.where(hit, int(d["w"]), 0)
    flips = (m[None, :] >> np.arange(16)[:, None]) & 1
    return np.where(flips == 1, -1.0, 1.0)


def psum_table(rec, off):
    """The pass's phase sums (layout in csrc/tile.hpp): per combo its
    records and its lane mask per wave."""
    ncombo, nrec, rec_off, mask_off = (int(v) for v in rec(off, np.dtype("<u4"), 4))
    cb = rec(off + 16, np.dtype("<u4"), ncombo + 1).astype(np.int64)
    recs = rec(off + rec_off, _PREC, nrec)
    masks = rec(off + mask_off, np.dtype("<u8"), 8 * ncombo).reshape(8, ncombo)
    assert ncombo % 4 == 0 and cb[0] == 0 and cb[-1] == nrec and np.all(np.diff(cb) >= 0)
    return cb, recs, masks


def epilogue_phase_factors(rec, op, w):
    """Factors of a phase run applied in a block's epilogue, per (element
    code, thread code), for tile index w: each combo's sum of the records
    whose tile-index test holds, added where the thread's bit of its wave's
    lane mask is set, per group; then subset sums over the element-code
    bits."""
    cb, recs, masks = psum_table(rec, int(op["data"]))
    goff = rec(int(op["tab"]), np.dtype("<u4"), 17).astype(np.int64)
    assert np.all(np.diff(goff) % 4 == 0)
    t = np.arange(512, dtype=np.uint64)
    acc = np.zeros((16, 512), np.uint64)
    for g in range(16):
        for c in range(goff[g], goff[g + 1]):
            s = 0
            for r in recs[cb[c]: cb[c + 1]]:
                s += int(r["w"]) if (w & int(r["om"])) == int(r["ov"]) else 0
            on = (masks[t >> np.uint64(6), c] >> (t & np.uint64(63))) & np.uint64(1)
            acc[g] = (acc[g] + on * np.uint64(s & 0xFFFFFFFF)) & np.uint64(0xFFFFFFFF)
    for b in range(4):
        for i in range(16):
            if (i >> b) & 1:
                acc[i] = (acc[i] + acc[i ^ (1 << b)]) & np.uint64(0xFFFFFFFF)
    return np.exp(2j * np.pi * (acc.astype(np.float64) / 2.0 ** 32))


@pytest.mark.parametrize("n,k_max,signs", [(13, 3, False), (13, 4, False), (15, 3, False), (15, 4, False),
                                           (15, 3, True), (15, 4, True)])
def test_epilogue_runs_reproduce_the_circuit(n, k_max, signs):
    """Pins the encoding of diagonal runs that a complex64 block applies to
    its outputs (13-qubit tiles; with 15 qubits the runs' gates also act on
    the two qubits outside the tile, so their terms test the tile index):
    emulating the single pass tile by tile and op by op from the plan image
    (blocks through their address tables and matrices, runs from their
    records over the block epilogue's layout or the standalone layout)
    gives the oracle's state of the whole circuit."""
    L = 13
    seed = 4100 + 10 * n + k_max + 100 * signs
    rng = np.random.Generator(np.random.PCG64(seed))
    gates = (blocks_and_diagonals(n, seed, signs_only=signs) if n == L
             else tile_blocks_outer_diagonals(L, n, seed, signs_only=signs))
    plan = qvm.Plan(gates, n, "c64", k_max=k_max, tile_qubits=L)
    rec, passes = plan_image(plan)
    assert len(passes) == 1 and passes[0]["remap"] == 0 and passes[0]["L"] == L
    pd = passes[0]
    c, qmask = int(pd["c"]), int(pd["qmask"])
    ldoff = rec(int(pd["ldoff"]), np.dtype("<u8"), 1 << (L - c))
    e = np.arange(1 << L, dtype=np.uint64)
    local = ((e & np.uint64((1 << c) - 1)) | ldoff[(e >> np.uint64(c)).astype(np.int64)]).astype(np.int64)
    psi0 = rng.standard_normal(1 << n) + 1j * rng.standard_normal(1 << n)
    psi0 /= np.linalg.norm(psi0)
    got = np.zeros(1 << n, np.complex128)
    ops = rec(int(pd["ops"]), _TOP, int(pd["nops"]))
    n_epi = n_sign = 0
    for w in range(1 << (n - L)):
        base = deposit(w, qmask)
        phys = base | local
        tile = psi0[phys].copy()
        nb, prev = 0, None
        for op in ops:
            if op["type"] == 1:
                blk = plan.block(nb)
                nb += 1
                assert blk["k"] == op["k"]
                ins, outs, _, epi_map = block_layout(rec, op, L, "c64")
                x = tile[ins]                           # columns of the block's input
                tile[outs] = x @ np.asarray(blk["matrix"]).T
                prev = (op, epi_map)
                continue
            if op["flags"] & 4:
                # applied in the preceding block's epilogue
                assert prev is not None and prev[0]["flags"] & 1
                if op["flags"] & 2:
                    off = rec(int(op["tab"]), np.dtype("<u4"), 17)
                    f = epilogue_sign_factors(rec(int(op["data"]), _ETERM, int(off[-1])), off, w)
                else:
                    assert int(op["data"]) == int(pd["psum"]) and pd["npsum"] > 0
                    f = epilogue_phase_factors(rec, op, w)
                n_epi += w == 0
                n_sign += w == 0 and bool(op["flags"] & 2)
                epi_map = prev[1]
                where = np.full((16, 512), -1, np.int64)
                where[epi_map[:, 1], epi_map[:, 0]] = epi_map[:, 2]
                fac = np.zeros(1 << L, np.complex128)
                fac[where.reshape(-1)] = f.reshape(-1)
                assert np.all(fac != 0)           # every element gets exactly one factor
                tile *= fac
            elif op["flags"] & 1:
                terms = rec(int(op["data"]), _DTERM, int(op["k"]))
                off = rec(int(op["tab"]), np.dtype("<u4"), 17)
                t = np.arange(512, dtype=np.uint64)
                live = terms[(np.uint64(base) & terms["omask"]) == terms["oval"]]
                # the standalone layout: element t + 512 i
                offs = np.searchsorted(np.flatnonzero((np.uint64(base) & terms["omask"]) == terms["oval"]), off)
                ang = run_angles(live, offs.astype(np.uint32), t, 4, np.uint64(0xFFFFFFFF)).reshape(-1)
                f = (np.where(ang >> np.uint64(31), -1.0, 1.0) if op["flags"] & 2
                     else np.exp(2j * np.pi * (ang.astype(np.float64) / 2.0 ** 32)))
                tile *= f
            else:
                for d in rec(int(op["data"]), _DSUB, int(op["k"])):
                    hit = ((e & np.uint64(d["lmask"])) == np.uint64(d["lval"])) & \
                        ((base & int(d["omask"])) == int(d["oval"]))
                    f = -1.0 if d["neg"] else d["pr"] + 1j * d["pi"]
                    tile = np.where(hit, tile * f, tile)
            prev = None
        assert nb == plan.stats()["blocks"]
        got[phys] = tile
    assert n_epi >= 1 and (n_sign >= 1 or not signs)
    want = oracle.apply_gates(psi0.copy(), n, gates)
    assert np.max(np.abs(got - want)) < 1e-7


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


def pass_gate_sets(plan, ngates):
    """The gates of each pass: execution positions are consecutive within a
    pass, and each pass's gate count is its pass feature 10."""
    from paper_2212_14201_amd import learned_planner
    counts = learned_planner.plan_features(plan)[:, 10].astype(int)
    pos, unit = plan.schedule()
    order = [i for i in np.argsort(pos, kind="stable") if pos[i] >= 0]
    out, o = [], 0
    for c in counts:
        out.append(frozenset(order[o:o + c]))
        o += c
    assert o == len(order)
    return out


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_per_pass_block_widths(seed):
    """Tile passes take the same gates whatever the block width, so a plan
    with a width per pass has pass i of every fixed-width plan; it is valid,
    its blocks respect each pass's width, and with one width throughout it
    is the fixed-width plan."""
    n, gates = random_planner_circuit(7000 + seed, n_range=(14, 16), g_range=(150, 250))
    ga = qvm.GateArray(gates)
    fixed = {k: qvm.Plan(ga, n, "c64", k_max=k, tile_qubits=11) for k in (3, 4, 5)}
    sets = {k: pass_gate_sets(p, len(gates)) for k, p in fixed.items()}
    assert sets[3] == sets[4] == sets[5]
    npass = fixed[3].stats()["passes"]
    rng = np.random.default_rng(seed)
    ks = rng.integers(3, 6, npass).astype(np.int32)
    plan = qvm.Plan(ga, n, "c64", tile_qubits=11, k_of_pass=ks)
    assert pass_gate_sets(plan, len(gates)) == sets[3]
    units = units_in_order(plan, len(gates))
    wg = on_wires(gates)
    kept = sorted(wg)
    remap = {g: j for j, g in enumerate(kept)}
    ok, why = oracle.validate_plan([wg[i] for i in kept], [[remap[i] for i in u] for u in units], n)
    assert ok, why
    for b in range(plan.stats()["blocks"]):
        blk = plan.block(b)
        assert blk["k_true"] <= ks[blk["pass"]]
        want = oracle.block_matrix([wg[i] for i in blk["gates"]], blk["qubits"])
        assert np.max(np.abs(blk["matrix"] - want)) < 1e-13
    for k in (3, 4, 5):
        same = qvm.Plan(ga, n, "c64", tile_qubits=11, k_of_pass=[k])
        assert same.stats() == fixed[k].stats()
    with pytest.raises(qvm.QvmError):
        qvm.Plan(ga, n, "c64", tile_qubits=0, k_of_pass=[3])
    with pytest.raises(qvm.QvmError):
        qvm.Plan(ga, n, "c128", tile_qubits=12, k_of_pass=[3, 6])
