"""The peephole pre-pass (qvm_simplify) on the host: crafted cases with the
outcome fixed by the rules, and random circuits whose simplified form must
give the same state as the original under the FP64 oracle."""
import math

import numpy as np
import pytest

import oracle
from workloads import Gate

qvm = pytest.importorskip("paper_2212_14201_amd.qvm")

NAME = {v: k for k, v in qvm.KIND.items() if k not in ("matrix",)}


def as_gates(ga):
    """Gate objects back from packed records (matrices read through u)."""
    out = []
    for i in range(ga.n):
        r = ga.arr[i]
        k = int(r.k)
        targets = tuple(int(r.targets[j]) for j in range(k))
        controls = tuple(q for q in range(64) if (int(r.ctrl_mask) >> q) & 1)
        name = NAME[int(r.kind)]
        if name == "unitary":
            d = 1 << k
            m = np.ctypeslib.as_array(r.u, shape=(2 * d * d,)).copy().view(np.complex128).reshape(d, d)
            out.append(Gate("unitary", targets, controls, (), -1, m))
        else:
            out.append(Gate(name, targets, controls, tuple(float(r.params[j]) for j in range(3))))
    return out


def simp(gates, n=4):
    return as_gates(qvm.simplify(gates, n))


def names(gates):
    return [(g.name, g.targets, g.controls) for g in gates]


def test_identity_pairs_and_blocking():
    assert simp([Gate("h", (0,)), Gate("h", (0,))]) == []
    assert names(simp([Gate("h", (0,)), Gate("x", (1,)), Gate("h", (0,))])) == [("x", (1,), ())]
    kept = simp([Gate("h", (0,)), Gate("x", (1,), (0,)), Gate("h", (0,))])
    assert len(kept) == 3                         # the CNOT touches qubit 0
    assert simp([Gate("x", (0,), (1,)), Gate("x", (0,), (1,))]) == []
    assert len(simp([Gate("x", (0,), (1,)), Gate("x", (0,), (2,))])) == 2
    assert simp([Gate("swap", (0, 1)), Gate("swap", (1, 0))]) == []
    assert simp([Gate("i", (2,))]) == []
    # cascade: the inner pair cancels, then the outer one
    assert simp([Gate("x", (0,)), Gate("h", (0,)), Gate("h", (0,)), Gate("x", (0,))]) == []


def test_phase_combinations():
    assert names(simp([Gate("t", (1,)), Gate("t", (1,))])) == [("s", (1,), ())]
    assert names(simp([Gate("t", (1,))] * 4)) == [("z", (1,), ())]
    assert simp([Gate("t", (1,))] * 8) == []
    assert simp([Gate("s", (1,)), Gate("sdg", (1,))]) == []
    assert simp([Gate("t", (1,)), Gate("t", (1,)), Gate("sdg", (1,))]) == []
    assert names(simp([Gate("h", (0,)), Gate("s", (0,)), Gate("s", (0,)), Gate("h", (0,))])) == \
        [("h", (0,), ()), ("z", (0,), ()), ("h", (0,), ())]


def test_rotation_merges():
    out = simp([Gate("rz", (2,), (), (0.3,)), Gate("rz", (2,), (), (0.5,)), Gate("rz", (2,), (), (-0.1,))])
    assert names(out) == [("rz", (2,), ())] and math.isclose(out[0].params[0], 0.7, abs_tol=1e-15)
    assert simp([Gate("rx", (0,), (), (0.4,)), Gate("rx", (0,), (), (-0.4,))]) == []
    out = simp([Gate("rzz", (0, 1), (), (0.2,)), Gate("rzz", (1, 0), (), (0.3,))])
    assert len(out) == 1 and math.isclose(out[0].params[0], 0.5, abs_tol=1e-15)
    # different axes, or different controls, stay apart
    assert len(simp([Gate("rx", (0,), (), (0.2,)), Gate("ry", (0,), (), (0.2,))])) == 2
    assert len(simp([Gate("p", (0,), (1,), (0.2,)), Gate("p", (0,), (), (0.2,))])) == 2
    out = simp([Gate("p", (0,), (1,), (0.2,)), Gate("p", (0,), (1,), (0.25,))])
    assert len(out) == 1 and out[0].controls == (1,)


def test_matrix_gates_pass_through():
    u = np.array([[0, 1], [1, 0]], dtype=complex)
    out = simp([Gate("unitary", (0,), (), (), -1, u), Gate("h", (1,)), Gate("h", (1,))])
    assert len(out) == 1 and np.array_equal(out[0].matrix, u)


def redundant_circuit(n, count, seed):
    """Random gates from a small set on few qubits, so that pairs and runs
    of mergeable gates are frequent."""
    rng = np.random.Generator(np.random.PCG64(seed))
    one = ["h", "x", "y", "z", "s", "sdg", "t", "tdg", "rx", "ry", "rz", "p", "i"]
    gates = []
    for _ in range(count):
        r = rng.random()
        q = int(rng.integers(0, n))
        if r < 0.7:
            name = one[int(rng.integers(0, len(one)))]
            par = (float(rng.choice([0.25, -0.25, 1.1, -1.1, 0.5])),) if name in ("rx", "ry", "rz", "p") else ()
            ctrl = () if rng.random() < 0.7 else (int((q + 1 + rng.integers(0, n - 1)) % n),)
            gates.append(Gate(name, (q,), ctrl, par))
        elif r < 0.85:
            a, b = (int(v) for v in rng.choice(n, 2, replace=False))
            gates.append(Gate("x", (a,), (b,)) if rng.random() < 0.5 else Gate("swap", (a, b)))
        else:
            a, b = (int(v) for v in rng.choice(n, 2, replace=False))
            gates.append(Gate("rzz", (a, b), (), (float(rng.choice([0.3, -0.3, 0.7])),)))
    return gates


@pytest.mark.parametrize("seed", range(6))
def test_simplified_circuit_keeps_the_state(seed):
    n = 3 + seed % 4
    gates = redundant_circuit(n, 200, 4100 + seed)
    out = simp(gates, n)
    assert len(out) < len(gates)
    x = (7 * seed) % (1 << n)
    a = oracle.simulate(n, gates, init=x)
    b = oracle.simulate(n, out, init=x)
    assert np.max(np.abs(a - b)) < 1e-12


def test_invalid_gate_rejected():
    with pytest.raises(qvm.QvmError):
        qvm.simplify([Gate("h", (5,))], 3)
