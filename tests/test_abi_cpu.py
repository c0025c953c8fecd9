"""Host-side checks of the C ABI: exports, lowering, validation.

No call here reaches the GPU: argument errors are returned before anything
is enqueued, and gate lowering runs on the host.
"""
import ctypes
import os

import numpy as np
import pytest

import oracle
from tests.util import header_functions
from workloads import Gate, random_mixed_circuit

qvm = pytest.importorskip("paper_2212_14201_amd.qvm")


def test_every_declared_symbol_is_exported():
    L = qvm.lib()
    names = header_functions()
    assert len(names) >= 19
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing


def test_struct_layout():
    assert ctypes.sizeof(qvm.QvmGate) == 72
    assert qvm.QvmGate.ctrl_mask.offset == 32
    assert qvm.QvmGate.u.offset == 64


@pytest.mark.parametrize("name,nt,np_", [("h", 1, 0), ("x", 1, 0), ("y", 1, 0), ("z", 1, 0),
                                        ("s", 1, 0), ("sdg", 1, 0), ("t", 1, 0), ("tdg", 1, 0),
                                        ("rx", 1, 1), ("ry", 1, 1), ("rz", 1, 1), ("p", 1, 1),
                                        ("u3", 1, 3), ("rzz", 2, 1), ("swap", 2, 0)])
def test_lowering_matches_oracle(name, nt, np_):
    rng = np.random.default_rng(hash(name) % 1000)
    for _ in range(5):
        g = Gate(name, tuple(range(nt)), (), tuple(rng.uniform(-7, 7, np_)))
        a = qvm.gate_matrix(g)
        b = oracle.gate_matrix(g)
        assert np.max(np.abs(a - b)) <= 4e-16


def test_lowering_explicit_matrix_passthrough():
    for g in random_mixed_circuit(4, 30, 1, names=["unitary"]):
        assert np.array_equal(qvm.gate_matrix(g), g.matrix)


def _status(fn, *args):
    return fn(*args)


def test_lowering_rejects_bad_gates():
    with pytest.raises(qvm.QvmError) as e:
        qvm.gate_matrix(Gate("rzz", (0,), (), (1.0,)))
    assert e.value.status == -1
    with pytest.raises(qvm.QvmError):
        qvm.gate_matrix(Gate("h", (0, 0)))


def test_workspace_bytes():
    assert qvm.workspace_bytes(0, "c64") == 0
    assert qvm.workspace_bytes(35, "c64") == 0
    for n in (1, 12, 30, 34):
        assert qvm.workspace_bytes(n, "c128") > 0


class FakeSV:
    """A handle bound to aligned dummy addresses: valid for host-side
    validation only (never used to launch)."""

    def __init__(self, n=5, dt=2):
        self.h = ctypes.c_void_p()
        wb = qvm.lib().qvm_workspace_bytes(n, dt)
        st = qvm.lib().qvm_sv_create(n, dt, 1 << 20, 1 << 21, wb, None, ctypes.byref(self.h))
        assert st == 0

    def __del__(self):
        qvm.lib().qvm_sv_destroy(self.h)


def test_create_validation():
    L = qvm.lib()
    h = ctypes.c_void_p()
    assert L.qvm_sv_create(0, 2, 256, 256, 1 << 30, None, ctypes.byref(h)) == -1
    assert L.qvm_sv_create(35, 2, 256, 256, 1 << 30, None, ctypes.byref(h)) == -1
    assert L.qvm_sv_create(5, 3, 256, 256, 1 << 30, None, ctypes.byref(h)) == -1
    assert L.qvm_sv_create(5, 2, None, 256, 1 << 30, None, ctypes.byref(h)) == -1
    assert L.qvm_sv_create(5, 2, 264, 256, 1 << 30, None, ctypes.byref(h)) == -1   # misaligned
    assert L.qvm_sv_create(5, 2, 256, 256, 16, None, ctypes.byref(h)) == -3        # workspace
    assert L.qvm_sv_destroy(None) == 0


def test_apply_validation_before_enqueue():
    L = qvm.lib()
    sv = FakeSV(5)

    def st(g):
        ga = qvm.GateArray([g])
        return L.qvm_apply(sv.h, ga.ptr())

    assert st(Gate("h", (5,))) == -2                     # qubit >= n
    assert st(Gate("x", (1,), (1,))) == -1               # control overlaps target
    assert st(Gate("x", (1,), (7,))) == -2               # control >= n
    assert st(Gate("swap", (2, 2))) == -1                # duplicate target
    m = np.eye(16, dtype=complex)
    assert st(Gate("unitary", (0, 1, 2, 3), (), (), -1, m)) == -6   # k > 3 plain
    assert "k <= 3" in L.qvm_last_error().decode()
    # a bad gate anywhere in a list fails the whole list before any launch
    ga = qvm.GateArray([Gate("h", (0,)), Gate("h", (9,))])
    assert L.qvm_run(sv.h, ga.ptr(), 2) == -2
    assert b"gate 1" in L.qvm_last_error()
    assert L.qvm_init_basis(sv.h, 32) == -2
    assert L.qvm_apply(None, ga.ptr()) == -1


def test_readout_validation():
    L = qvm.lib()
    sv = FakeSV(6)
    out = np.zeros(64)
    dp = out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    q = np.array([1, 1], np.int32)
    assert L.qvm_probabilities(sv.h, 2, q.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), dp) == -1
    q = np.array([1, 6], np.int32)
    assert L.qvm_probabilities(sv.h, 2, q.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), dp) == -2
    assert L.qvm_probabilities(sv.h, 3, None, dp) == -1
    u = np.array([0.5, 1.0])
    o = np.zeros(2, np.uint64)
    assert L.qvm_sample(sv.h, 2, u.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                        o.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))) == -2
    xs = np.array([1 << 6], np.uint64)
    zs = np.array([0], np.uint64)
    assert L.qvm_expect_pauli(sv.h, 1, xs.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)),
                              zs.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)), None,
                              dp, None) == -2
    assert L.qvm_copy_amplitudes(sv.h, 60, 5, dp) == -2


def test_one_hip_runtime_in_process():
    """The binding loads torch before the library, so exactly one HIP runtime
    (torch's) is mapped: torch's device memory and streams are then valid
    handles inside the library."""
    import re
    import subprocess
    import sys
    code = ("import sys, re; sys.path.insert(0, %r)\n"
            "from paper_2212_14201_amd import qvm\n"
            "from workloads import Gate\n"
            "qvm.Plan([Gate('h', (0,))], 3, 'c64', k_max=3)\n"   # first library call, before any torch use
            "print(sorted(set(re.findall(r'\\S*libamdhip64\\S*', open('/proc/self/maps').read()))))"
            % os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    out = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=300)
    assert out.returncode == 0, out.stderr
    libs = eval(out.stdout.strip().splitlines()[-1])
    assert len(libs) == 1, libs


def test_adjoint_group_count_host_only():
    """qvm_adjoint_group_count (host-only): gates on one target form one
    group; the 20-qubit ansatz needs at least five groups (20 targets, at
    most four per complex64 group, three per complex128 one) and at most one
    per gate; invalid gates are rejected."""
    adj = pytest.importorskip("paper_2212_14201_amd.adjoint")
    from workloads import hardware_efficient_ansatz
    from paper_2212_14201_amd.qvm import GateArray, _dt, _gp, _i32p
    import ctypes

    def count(n, gates, n_params, dtype="c64"):
        L = adj._declare()
        ga = GateArray(gates)
        pidx = np.ascontiguousarray([getattr(g, "pidx", -1) for g in gates], dtype=np.int32)
        out = ctypes.c_int32()
        st = L.qvm_adjoint_group_count(n, _dt(dtype), ga.ptr(), ga.n, pidx.ctypes.data_as(_i32p), n_params,
                                       ctypes.byref(out))
        return st, out.value

    one = [Gate("ry", (3,), (), (0.0,), pidx=i) for i in range(10)]
    assert count(6, one, 10) == (0, 1)
    gates, P = hardware_efficient_ansatz(20, 16)
    st, g64 = count(20, gates, P)
    st2, g128 = count(20, gates, P, "c128")
    assert st == 0 and st2 == 0
    assert 5 <= g64 <= len(gates) and g64 <= g128 <= len(gates)   # 20 targets, at most 4 per group
    bad = [Gate("h", (25,))]
    assert count(20, bad, 0)[0] != 0
