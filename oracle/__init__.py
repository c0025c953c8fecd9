"""FP64 CPU oracle for the full-amplitude state-vector path.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg are the only users.  The product library never imports,
links or calls anything here, and nothing here imports the product package.

The arithmetic lives in ``qvm_oracle.c`` (plain loops, FP64, compensated
sums); this module marshals gate lists from ``workloads`` into it.  The one
pure-Python piece is the plan validator and block-matrix builder for gate
fusion (paper, "Quantum circuit fusion"), which reuse the C gate-application
routine on a k-qubit register.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# QVM_ORACLE_LIBRARY names another build of the oracle (the host-sanitizer tier)
_LIB_PATH = os.environ.get("QVM_ORACLE_LIBRARY") or os.path.join(HERE, "liboracle.so")
_lib = None

_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int)
_i64p = ctypes.POINTER(ctypes.c_int64)
_u64p = ctypes.POINTER(ctypes.c_uint64)


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            from . import build as _b
            _b.build()
        L = ctypes.CDLL(_LIB_PATH)
        L.orc_gate_matrix.argtypes = [ctypes.c_char_p, _dp, _dp]
        L.orc_gate_matrix.restype = ctypes.c_int
        L.orc_init_basis.argtypes = [_dp, ctypes.c_int, ctypes.c_uint64]
        L.orc_apply.argtypes = [_dp, ctypes.c_int, _dp, ctypes.c_int, _ip, ctypes.c_uint64]
        L.orc_run.argtypes = [_dp, ctypes.c_int, ctypes.c_int64, _dp, _i64p, _ip, _ip, _u64p]
        L.orc_probabilities.argtypes = [_dp, ctypes.c_int, _dp]
        L.orc_marginal.argtypes = [_dp, ctypes.c_int, ctypes.c_int, _ip, _dp]
        L.orc_norm2.argtypes = [_dp, ctypes.c_int]
        L.orc_norm2.restype = ctypes.c_double
        L.orc_expect_pauli.argtypes = [_dp, ctypes.c_int, ctypes.c_uint64, ctypes.c_uint64, _dp]
        L.orc_expect_pauli.restype = ctypes.c_double
        L.orc_apply_pauli.argtypes = [_dp, ctypes.c_int, ctypes.c_uint64, ctypes.c_uint64,
                                      ctypes.c_double, _dp, ctypes.c_int]
        L.orc_sample.argtypes = [_dp, ctypes.c_int, ctypes.c_int64, _dp, _u64p, _dp]
        L.orc_adjoint.argtypes = [ctypes.c_int, ctypes.c_int64, _dp, _i64p, _ip, _ip, _u64p,
                                  _ip, _ip, ctypes.c_int64, _u64p, _u64p, _dp, _dp, _dp]
        L.orc_adjoint.restype = ctypes.c_int
        L.orc_max_threads.restype = ctypes.c_int
        L.orc_set_threads.argtypes = [ctypes.c_int]
        _lib = L
    return _lib


def _d(a):
    return a.ctypes.data_as(_dp)


def max_threads() -> int:
    return int(lib().orc_max_threads())


def set_threads(t: int) -> None:
    """Thread count of the oracle's parallel loops from now on."""
    lib().orc_set_threads(int(t))


def gate_matrix(gate) -> np.ndarray:
    """The gate's target matrix (controls excluded), complex128 2^k x 2^k."""
    if gate.name == "unitary":
        m = np.asarray(gate.matrix, dtype=np.complex128)
        return m.copy()
    buf = np.zeros(2 * 16, dtype=np.float64)
    p = np.zeros(3, dtype=np.float64)
    p[:len(gate.params)] = gate.params
    k = lib().orc_gate_matrix(gate.name.encode(), _d(p), _d(buf))
    if k < 0:
        raise ValueError(f"unknown gate {gate.name!r}")
    dim = 1 << k
    if k != len(gate.targets):
        raise ValueError(f"gate {gate.name} takes {k} targets")
    return buf[:2 * dim * dim].view(np.complex128).reshape(dim, dim).copy()


def _cmask(ctrls) -> int:
    m = 0
    for c in ctrls:
        m |= 1 << int(c)
    return m


def basis_state(n: int, x: int = 0) -> np.ndarray:
    psi = np.empty(1 << n, dtype=np.complex128)
    lib().orc_init_basis(_d(psi.view(np.float64)), n, x)
    return psi


def apply_matrix(psi: np.ndarray, n: int, u: np.ndarray, targets, controls=()):
    u = np.ascontiguousarray(u, dtype=np.complex128)
    t = np.zeros(6, dtype=np.int32)
    t[:len(targets)] = targets
    lib().orc_apply(_d(psi.view(np.float64)), n, _d(u.view(np.float64)), len(targets),
                    t.ctypes.data_as(_ip), _cmask(controls))


def apply_gates(psi: np.ndarray, n: int, gates, params=None):
    """Apply gates in order, in place.  Trainable gates (pidx >= 0) take
    their angle from ``params`` when it is given."""
    for g in gates:
        if params is not None and g.pidx >= 0:
            g = type(g)(g.name, g.targets, g.controls, (float(params[g.pidx]),), g.pidx)
        apply_matrix(psi, n, gate_matrix(g), g.targets, g.controls)
    return psi


def simulate(n: int, gates, init: int = 0, params=None) -> np.ndarray:
    return apply_gates(basis_state(n, init), n, gates, params)


def probabilities(psi: np.ndarray) -> np.ndarray:
    n = int(psi.size).bit_length() - 1
    p = np.empty(psi.size, dtype=np.float64)
    lib().orc_probabilities(_d(psi.view(np.float64)), n, _d(p))
    return p


def marginal(psi: np.ndarray, qubits) -> np.ndarray:
    n = int(psi.size).bit_length() - 1
    q = np.asarray(qubits, dtype=np.int32)
    out = np.empty(1 << len(q), dtype=np.float64)
    lib().orc_marginal(_d(psi.view(np.float64)), n, len(q), q.ctypes.data_as(_ip), _d(out))
    return out


def norm2(psi: np.ndarray) -> float:
    n = int(psi.size).bit_length() - 1
    return float(lib().orc_norm2(_d(psi.view(np.float64)), n))


def expect_pauli(psi: np.ndarray, x: int, z: int):
    """Returns (re, im) of <psi|P|psi> for the symplectic string (x, z)."""
    n = int(psi.size).bit_length() - 1
    im = ctypes.c_double(0.0)
    re = lib().orc_expect_pauli(_d(psi.view(np.float64)), n, int(x), int(z), ctypes.byref(im))
    return float(re), float(im.value)


def expect_z_all(psi: np.ndarray) -> np.ndarray:
    n = int(psi.size).bit_length() - 1
    return np.array([expect_pauli(psi, 0, 1 << q)[0] for q in range(n)])


def expect_zz(psi: np.ndarray, pairs) -> np.ndarray:
    return np.array([expect_pauli(psi, 0, (1 << a) | (1 << b))[0] for a, b in pairs])


def apply_pauli_sum(psi: np.ndarray, xs, zs, cs) -> np.ndarray:
    n = int(psi.size).bit_length() - 1
    out = np.zeros_like(psi)
    for x, z, c in zip(xs, zs, cs):
        lib().orc_apply_pauli(_d(psi.view(np.float64)), n, int(x), int(z), float(c),
                              _d(out.view(np.float64)), 1)
    return out


def sample(psi: np.ndarray, uniforms):
    """Returns (indices, margins) for the uniform stream."""
    n = int(psi.size).bit_length() - 1
    u = np.ascontiguousarray(uniforms, dtype=np.float64)
    out = np.empty(u.size, dtype=np.uint64)
    mar = np.empty(u.size, dtype=np.float64)
    lib().orc_sample(_d(psi.view(np.float64)), n, u.size, _d(u), out.ctypes.data_as(_u64p), _d(mar))
    return out, mar


_GEN = {"rx": 1, "ry": 2, "rz": 3}


def _pack(gates, params=None):
    mats, offs, ks, tg, cm, gen, pidx = [], [], [], [], [], [], []
    off = 0
    for g in gates:
        if params is not None and g.pidx >= 0:
            g = type(g)(g.name, g.targets, g.controls, (float(params[g.pidx]),), g.pidx)
        m = gate_matrix(g)
        mats.append(m.ravel())
        offs.append(off)
        off += 2 * m.size
        ks.append(len(g.targets))
        t = list(g.targets) + [0] * (6 - len(g.targets))
        tg.extend(t)
        cm.append(_cmask(g.controls))
        if g.pidx >= 0:
            if g.name not in _GEN:
                raise ValueError("trainable gates must be rx/ry/rz")
            gen.append(_GEN[g.name])
        else:
            gen.append(0)
        pidx.append(max(g.pidx, 0))
    flat = np.concatenate(mats).astype(np.complex128) if mats else np.zeros(1, np.complex128)
    return (flat.view(np.float64).copy(), np.array(offs, np.int64), np.array(ks, np.int32),
            np.array(tg, np.int32), np.array(cm, np.uint64), np.array(gen, np.int32),
            np.array(pidx, np.int32))


def run_packed(n: int, gates, init: int = 0, params=None) -> np.ndarray:
    """Same as simulate(), one C call for the whole list."""
    mats, offs, ks, tg, cm, _, _ = _pack(gates, params)
    psi = basis_state(n, init)
    lib().orc_run(_d(psi.view(np.float64)), n, len(gates), _d(mats), offs.ctypes.data_as(_i64p),
                  ks.ctypes.data_as(_ip), tg.ctypes.data_as(_ip), cm.ctypes.data_as(_u64p))
    return psi


def adjoint(n: int, gates, params, xs, zs, cs, nparams=None):
    """f(theta) = <psi|H|psi> and its gradient by the reverse sweep."""
    mats, offs, ks, tg, cm, gen, pidx = _pack(gates, params)
    P = nparams if nparams is not None else len(params)
    grad = np.zeros(P, dtype=np.float64)
    f = ctypes.c_double(0.0)
    xs = np.ascontiguousarray(xs, dtype=np.uint64)
    zs = np.ascontiguousarray(zs, dtype=np.uint64)
    cs = np.ascontiguousarray(cs, dtype=np.float64)
    rc = lib().orc_adjoint(n, len(gates), _d(mats), offs.ctypes.data_as(_i64p),
                           ks.ctypes.data_as(_ip), tg.ctypes.data_as(_ip), cm.ctypes.data_as(_u64p),
                           gen.ctypes.data_as(_ip), pidx.ctypes.data_as(_ip), xs.size,
                           xs.ctypes.data_as(_u64p), zs.ctypes.data_as(_u64p), _d(cs),
                           ctypes.byref(f), _d(grad))
    if rc != 0:
        raise MemoryError("oracle adjoint allocation failed")
    return float(f.value), grad


def energy(n: int, gates, params, xs, zs, cs) -> float:
    psi = run_packed(n, gates, 0, params)
    return float(sum(c * expect_pauli(psi, x, z)[0] for x, z, c in zip(xs, zs, cs)))


# ---------------------------------------------------------------------------
# Gate fusion (paper, "Quantum circuit fusion"): a block over qubits
# (b_0..b_{k-1}) has matrix G_m ... G_1, each gate embedded in the k-qubit
# register with b_r <-> bit r.  Built column by column by applying the gates
# to the register's basis states.
# ---------------------------------------------------------------------------
def block_matrix(gates, block_qubits) -> np.ndarray:
    bq = list(block_qubits)
    pos = {q: r for r, q in enumerate(bq)}
    k = len(bq)
    dim = 1 << k
    M = np.zeros((dim, dim), dtype=np.complex128)
    for col in range(dim):
        v = basis_state(k, col)
        for g in gates:
            apply_matrix(v, k, gate_matrix(g), [pos[q] for q in g.targets],
                         [pos[q] for q in g.controls])
        M[:, col] = v
    return M


def is_diagonal(gate) -> bool:
    """True when the gate's target matrix has zeros off its diagonal (then,
    controls included, the gate is diagonal in the computational basis)."""
    u = gate_matrix(gate)
    return not np.any(u - np.diag(np.diag(u)))


def validate_plan(gates, blocks, k_max: int):
    """A plan is a list of blocks, each a list of gate indices, in execution
    order.  Valid iff every gate is in exactly one block, every block spans
    at most k_max qubits, and the execution order respects the dependency
    graph of the circuit: two gates that share a qubit keep their program
    order unless both are diagonal (diagonal matrices commute).  Per qubit:
    a non-diagonal gate runs after every earlier gate on that qubit, a
    diagonal gate after the last earlier non-diagonal one.  Returns
    (ok, reason)."""
    seen = {}
    for b, blk in enumerate(blocks):
        qs = set()
        for gi in blk:
            if gi in seen:
                return False, f"gate {gi} in blocks {seen[gi]} and {b}"
            seen[gi] = b
            qs.update(gates[gi].qubits())
        if len(qs) > k_max:
            return False, f"block {b} spans {len(qs)} > {k_max} qubits"
    if len(seen) != len(gates):
        return False, "not every gate is in a block"
    # position of each gate in execution order
    order = {}
    t = 0
    for blk in blocks:
        for gi in blk:
            order[gi] = t
            t += 1
    diag = [is_diagonal(g) for g in gates]
    last_nd = {}        # qubit -> last non-diagonal gate on it
    since = {}          # qubit -> diagonal gates on it after that one
    for gi, g in enumerate(gates):
        for q in g.qubits():
            before = [last_nd[q]] if q in last_nd else []
            if not diag[gi]:
                before += since.get(q, [])
            for p in before:
                if order[p] > order[gi]:
                    return False, f"gates {p} and {gi} on qubit {q} out of order"
            if diag[gi]:
                since.setdefault(q, []).append(gi)
            else:
                last_nd[q] = gi
                since[q] = []
    return True, ""
