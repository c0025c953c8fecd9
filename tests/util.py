"""Shared helpers for the test suite (tolerances, oracle shortcuts)."""
import math
import os
import re

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

U32 = 2.0 ** -24          # unit roundoff of binary32

C128_TOL = 1e-12          # max-abs amplitude error allowed in complex128


def c64_bound(ks):
    """Stated per-result bound for complex64 amplitudes after passes whose
    matrices are 2^k x 2^k: probabilistic rounding-error model, each pass
    contributing (2^k + 4) roundings of size u, summed in quadrature, with a
    safety factor of 10."""
    s = sum((1 << k) + 4 for k in ks)
    return 10.0 * math.sqrt(max(s, 1)) * U32


def gate_ks(gates):
    return [len(g.targets) for g in gates]


def header_functions():
    """Every function declared in include/*.h."""
    names = []
    inc = os.path.join(ROOT, "include")
    for f in sorted(os.listdir(inc)):
        if f.endswith(".h"):
            txt = open(os.path.join(inc, f)).read()
            txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
            names += re.findall(r"\b(qvm_[a-z0-9_]+)\s*\(", txt)
    return sorted(set(names))


# Device-image records of the tile kernel (layouts in csrc/tile.hpp).
_PD = np.dtype([("L", "<i4"), ("c", "<i4"), ("nops", "<i4"), ("remap", "<i4"), ("kmax", "<i4"),
                ("first_block", "<i4"), ("qmask", "<u8"), ("ops", "<u8"), ("ldoff", "<u8"),
                ("rmhi", "<u8"), ("rmlo", "<u8"), ("tabs", "<u8"), ("cistab", "<u8"), ("psum", "<u8"),
                ("npsum", "<i4"), ("pad", "<i4")])
_TOP = np.dtype([("type", "<i4"), ("k", "<i4"), ("lb", "<i4", 6), ("data", "<u8"),
                 ("next_block", "<i4"), ("flags", "<i4"), ("tab", "<u8"), ("next_data", "<u8")])
_DSUB = np.dtype([("lmask", "<u4"), ("lval", "<u4"), ("neg", "<i4"), ("rows", "<u4"), ("omask", "<u8"),
                  ("oval", "<u8"), ("pr", "<f8"), ("pi", "<f8"), ("turns", "<u8"), ("pad", "<u8")])
_DTERM = np.dtype([("omask", "<u8"), ("oval", "<u8"), ("turns", "<u8"), ("lmask", "<u4"), ("lval", "<u4")])
_ETERM = np.dtype([("om", "<u4"), ("ov", "<u4"), ("lm", "<u4"), ("lv", "<u4"), ("w", "<u4"), ("pad", "<u4", 3)])
_PREC = np.dtype([("om", "<u4"), ("ov", "<u4"), ("w", "<u4"), ("pad", "<u4")])


def plan_image(plan):
    """(record reader, pass descriptors) of a plan's device image."""
    import ctypes
    from paper_2212_14201_amd import qvm
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


def epilogue_runs(plan, signs=False):
    """Diagonal runs of a plan that ride in a block's epilogue (with signs:
    only those whose terms are all factors of -1)."""
    rec, passes = plan_image(plan)
    want = 4 | (2 if signs else 0)
    return sum(int(op["flags"]) & want == want for pd in passes
               for op in rec(int(pd["ops"]), _TOP, int(pd["nops"])) if op["type"] == 2)


def blocks_and_diagonals(n, seed, layers=14, signs_only=False):
    """Layers of three dense gates (H, RX, CNOT) each followed by 2..8
    diagonal gates (RZ, CZ, controlled phase, RZZ, T; with signs_only CZ and
    Z only) on random qubits: the diagonal runs land right after blocks."""
    from workloads import Gate
    rng = np.random.Generator(np.random.PCG64(seed))
    gates = []
    for _ in range(layers):
        for _ in range(3):
            a, b = (int(v) for v in rng.choice(n, 2, replace=False))
            th = float(rng.uniform(0, 2 * np.pi))
            gates.append([Gate("h", (a,)), Gate("rx", (a,), (), (th,)), Gate("x", (a,), (b,))][int(rng.integers(0, 3))])
        for _ in range(int(rng.integers(2, 9))):
            a, b = (int(v) for v in rng.choice(n, 2, replace=False))
            th = float(rng.uniform(0, 2 * np.pi))
            if signs_only:
                gates.append([Gate("z", (a,), (b,)), Gate("z", (a,))][int(rng.integers(0, 2))])
                continue
            gates.append([Gate("rz", (a,), (), (th,)), Gate("z", (a,), (b,)), Gate("p", (a,), (b,), (th,)),
                          Gate("rzz", (a, b), (), (th,)), Gate("t", (a,))][int(rng.integers(0, 5))])
    return gates


def tile_blocks_outer_diagonals(n_tile, n, seed, layers=14, signs_only=False):
    """blocks_and_diagonals with the dense gates on qubits below n_tile and
    the diagonal gates on any of the n qubits: one pass of n_tile-qubit
    tiles whose diagonal runs test the tile's outer bits."""
    from workloads import Gate
    rng = np.random.Generator(np.random.PCG64(seed))
    gates = []
    for _ in range(layers):
        for _ in range(3):
            a, b = (int(v) for v in rng.choice(n_tile, 2, replace=False))
            th = float(rng.uniform(0, 2 * np.pi))
            gates.append([Gate("h", (a,)), Gate("rx", (a,), (), (th,)), Gate("x", (a,), (b,))][int(rng.integers(0, 3))])
        for _ in range(int(rng.integers(2, 9))):
            a, b = (int(v) for v in rng.choice(n, 2, replace=False))
            th = float(rng.uniform(0, 2 * np.pi))
            if signs_only:
                gates.append([Gate("z", (a,), (b,)), Gate("z", (a,))][int(rng.integers(0, 2))])
                continue
            gates.append([Gate("rz", (a,), (), (th,)), Gate("z", (a,), (b,)), Gate("p", (a,), (b,), (th,)),
                          Gate("rzz", (a, b), (), (th,)), Gate("t", (a,))][int(rng.integers(0, 5))])
    return gates


def cdf_window(samples, cdf, uniforms, eps):
    """Validity of samples drawn from a perturbed state: with C the FP64
    cumulative probability of a reference state (C[-1] its total), sample s
    for uniform u is valid when C(s-1) - eps <= u C[-1] <= C(s) + eps
    (C(-1) = 0).  If every C of the sampling state is within eps/2 of the
    reference's, every exact sample of that state passes.  Returns (ok,
    slack) per sample, slack >= 0 exactly when ok."""
    s = np.asarray(samples, dtype=np.int64)
    t = np.asarray(uniforms, dtype=np.float64) * cdf[-1]
    hi = cdf[s]
    lo = np.where(s > 0, cdf[np.maximum(s - 1, 0)], 0.0)
    slack = np.minimum(t - (lo - eps), (hi + eps) - t)
    return slack >= 0, slack


def cdf_eps(tau):
    """Stated bound on the sampling window for a state with 2-norm error at
    most tau: sum_i |dp_i| <= 2 tau + tau^2 bounds the error of every
    cumulative probability, counted once for C(s) and once for the total."""
    return 2.0 * (2.0 * tau + tau * tau)



def long_phase_run(n, count, seed):
    """Three U3 gates (one block), then `count` controlled phases with
    distinct angles on random qubit pairs: a diagonal run of `count` terms
    after a block."""
    from workloads import Gate
    rng = np.random.Generator(np.random.PCG64(seed))
    gates = [Gate("u3", (q,), (), tuple(rng.uniform(0, 2 * np.pi, 3))) for q in range(3)]
    for _ in range(count):
        t, c = (int(v) for v in rng.choice(n, 2, replace=False))
        gates.append(Gate("p", (t,), (c,), (float(rng.uniform(0, 2 * np.pi)),)))
    return gates
