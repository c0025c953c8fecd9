"""Python binding of ``libqvm.so`` (argument marshalling only).

Every operation runs in the HIP library; this module converts gate lists
into ``qvm_gate`` records, hands torch-owned device buffers and the current
torch stream to the C ABI, and turns status codes into exceptions.  There
is no fallback: if the library is missing, importing this module raises.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
# QVM_LIBRARY names another build of the library (the host-sanitizer tier)
LIB_PATH = os.environ.get("QVM_LIBRARY") or os.path.join(PKG, "libqvm.so")

QVM_C64, QVM_C128 = 1, 2
MAX_K = 6

KIND = {"unitary": 0, "matrix": 0, "i": 1, "h": 2, "x": 3, "y": 4, "z": 5, "s": 6,
        "sdg": 7, "t": 8, "tdg": 9, "rx": 10, "ry": 11, "rz": 12, "p": 13, "u3": 14,
        "rzz": 15, "swap": 16}

STATUS = {0: "QVM_OK", -1: "QVM_EARG", -2: "QVM_ERANGE", -3: "QVM_ENOMEM",
          -4: "QVM_EDEVICE", -5: "QVM_ESTATE", -6: "QVM_EUNSUPPORTED"}


class QvmError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class QvmGate(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("k", ctypes.c_int32),
                ("targets", ctypes.c_int32 * MAX_K), ("ctrl_mask", ctypes.c_uint64),
                ("params", ctypes.c_double * 3), ("u", ctypes.POINTER(ctypes.c_double))]


assert ctypes.sizeof(QvmGate) == 72

_vp = ctypes.c_void_p
_dp = ctypes.POINTER(ctypes.c_double)
_u64p = ctypes.POINTER(ctypes.c_uint64)
_i32p = ctypes.POINTER(ctypes.c_int32)
_u32p = ctypes.POINTER(ctypes.c_uint32)
_gp = ctypes.POINTER(QvmGate)

_lib = None


def _declare(L):
    st = ctypes.c_int
    sig = {
        "qvm_gate_matrix": (st, [_gp, _dp]),
        "qvm_workspace_bytes": (ctypes.c_size_t, [ctypes.c_int, ctypes.c_int]),
        "qvm_sv_create": (st, [ctypes.c_int, ctypes.c_int, _vp, _vp, ctypes.c_size_t, _vp,
                               ctypes.POINTER(_vp)]),
        "qvm_sv_destroy": (st, [_vp]),
        "qvm_sv_set_stream": (st, [_vp, _vp]),
        "qvm_init_basis": (st, [_vp, ctypes.c_uint64]),
        "qvm_apply": (st, [_vp, _gp]),
        "qvm_run": (st, [_vp, _gp, ctypes.c_size_t]),
        "qvm_apply_kraus": (st, [_vp, ctypes.c_int32, ctypes.c_int32, _dp, ctypes.c_double,
                                 _i32p, _dp]),
        "qvm_get_layout": (st, [_vp, _i32p]),
        "qvm_reset_layout": (st, [_vp]),
        "qvm_probabilities": (st, [_vp, ctypes.c_int, _i32p, _dp]),
        "qvm_expect_z_all": (st, [_vp, _dp]),
        "qvm_expect_pauli": (st, [_vp, ctypes.c_size_t, _u64p, _u64p, _dp, _dp, _dp]),
        "qvm_sample": (st, [_vp, ctypes.c_size_t, _dp, _u64p]),
        "qvm_norm": (st, [_vp, _dp]),
        "qvm_renormalize": (st, [_vp, _dp]),
        "qvm_copy_amplitudes": (st, [_vp, ctypes.c_uint64, ctypes.c_uint64, _dp]),
        "qvm_gather_amplitudes": (st, [_vp, ctypes.c_size_t, _u64p, _dp]),
        "qvm_last_error": (ctypes.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    return sig


def lib():
    """The loaded library.  Raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "paper_2212_14201_amd/build.py (no fallback exists)")
        # torch first: its HIP runtime has the same soname as the system one,
        # so the library then binds to the runtime that owns torch's device
        # memory and streams (one HIP runtime per process).  Loaded the other
        # way round, two runtimes coexist and the library's may see no device.
        import torch  # noqa: F401
        L = ctypes.CDLL(LIB_PATH)
        _declare(L)
        _lib = L
    return _lib


def check(status):
    if status != 0:
        msg = lib().qvm_last_error()
        raise QvmError(status, msg.decode() if msg else "")
    return status


# ------------------------------------------------------------------ gates
def _ctrl_mask(ctrls) -> int:
    m = 0
    for c in ctrls:
        m |= 1 << int(c)
    return m


class GateArray:
    """A packed array of qvm_gate records built from gate objects with
    ``name``, ``targets``, ``controls``, ``params`` and (for explicit
    unitaries) ``matrix`` attributes.  Keeps matrix buffers alive."""

    def __init__(self, gates, params=None):
        gates = list(gates)
        self.n = len(gates)
        self.arr = (QvmGate * max(1, self.n))()
        self._keep = []
        for i, g in enumerate(gates):
            rec = self.arr[i]
            kind = KIND[g.name]
            rec.kind = kind
            rec.k = len(g.targets)
            for r, t in enumerate(g.targets):
                rec.targets[r] = int(t)
            rec.ctrl_mask = _ctrl_mask(g.controls)
            ps = list(g.params)
            pidx = getattr(g, "pidx", -1)
            if params is not None and pidx is not None and pidx >= 0:
                ps = [float(params[pidx])]
            for j, p in enumerate(ps[:3]):
                rec.params[j] = float(p)
            if kind == 0:
                m = np.ascontiguousarray(np.asarray(g.matrix, dtype=np.complex128))
                buf = m.view(np.float64).ravel().copy()
                self._keep.append(buf)
                rec.u = buf.ctypes.data_as(_dp)
            else:
                rec.u = None

    def ptr(self):
        return ctypes.cast(self.arr, _gp)


class Circuit:
    """A circuit on n qubits under construction: a list of gate records
    (name, targets, controls, params[, matrix]) that the library calls take
    packed as a GateArray."""

    def __init__(self, n: int, gates=()):
        self.n = int(n)
        self.gates = []
        for g in gates:
            self.add(g)

    def add(self, gate):
        qs = tuple(gate.targets) + tuple(getattr(gate, "controls", ()))
        if any(q < 0 or q >= self.n for q in qs):
            raise ValueError(f"gate {gate.name} acts outside qubits 0..{self.n - 1}")
        self.gates.append(gate)
        return self

    def __len__(self):
        return len(self.gates)

    def __iter__(self):
        return iter(self.gates)

    def array(self) -> "GateArray":
        return GateArray(self.gates)


def plan(circuit, n: int | None = None, dtype: str = "c64", planner: str = "greedy",
         k_max: int = 3, tile_qubits: int = 13, defer_narrow: bool = True) -> "Plan":
    """A fused plan for a Circuit (or gate list).  planner="greedy": the
    greedy planner at (k_max, tile_qubits), by default with narrow trailing
    blocks left to a later pass (defer_narrow, tile passes only);
    planner="learned": the shipped cost model's choice among the candidate
    settings (needs the GPU for the model and fails when no model is
    shipped)."""
    if isinstance(circuit, Circuit):
        n = circuit.n if n is None else n
        gates = circuit.gates
    else:
        gates = circuit
    if n is None:
        raise ValueError("n is required for a plain gate list")
    if planner == "greedy":
        return Plan(gates, n, dtype, k_max=k_max, tile_qubits=tile_qubits,
                    defer_narrow=defer_narrow and tile_qubits > 0)
    if planner == "learned":
        from .learned_planner import load_default
        lp = load_default()
        if lp is None:
            raise RuntimeError("no trained cost model is shipped with this build")
        return lp.choose(gates if isinstance(gates, GateArray) else GateArray(gates), n, dtype)[1]
    raise ValueError(f"unknown planner {planner!r} (greedy or learned)")


def __getattr__(name):
    # torch.autograd.Function over the batched adjoint gradients, built on
    # first use (importing torch.autograd only when asked for)
    if name == "AdjointExpectation":
        from .adjoint import _function
        return _function()
    raise AttributeError(name)


def simplify(gates, n: int) -> "GateArray":
    """The library's peephole pre-pass (qvm_simplify): identity pairs removed,
    consecutive same-axis rotations merged.  Returns a new GateArray that
    keeps the input's matrix buffers alive."""
    ga = gates if isinstance(gates, GateArray) else GateArray(gates)
    L = lib()
    L.qvm_simplify.argtypes = [_gp, ctypes.c_size_t, ctypes.c_int, _gp, ctypes.POINTER(ctypes.c_size_t)]
    L.qvm_simplify.restype = ctypes.c_int
    out = GateArray([])
    out.arr = (QvmGate * max(1, ga.n))()
    cnt = ctypes.c_size_t()
    check(L.qvm_simplify(ga.ptr(), ga.n, int(n), ctypes.cast(out.arr, _gp), ctypes.byref(cnt)))
    out.n = int(cnt.value)
    out._keep = [ga]
    return out


def stream_copy(dst, src, stream=None):
    """qvm_stream_copy between two torch device tensors of equal byte size."""
    import torch
    L = lib()
    L.qvm_stream_copy.argtypes = [_vp, _vp, ctypes.c_size_t, _vp]
    L.qvm_stream_copy.restype = ctypes.c_int
    nb = src.numel() * src.element_size()
    if dst.numel() * dst.element_size() != nb:
        raise ValueError("stream_copy: sizes differ")
    if stream is None:
        stream = torch.cuda.current_stream(src.device).cuda_stream
    check(L.qvm_stream_copy(dst.data_ptr(), src.data_ptr(), nb, stream))


def gate_matrix(gate) -> np.ndarray:
    """The library's lowering of one gate (host only)."""
    ga = GateArray([gate])
    k = len(gate.targets)
    out = np.zeros(2 * (1 << (2 * k)), dtype=np.float64)
    check(lib().qvm_gate_matrix(ga.ptr(), out.ctypes.data_as(_dp)))
    return out.view(np.complex128).reshape(1 << k, 1 << k)


def workspace_bytes(n: int, dtype: str) -> int:
    return int(lib().qvm_workspace_bytes(n, _dt(dtype)))


def _dt(dtype) -> int:
    if dtype in ("c64", "complex64", QVM_C64):
        return QVM_C64
    if dtype in ("c128", "complex128", QVM_C128):
        return QVM_C128
    raise ValueError(f"unknown dtype {dtype!r}")


def _stream_ptr(device):
    import torch
    return torch.cuda.current_stream(device).cuda_stream


class StateVector:
    """2^n amplitudes in torch-owned device memory, driven by libqvm."""

    def __init__(self, n: int, dtype: str = "c128", device="cuda", init: int | None = 0):
        import torch
        self.n = int(n)
        self.dtype = "c64" if _dt(dtype) == QVM_C64 else "c128"
        self.device = torch.device(device)
        real = torch.float32 if self.dtype == "c64" else torch.float64
        self.amps = torch.empty(2 << self.n, dtype=real, device=self.device)
        self.work = torch.empty(workspace_bytes(self.n, self.dtype), dtype=torch.uint8,
                                device=self.device)
        h = _vp()
        check(lib().qvm_sv_create(self.n, _dt(self.dtype), self.amps.data_ptr(),
                                  self.work.data_ptr(), self.work.numel(),
                                  _stream_ptr(self.device), ctypes.byref(h)))
        self._h = h
        if init is not None:
            self.init_basis(init)

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().qvm_sv_destroy(self._h)
            self._h = _vp()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self):
        return self._h

    def sync_stream(self):
        """Re-bind the handle to torch's current stream."""
        check(lib().qvm_sv_set_stream(self._h, _stream_ptr(self.device)))

    # --------------------------------------------------------- evolution
    def init_basis(self, index: int = 0):
        check(lib().qvm_init_basis(self._h, int(index)))

    def apply(self, gate):
        ga = GateArray([gate])
        check(lib().qvm_apply(self._h, ga.ptr()))

    def run(self, gates, params=None):
        ga = gates if isinstance(gates, GateArray) else GateArray(gates, params)
        check(lib().qvm_run(self._h, ga.ptr(), ga.n))

    def apply_kraus(self, qubit: int, ops, u: float):
        """One Kraus channel on one qubit by a trajectory branching; ops is a
        sequence of 2x2 complex matrices.  Returns (branch, probabilities)."""
        k = np.ascontiguousarray(np.asarray(ops, dtype=np.complex128).reshape(-1, 2, 2))
        buf = np.ascontiguousarray(k.view(np.float64).reshape(-1))
        j = ctypes.c_int32(-1)
        probs = np.zeros(k.shape[0], dtype=np.float64)
        check(lib().qvm_apply_kraus(self._h, int(qubit), k.shape[0], buf.ctypes.data_as(_dp),
                                    float(u), ctypes.byref(j), probs.ctypes.data_as(_dp)))
        return int(j.value), probs

    def layout(self):
        out = np.zeros(self.n, dtype=np.int32)
        check(lib().qvm_get_layout(self._h, out.ctypes.data_as(_i32p)))
        return out

    def reset_layout(self):
        check(lib().qvm_reset_layout(self._h))

    # ------------------------------------------------------------ readout
    def probabilities(self, qubits=None) -> np.ndarray:
        if qubits is None:
            out = np.empty(1 << self.n, dtype=np.float64)
            check(lib().qvm_probabilities(self._h, self.n, None, out.ctypes.data_as(_dp)))
            return out
        q = np.ascontiguousarray(qubits, dtype=np.int32)
        out = np.empty(1 << q.size, dtype=np.float64)
        check(lib().qvm_probabilities(self._h, q.size, q.ctypes.data_as(_i32p),
                                      out.ctypes.data_as(_dp)))
        return out

    def expect_z_all(self) -> np.ndarray:
        out = np.empty(self.n, dtype=np.float64)
        check(lib().qvm_expect_z_all(self._h, out.ctypes.data_as(_dp)))
        return out

    def expect_pauli(self, xs, zs, coeffs=None):
        """Returns (per-term values, weighted sum or None)."""
        xs = np.ascontiguousarray(xs, dtype=np.uint64)
        zs = np.ascontiguousarray(zs, dtype=np.uint64)
        terms = np.empty(xs.size, dtype=np.float64)
        if coeffs is not None:
            cs = np.ascontiguousarray(coeffs, dtype=np.float64)
            tot = ctypes.c_double(0.0)
            check(lib().qvm_expect_pauli(self._h, xs.size, xs.ctypes.data_as(_u64p),
                                         zs.ctypes.data_as(_u64p), cs.ctypes.data_as(_dp),
                                         terms.ctypes.data_as(_dp), ctypes.byref(tot)))
            return terms, float(tot.value)
        check(lib().qvm_expect_pauli(self._h, xs.size, xs.ctypes.data_as(_u64p),
                                     zs.ctypes.data_as(_u64p), None,
                                     terms.ctypes.data_as(_dp), None))
        return terms, None

    def sample(self, uniforms) -> np.ndarray:
        u = np.ascontiguousarray(uniforms, dtype=np.float64)
        out = np.empty(u.size, dtype=np.uint64)
        check(lib().qvm_sample(self._h, u.size, u.ctypes.data_as(_dp),
                               out.ctypes.data_as(_u64p)))
        return out

    def norm(self) -> float:
        v = ctypes.c_double(0.0)
        check(lib().qvm_norm(self._h, ctypes.byref(v)))
        return float(v.value)

    def renormalize(self) -> float:
        v = ctypes.c_double(0.0)
        check(lib().qvm_renormalize(self._h, ctypes.byref(v)))
        return float(v.value)

    def amplitudes(self, first: int = 0, count: int | None = None) -> np.ndarray:
        if count is None:
            count = (1 << self.n) - first
        out = np.empty(2 * count, dtype=np.float64)
        check(lib().qvm_copy_amplitudes(self._h, int(first), int(count), out.ctypes.data_as(_dp)))
        return out.view(np.complex128)

    def gather(self, indices) -> np.ndarray:
        idx = np.ascontiguousarray(indices, dtype=np.uint64)
        out = np.empty(2 * idx.size, dtype=np.float64)
        check(lib().qvm_gather_amplitudes(self._h, idx.size, idx.ctypes.data_as(_u64p),
                                          out.ctypes.data_as(_dp)))
        return out.view(np.complex128)


# ------------------------------------------------------------------ plans
class QvmPlanStats(ctypes.Structure):
    _fields_ = [("n_passes", ctypes.c_int32), ("n_blocks", ctypes.c_int32),
                ("n_diag_ops", ctypes.c_int32), ("tile_qubits", ctypes.c_int32),
                ("blocks_by_k", ctypes.c_int32 * 8), ("device_bytes", ctypes.c_uint64)]


def _declare_plan(L):
    st = ctypes.c_int
    sig = {
        "qvm_plan_greedy": (st, [_gp, ctypes.c_size_t, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                 ctypes.c_int, ctypes.POINTER(_vp)]),
        "qvm_plan_greedy_ex": (st, [_gp, ctypes.c_size_t, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                    ctypes.c_int, ctypes.c_uint32, ctypes.POINTER(_vp)]),
        "qvm_plan_from_partition": (st, [_gp, ctypes.c_size_t, _u32p, ctypes.c_int, ctypes.c_int,
                                         ctypes.c_int, ctypes.POINTER(_vp)]),
        "qvm_plan_tile_per_pass": (st, [_gp, ctypes.c_size_t, ctypes.c_int, ctypes.c_int, _i32p,
                                        ctypes.c_int32, ctypes.c_int, ctypes.c_uint32, ctypes.POINTER(_vp)]),
        "qvm_plan_info": (st, [_vp, ctypes.POINTER(QvmPlanStats)]),
        "qvm_plan_block": (st, [_vp, ctypes.c_int32, _i32p, _i32p, _i32p, _i32p, _i32p, _i32p, _dp]),
        "qvm_plan_schedule": (st, [_vp, _i32p, _i32p]),
        "qvm_plan_final_layout": (st, [_vp, _i32p]),
        "qvm_run_plan": (st, [_vp, _vp]),
        "qvm_plan_destroy": (st, [_vp]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args


QVM_PLAN_NO_IMAGE = 1
QVM_PLAN_DEFER_NARROW = 2


class Plan:
    """A fused execution plan (host object built by the library).

    image=False builds it for scoring only (schedule, statistics and pass
    features without block matrices or device image); such a plan cannot run.
    k_of_pass: tile passes whose block width is chosen per pass
    (qvm_plan_tile_per_pass; k_max is then ignored).  defer_narrow: tile
    passes leave blocks narrower than 3 qubits that end their wires' work in
    the pass to a later pass (QVM_PLAN_DEFER_NARROW)."""

    def __init__(self, gates, n: int, dtype: str = "c64", k_max: int = 5, tile_qubits: int = 0,
                 partition=None, image: bool = True, k_of_pass=None, defer_narrow: bool = False):
        _declare_plan(lib())
        self.gates = gates if isinstance(gates, GateArray) else GateArray(gates)
        self.n = int(n)
        self.dtype = "c64" if _dt(dtype) == QVM_C64 else "c128"
        self.k_max, self.tile_qubits, self.image = int(k_max), int(tile_qubits), bool(image)
        h = _vp()
        self.k_of_pass = None if k_of_pass is None else [int(k) for k in k_of_pass]
        self.defer_narrow = bool(defer_narrow)
        if defer_narrow and (k_of_pass is not None or partition is not None):
            raise ValueError("defer_narrow applies to the greedy planner only")
        if k_of_pass is not None:
            if partition is not None:
                raise ValueError("k_of_pass and partition are exclusive")
            ks = np.ascontiguousarray(k_of_pass, dtype=np.int32)
            self.k_max = int(ks.max()) if ks.size else 0
            flags = 0 if image else QVM_PLAN_NO_IMAGE
            check(lib().qvm_plan_tile_per_pass(self.gates.ptr(), self.gates.n, self.n, int(tile_qubits),
                                               ks.ctypes.data_as(_i32p), int(ks.size), _dt(dtype), flags,
                                               ctypes.byref(h)))
        elif partition is None:
            flags = (0 if image else QVM_PLAN_NO_IMAGE) | (QVM_PLAN_DEFER_NARROW if defer_narrow else 0)
            check(lib().qvm_plan_greedy_ex(self.gates.ptr(), self.gates.n, self.n, int(k_max),
                                           int(tile_qubits), _dt(dtype), flags, ctypes.byref(h)))
        elif not image:
            raise ValueError("scoring-only plans are built by the greedy planner only")
        else:
            part = np.ascontiguousarray(partition, dtype=np.uint32)
            check(lib().qvm_plan_from_partition(self.gates.ptr(), self.gates.n,
                                                part.ctypes.data_as(_u32p), self.n, int(k_max),
                                                _dt(dtype), ctypes.byref(h)))
        self._h = h

    def __del__(self):
        try:
            if self._h.value:
                lib().qvm_plan_destroy(self._h)
                self._h = _vp()
        except Exception:
            pass

    def stats(self) -> dict:
        s = QvmPlanStats()
        check(lib().qvm_plan_info(self._h, ctypes.byref(s)))
        return {"passes": s.n_passes, "blocks": s.n_blocks, "diag_ops": s.n_diag_ops,
                "tile_qubits": s.tile_qubits, "blocks_by_k": list(s.blocks_by_k),
                "device_bytes": int(s.device_bytes)}

    def block(self, i: int) -> dict:
        k = ctypes.c_int32()
        kt = ctypes.c_int32()
        ng = ctypes.c_int32()
        ps = ctypes.c_int32()
        check(lib().qvm_plan_block(self._h, i, ctypes.byref(k), ctypes.byref(kt), None,
                                   ctypes.byref(ng), None, ctypes.byref(ps), None))
        qs = np.zeros(k.value, np.int32)
        gi = np.zeros(ng.value, np.int32)
        m = np.zeros(2 << (2 * k.value), np.float64)
        check(lib().qvm_plan_block(self._h, i, None, None, qs.ctypes.data_as(_i32p), None,
                                   gi.ctypes.data_as(_i32p), None, m.ctypes.data_as(_dp)))
        return {"k": k.value, "k_true": kt.value, "qubits": qs.tolist(), "gates": gi.tolist(),
                "pass": ps.value, "matrix": m.view(np.complex128).reshape(1 << k.value, 1 << k.value)}

    def schedule(self):
        pos = np.zeros(self.gates.n, np.int32)
        unit = np.zeros(self.gates.n, np.int32)
        check(lib().qvm_plan_schedule(self._h, pos.ctypes.data_as(_i32p), unit.ctypes.data_as(_i32p)))
        return pos, unit

    def final_layout(self):
        out = np.zeros(self.n, np.int32)
        check(lib().qvm_plan_final_layout(self._h, out.ctypes.data_as(_i32p)))
        return out

    def run(self, sv: "StateVector"):
        check(lib().qvm_run_plan(sv.handle, self._h))
