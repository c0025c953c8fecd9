"""Noisy simulation by Kraus trajectories (paper, "Noise simulation method").

The paper's noise models are single-qubit Kraus operator sets with an
adjustable error rate, attached to gate types.  One noisy run here is one
trajectory: after every gate whose type carries a model, each qubit the gate
touches (targets, then controls) goes through one branching of the channel
(``StateVector.apply_kraus``: branch weights from the qubit's reduced
density matrix in FP64, the branch drawn with the caller's next uniform, the
chosen operator applied by the plain gate kernels).  Averaged over many
trajectories the states reproduce the channel's density matrix.

Channels (the paper's equations):
  damping         [[1, 0], [0, sqrt(1-p)]],  [[0, sqrt(p)], [0, 0]]
  dephasing       sqrt(1-p) I,  sqrt(p) Z          (phase_flip is the same set)
  decoherence     K_a(damping, p1) K_b(dephasing, p2) for a, b in {1, 2}, with
                  p1 = 1 - exp(-tgate/T1), p2 = (1 - exp(-(tgate/T2 - tgate/(2 T1)))) / 2
  depolarizing    sqrt(1 - 3p/4) I,  sqrt(p)/2 X,  sqrt(p)/2 Y,  sqrt(p)/2 Z
  bit_phase_flip  sqrt(1-p) I,  sqrt(p) Y           (printed as the bit-or-phase flip)
  bit_flip        sqrt(1-p) I,  sqrt(p) X           (the flip the paper's example names)
  phase_damping   [[1, 0], [0, sqrt(1-p)]],  [[0, 0], [0, sqrt(p)]]
"""
from __future__ import annotations

import numpy as np

CHANNELS = {"damping": 0, "dephasing": 1, "phase_flip": 1, "decoherence": 2, "depolarizing": 3,
            "bit_phase_flip": 4, "bit_flip": 5, "phase_damping": 6}


def kraus_ops(kind: str, p: float = 0.0, t1: float = 0.0, t2: float = 0.0,
              tgate: float = 0.0) -> np.ndarray:
    """Kraus operators of a channel as an (m, 2, 2) complex128 array, lowered
    by the library (``qvm_kraus_ops``).  ValueError for an unknown kind or
    invalid rates."""
    import ctypes
    from .qvm import QvmError, check, lib
    if kind not in CHANNELS:
        raise ValueError(f"unknown channel {kind!r}")
    L = lib()
    L.qvm_kraus_ops.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                ctypes.c_double, ctypes.POINTER(ctypes.c_double),
                                ctypes.POINTER(ctypes.c_int32)]
    L.qvm_kraus_ops.restype = ctypes.c_int
    buf = np.zeros(16 * 8, dtype=np.float64)
    m = ctypes.c_int32(0)
    try:
        check(L.qvm_kraus_ops(CHANNELS[kind], float(p), float(t1), float(t2), float(tgate),
                              buf.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), ctypes.byref(m)))
    except QvmError as e:
        raise ValueError(str(e)) from None
    return buf[: 8 * m.value].view(np.complex128).reshape(m.value, 2, 2).copy()


_CONTROLLED = {("x", 1): "cnot", ("x", 2): "toffoli", ("z", 1): "cz", ("p", 1): "cr"}


def gate_type(g) -> str:
    """The type a noise model attaches to: cnot, toffoli, cz and cr for the
    controlled X / Z / P gates, otherwise the gate's name (with "+kc" for k
    other controls, so an "x" entry never matches a controlled X)."""
    k = len(g.controls)
    if k == 0:
        return g.name
    return _CONTROLLED.get((g.name, k), f"{g.name}+{k}c")


class NoiseModel:
    """Channels attached to gate types (``gate_type``): after every gate of
    that type, the channel acts on each qubit the gate touches (targets,
    then controls)."""

    def __init__(self, entries=()):
        self.entries = []
        for name, kind, params in entries:
            self.add(name, kind, **params)

    def add(self, gate_name: str, kind: str, **params):
        self.entries.append((gate_name, kind, params, kraus_ops(kind, **params)))
        return self

    def channels_for(self, gate):
        t = gate_type(gate)
        return [ops for name, _, _, ops in self.entries if name == t]

    def branchings(self, gates) -> int:
        """Uniforms one trajectory of this gate list consumes."""
        return sum(len(self.channels_for(g)) * (len(g.targets) + len(g.controls)) for g in gates)


def run_trajectory(sv, gates, model: NoiseModel, uniforms, init: int = 0):
    """One noisy run from |init>: gates without noise go to the plain path
    in batches; each noisy gate is followed by its branchings.  Returns the
    chosen branch of every branching, in order."""
    need = model.branchings(gates)
    u = np.asarray(uniforms, dtype=np.float64)
    if u.size < need:
        raise ValueError(f"{need} uniforms needed, {u.size} given")
    sv.init_basis(init)
    branches = []
    k = 0
    batch = []
    for g in gates:
        batch.append(g)
        chans = model.channels_for(g)
        if not chans:
            continue
        sv.run(batch)
        batch = []
        for ops in chans:
            for q in tuple(g.targets) + tuple(g.controls):
                j, _ = sv.apply_kraus(q, ops, u[k])
                k += 1
                branches.append(j)
    if batch:
        sv.run(batch)
    return branches
