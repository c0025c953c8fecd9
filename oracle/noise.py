"""Noisy simulation by Kraus trajectories, FP64 (paper, "Noise simulation method").

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg are the only users; the product library never imports or
calls anything here, and nothing here imports the product package.

The channels are the paper's single-qubit Kraus sets (its damping,
dephasing, decoherence, depolarizing, bit-or-phase flip and phase damping
equations), written out here from those equations.  A trajectory step is the
plain definition: the weight of branch i is ||K_i psi||^2 (the operator
applied to a copy of the state), the branch is drawn with a uniform u
against the cumulative weights, and the state becomes K_j psi rescaled to
its previous norm.  ``channel`` evolves a density matrix, sum_i K_i rho
K_i^dag, for the checks that pin the trajectories to the channel.
"""
from __future__ import annotations

import math

import numpy as np

from . import apply_gates, apply_matrix, basis_state

_I = np.eye(2, dtype=np.complex128)
_X = np.array([[0, 1], [1, 0]], dtype=np.complex128)
_Y = np.array([[0, -1j], [1j, 0]], dtype=np.complex128)
_Z = np.array([[1, 0], [0, -1]], dtype=np.complex128)


def _damping(p):
    # paper: K1 = [[1, 0], [0, sqrt(1-p)]], K2 = [[0, sqrt(p)], [0, 0]]
    return [np.array([[1, 0], [0, math.sqrt(1 - p)]], dtype=np.complex128),
            np.array([[0, math.sqrt(p)], [0, 0]], dtype=np.complex128)]


def _dephasing(p):
    # paper: K1 = sqrt(1-p) I, K2 = diag(sqrt(p), -sqrt(p))
    return [math.sqrt(1 - p) * _I, math.sqrt(p) * _Z]


def kraus(kind: str, p: float = 0.0, t1: float = 0.0, t2: float = 0.0, tgate: float = 0.0):
    """The Kraus operators (2x2 complex128) of one of the paper's channels."""
    if kind == "damping":
        return _damping(p)
    if kind in ("dephasing", "phase_flip"):
        return _dephasing(p)
    if kind == "decoherence":
        # paper: p_damping = 1 - exp(-tgate/T1),
        # p_dephasing = (1 - exp(-(tgate/T2 - tgate/(2 T1)))) / 2, and the four
        # products K_a(damping) K_b(dephasing)
        pd = 1.0 - math.exp(-tgate / t1)
        pf = 0.5 * (1.0 - math.exp(-(tgate / t2 - tgate / (2.0 * t1))))
        D, F = _damping(pd), _dephasing(pf)
        return [D[0] @ F[0], D[0] @ F[1], D[1] @ F[0], D[1] @ F[1]]
    if kind == "depolarizing":
        # paper: sqrt(1 - 3p/4) I, sqrt(p)/2 X, sqrt(p)/2 Y, sqrt(p)/2 Z
        h = math.sqrt(p) / 2
        return [math.sqrt(1 - 3 * p / 4) * _I, h * _X, h * _Y, h * _Z]
    if kind == "bit_phase_flip":
        # paper's "bit or phase flip": sqrt(1-p) I, [[0, -i sqrt(p)], [i sqrt(p), 0]]
        return [math.sqrt(1 - p) * _I,
                np.array([[0, -1j * math.sqrt(p)], [1j * math.sqrt(p), 0]], dtype=np.complex128)]
    if kind == "bit_flip":
        return [math.sqrt(1 - p) * _I, math.sqrt(p) * _X]
    if kind == "phase_damping":
        # paper: K1 = [[1, 0], [0, sqrt(1-p)]], K2 = [[0, 0], [0, sqrt(p)]]
        return [np.array([[1, 0], [0, math.sqrt(1 - p)]], dtype=np.complex128),
                np.array([[0, 0], [0, math.sqrt(p)]], dtype=np.complex128)]
    raise ValueError(f"unknown channel {kind!r}")


def branch_weights(psi: np.ndarray, n: int, q: int, ops) -> np.ndarray:
    """||K_i psi||^2 for every operator, each applied to a copy of psi."""
    w = np.zeros(len(ops))
    for i, K in enumerate(ops):
        phi = psi.copy()
        apply_matrix(phi, n, K, [q])
        w[i] = float(np.vdot(phi, phi).real)
    return w


def trajectory_step(psi: np.ndarray, n: int, q: int, ops, u: float):
    """One branching of the channel on qubit q: returns (new state, branch,
    distance of u * total from the nearest cumulative boundary / total)."""
    w = branch_weights(psi, n, q, ops)
    total = float(w.sum())
    cum = np.cumsum(w)
    j = int(np.argmax(cum > u * total)) if np.any(cum > u * total) else len(ops) - 1
    margin = float(np.min(np.abs(cum[:-1] - u * total))) / total if len(ops) > 1 else 1.0
    phi = psi.copy()
    apply_matrix(phi, n, ops[j], [q])
    phi *= math.sqrt(total / w[j])
    return phi, j, margin


def gate_type(g) -> str:
    """The gate type a noise model names: controlled X / Z / P with one
    control are cnot / cz / cr, X with two controls is toffoli, any other
    gate its own name (an X with a control is not an "x")."""
    c = len(g.controls)
    if g.name == "x" and c in (1, 2):
        return "cnot" if c == 1 else "toffoli"
    if g.name in ("z", "p") and c == 1:
        return "cz" if g.name == "z" else "cr"
    return g.name if c == 0 else f"{g.name}+{c}c"


def noisy_run(n: int, gates, model, uniforms, init: int = 0):
    """A circuit with noise: after every gate whose type the model names,
    that entry's channel acts on each qubit the gate touches (targets, then
    controls), each branching consuming the next uniform.  model: list of
    (gate type, channel kind, parameters dict).  Returns (state, branches,
    margins)."""
    psi = basis_state(n, init)
    branches, margins = [], []
    k = 0
    for g in gates:
        apply_gates(psi, n, [g])
        for name, kind, params in model:
            if name != gate_type(g):
                continue
            ops = kraus(kind, **params)
            for q in tuple(g.targets) + tuple(g.controls):
                psi, j, m = trajectory_step(psi, n, q, ops, float(uniforms[k]))
                k += 1
                branches.append(j)
                margins.append(m)
    return psi, branches, margins


def channel(rho: np.ndarray, n: int, q: int, ops) -> np.ndarray:
    """sum_i K_i rho K_i^dag for the channel on qubit q of an n-qubit density
    matrix (2^n x 2^n, index = basis state)."""
    out = np.zeros_like(rho)
    for K in ops:
        A = rho.copy()
        for c in range(A.shape[1]):              # K acting on the row index
            col = np.ascontiguousarray(A[:, c])
            apply_matrix(col, n, K, [q])
            A[:, c] = col
        A = A.conj().T                           # (K rho)^dag = rho K^dag
        for c in range(A.shape[1]):
            col = np.ascontiguousarray(A[:, c])
            apply_matrix(col, n, K, [q])
            A[:, c] = col
        out += A.conj().T                        # K rho K^dag
    return out
