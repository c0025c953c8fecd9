"""Seeded circuit and observable generators.

Gate names follow the paper's gate set (H, X, Y, Z, S, T, RX, RY, RZ, U3,
CNOT, CZ, CR, Toffoli, arbitrary unitaries; paper, "Structure of QPanda" and
"Performance of basic gates"), written in a canonical controlled form:

    CNOT(c, t)       -> Gate("x",  (t,),  (c,))
    CZ(a, b)         -> Gate("z",  (b,),  (a,))
    CR(c, t, theta)  -> Gate("p",  (t,),  (c,), (theta,))
    Toffoli(a, b, t) -> Gate("x",  (t,),  (a, b))

Other names: "h", "y", "s", "t", "rx", "ry", "rz" (one angle), "u3" (three
angles, OpenQASM 2 form), "rzz" (one angle, two targets), "swap" (two
targets) and "unitary" (explicit 2^k x 2^k matrix, k = len(targets)).
Qubit q is bit q of the amplitude index.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Optional, Sequence

import numpy as np

TWO_PI = 2.0 * math.pi


@dataclass(frozen=True)
class Gate:
    name: str
    targets: tuple
    controls: tuple = ()
    params: tuple = ()
    pidx: int = -1                 # parameter index for trainable rotations
    matrix: Optional[np.ndarray] = field(default=None, compare=False)

    def qubits(self):
        return tuple(self.targets) + tuple(self.controls)


def qubits_of(gates: Sequence[Gate]) -> set:
    out = set()
    for g in gates:
        out.update(g.qubits())
    return out


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def uniform_stream(seed: int, count: int) -> np.ndarray:
    """Uniforms in [0, 1) for sampling, drawn once from the seed."""
    return _rng(seed).random(count)


def noisy_layers(n: int, layers: int, seed: int):
    """Layers of RY and RZ on every qubit (seeded angles), then a brick of
    CNOTs and CZs, then one H on a random qubit: every gate type a noise
    model usually names occurs many times."""
    rng = _rng(seed)
    g = []
    for l in range(layers):
        for q in range(n):
            g.append(Gate("ry", (q,), (), (float(rng.uniform(0, TWO_PI)),)))
            g.append(Gate("rz", (q,), (), (float(rng.uniform(0, TWO_PI)),)))
        for q in range(l % 2, n - 1, 2):
            g.append(Gate("x", (q + 1,), (q,)) if (q // 2 + l) % 2 == 0 else Gate("z", (q + 1,), (q,)))
        g.append(Gate("h", (int(rng.integers(0, n)),)))
    return g


def _cz_brick(n: int, layer: int):
    start = 0 if layer % 2 == 0 else 1
    return [Gate("z", (i + 1,), (i,)) for i in range(start, n - 1, 2)]


def layered_u3_cz(n: int, depth: int, seed: int, rng=None):
    """`depth` layers of U3(theta, phi, lambda) on every qubit, angles
    uniform in [0, 2pi), each followed by a CZ brick on (i, i+1): even i on
    even layers, odd i on odd layers."""
    rng = rng if rng is not None else _rng(seed)
    gates = []
    for layer in range(depth):
        ang = rng.random((n, 3)) * TWO_PI
        for q in range(n):
            gates.append(Gate("u3", (q,), (), tuple(float(a) for a in ang[q])))
        gates.extend(_cz_brick(n, layer))
    return gates


def qft_circuit(n: int, with_swaps: bool = True):
    """Quantum Fourier transform with qubit 0 as the least significant bit:
    for j = n-1 .. 0: H(q_j), then CR(pi / 2^(j-m)) controlled by q_m on
    q_j for m = j-1 .. 0; finally SWAP(q_i, q_{n-1-i}) for i < n/2.
    On |x> it yields N^{-1/2} sum_y exp(2 pi i x y / N) |y>."""
    gates = []
    for j in range(n - 1, -1, -1):
        gates.append(Gate("h", (j,)))
        for m in range(j - 1, -1, -1):
            gates.append(Gate("p", (j,), (m,), (math.pi / float(2 ** (j - m)),)))
    if with_swaps:
        for i in range(n // 2):
            gates.append(Gate("swap", (i, n - 1 - i)))
    return gates


def qft_then_brick(n: int, layers: int, seed: int):
    """Fused-path workload: a seeded random basis state |x>, the QFT, then
    `layers` of U3 + CZ brick.  Returns (x, gates)."""
    rng = _rng(seed)
    x = int(rng.integers(0, 2 ** n))
    gates = qft_circuit(n) + layered_u3_cz(n, layers, seed, rng=rng)
    return x, gates


def hardware_efficient_ansatz(n: int, layers: int):
    """Per layer: RY on every qubit, RZ on every qubit, CNOT(i -> i+1) for
    i = 0..n-2.  Parameter index = 2n*layer + n*[RZ] + qubit."""
    gates = []
    for layer in range(layers):
        for q in range(n):
            gates.append(Gate("ry", (q,), (), (0.0,), pidx=2 * n * layer + q))
        for q in range(n):
            gates.append(Gate("rz", (q,), (), (0.0,), pidx=2 * n * layer + n + q))
        for q in range(n - 1):
            gates.append(Gate("x", (q + 1,), (q,)))
    return gates, 2 * n * layers


def random_pauli_sum(n: int, terms: int, seed: int, wmin=2, wmax=4):
    """`terms` Pauli strings with weight uniform in {wmin..wmax}, distinct
    uniform qubits, letters uniform in {X, Y, Z}, N(0,1) coefficients.
    Returns (x_masks, z_masks, coeffs, labels) in symplectic form."""
    rng = _rng(seed)
    xs, zs, cs, labels = [], [], [], []
    for _ in range(terms):
        w = int(rng.integers(wmin, wmax + 1))
        qs = rng.choice(n, size=w, replace=False)
        letters = rng.integers(0, 3, size=w)
        x = z = 0
        lab = []
        for q, l in zip(qs, letters):
            q = int(q)
            if l == 0:
                x |= 1 << q
                lab.append(f"X{q}")
            elif l == 1:
                x |= 1 << q
                z |= 1 << q
                lab.append(f"Y{q}")
            else:
                z |= 1 << q
                lab.append(f"Z{q}")
        xs.append(x)
        zs.append(z)
        cs.append(float(rng.standard_normal()))
        labels.append(" ".join(lab))
    return (np.array(xs, dtype=np.uint64), np.array(zs, dtype=np.uint64),
            np.array(cs, dtype=np.float64), labels)


PLANNER_GATESET = ("h", "t", "rx", "rz", "rzz", "cnot", "cz", "toffoli")


def random_planner_circuit(seed: int, n_range=(26, 32), g_range=(100, 500),
                           n: Optional[int] = None, ngates: Optional[int] = None):
    """Learned-planner workload: n ~ U{26..32}, gate count ~ U{100..500},
    gate type uniform over {H, T, RX, RZ, RZZ, CNOT, CZ, Toffoli}, distinct
    uniform qubits, angles uniform in [0, 2pi).  Returns (n, gates)."""
    rng = _rng(seed)
    nn = int(rng.integers(n_range[0], n_range[1] + 1))
    gg = int(rng.integers(g_range[0], g_range[1] + 1))
    if n is not None:
        nn = n
    if ngates is not None:
        gg = ngates
    gates = []
    for _ in range(gg):
        kind = PLANNER_GATESET[int(rng.integers(0, len(PLANNER_GATESET)))]
        if kind in ("h", "t"):
            q = int(rng.integers(0, nn))
            gates.append(Gate(kind, (q,)))
        elif kind in ("rx", "rz"):
            q = int(rng.integers(0, nn))
            gates.append(Gate(kind, (q,), (), (float(rng.random() * TWO_PI),)))
        elif kind == "rzz":
            a, b = (int(v) for v in rng.choice(nn, size=2, replace=False))
            gates.append(Gate("rzz", (a, b), (), (float(rng.random() * TWO_PI),)))
        elif kind == "cnot":
            c, t = (int(v) for v in rng.choice(nn, size=2, replace=False))
            gates.append(Gate("x", (t,), (c,)))
        elif kind == "cz":
            a, b = (int(v) for v in rng.choice(nn, size=2, replace=False))
            gates.append(Gate("z", (b,), (a,)))
        else:
            a, b, t = (int(v) for v in rng.choice(nn, size=3, replace=False))
            gates.append(Gate("x", (t,), (a, b)))
    return nn, gates


PLANNER_FAMILIES = ("random", "random_long", "layered", "qft", "rotation_cnot")


def planner_mix_circuit(seed: int):
    """Training circuits for the cost model: a seeded mixture of circuit
    families so that pass shapes cover what users run, not only the random
    gate soup.  Family (by seed): random 100-500 gates (45%), random
    500-1,500 gates (15%), U3 + CZ brick of depth 4-40 (20%), QFT followed
    by a brick of depth 0-20 (10%), rotation + cyclic CNOT layers, 2-12 of
    them (10%); n ~ U{26..32} for the short random circuits and U{26..30}
    for the others (their passes are long; the qubit count is a feature, so
    the model still sees its scaling).  Returns (n, gates, family)."""
    rng = _rng(seed)
    u = rng.random()
    sub = int(rng.integers(0, 2 ** 31))
    if u < 0.45:
        n, gates = random_planner_circuit(sub)
        return n, gates, "random"
    if u < 0.60:
        n, gates = random_planner_circuit(sub, n_range=(26, 30), g_range=(500, 1500))
        return n, gates, "random_long"
    n = int(rng.integers(26, 31))
    if u < 0.80:
        return n, layered_u3_cz(n, int(rng.integers(4, 41)), sub), "layered"
    if u < 0.90:
        gates = qft_circuit(n) + layered_u3_cz(n, int(rng.integers(0, 21)), sub)
        return n, gates, "qft"
    return n, rotation_cnot_circuit(n, int(rng.integers(2, 13)), sub), "rotation_cnot"


def _random_unitary(rng, dim):
    z = rng.standard_normal((dim, dim)) + 1j * rng.standard_normal((dim, dim))
    q, r = np.linalg.qr(z)
    d = np.diag(r)
    return q * (d / np.abs(d))


ONE_Q = ("h", "x", "y", "z", "s", "t", "rx", "ry", "rz", "u3", "p")


def random_mixed_circuit(n: int, ngates: int, seed: int, kmax: int = 3,
                         max_ctrl: int = 2, names: Sequence[str] = None):
    """Random gates of every kind used by the tests: named one-qubit gates,
    rzz, swap and explicit unitaries on up to `kmax` targets, each with up
    to `max_ctrl` random controls."""
    rng = _rng(seed)
    kinds = list(names) if names else list(ONE_Q) + ["rzz", "swap", "unitary"]
    gates = []
    for _ in range(ngates):
        kind = kinds[int(rng.integers(0, len(kinds)))]
        if kind == "unitary":
            k = int(rng.integers(1, min(kmax, n) + 1))
        elif kind in ("rzz", "swap"):
            k = 2
        else:
            k = 1
        if k > n:
            continue
        nc = int(rng.integers(0, min(max_ctrl, n - k) + 1))
        qs = [int(v) for v in rng.choice(n, size=k + nc, replace=False)]
        tg, ct = tuple(qs[:k]), tuple(qs[k:])
        if kind == "unitary":
            gates.append(Gate("unitary", tg, ct, (), -1, _random_unitary(rng, 2 ** k)))
        elif kind in ("rx", "ry", "rz", "p", "rzz"):
            gates.append(Gate(kind, tg, ct, (float(rng.random() * TWO_PI),)))
        elif kind == "u3":
            gates.append(Gate(kind, tg, ct, tuple(float(a) for a in rng.random(3) * TWO_PI)))
        else:
            gates.append(Gate(kind, tg, ct))
    return gates


def ghz_circuit(n: int):
    """H(0), then CNOT(q -> q+1) for q = 0..n-2."""
    return [Gate("h", (0,))] + [Gate("x", (q + 1,), (q,)) for q in range(n - 1)]


def w_circuit(n: int):
    """X(0); for k = 0..n-2: RY(2 arccos(1/sqrt(n-k))) on q_{k+1} controlled
    by q_k, then CNOT(q_{k+1} -> q_k).  Gives amplitude 1/sqrt(n) on every
    weight-one basis state."""
    gates = [Gate("x", (0,))]
    for k in range(n - 1):
        th = 2.0 * math.acos(1.0 / math.sqrt(n - k))
        gates.append(Gate("ry", (k + 1,), (k,), (th,)))
        gates.append(Gate("x", (k,), (k + 1,)))
    return gates


def rotation_cnot_circuit(n: int, layers: int, seed: int):
    """The paper's comparison circuit shape: a rotation layer (RX, RY, RZ
    on every qubit, seeded angles) and a CNOT layer with target i and
    control (i+1) mod n, repeated `layers` times from |0>."""
    rng = _rng(seed)
    gates = []
    for _ in range(layers):
        ang = rng.random((n, 3)) * TWO_PI
        for q in range(n):
            gates.append(Gate("rx", (q,), (), (float(ang[q, 0]),)))
            gates.append(Gate("ry", (q,), (), (float(ang[q, 1]),)))
            gates.append(Gate("rz", (q,), (), (float(ang[q, 2]),)))
        for i in range(n):
            gates.append(Gate("x", (i,), ((i + 1) % n,)))
    return gates


# Seeds fixed per workload so that every consumer regenerates the same input.
SEEDS = {"layered12": 1201, "layered28": 2801, "qft30": 3001,
         "hea20": 2001, "pauli20": 2002, "planner": 5000, "samples28": 2803}


def config_circuit(name: str):
    """The named workloads at full size: returns a dict describing them."""
    if name == "layered12":
        return {"n": 12, "init": 0, "gates": layered_u3_cz(12, 20, SEEDS[name])}
    if name == "layered28":
        return {"n": 28, "init": 0, "gates": layered_u3_cz(28, 40, SEEDS[name]),
                "uniforms": uniform_stream(SEEDS["samples28"], 1024)}
    if name == "qft30":
        x, gates = qft_then_brick(30, 30, SEEDS[name])
        return {"n": 30, "init": x, "gates": gates}
    raise KeyError(name)


def mlp_init(d: int, hidden: int, seed: int):
    """Seeded initial weights for the three-layer cost-model MLP (He-normal
    for the ReLU layers), as float64 arrays [W1 (d,H), b1, W2 (H,H), b2,
    W3 (H,1), b3]."""
    rng = _rng(seed)
    W1 = rng.standard_normal((d, hidden)) * math.sqrt(2.0 / d)
    W2 = rng.standard_normal((hidden, hidden)) * math.sqrt(2.0 / hidden)
    W3 = rng.standard_normal((hidden, 1)) * math.sqrt(1.0 / hidden)
    return [W1, np.zeros(hidden), W2, np.zeros(hidden), W3, np.zeros(1)]
