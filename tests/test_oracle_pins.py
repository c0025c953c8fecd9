"""Pins for the FP64 oracle against facts fixed outside it.

The paper prints no gate matrices, amplitudes, probabilities or expectation
values for the full-amplitude path, so every pin here is mathematical:
library routines (matrix exponential, FFT, tensor contraction), closed forms
(GHZ, W, QFT), invariants (unitarity, norm, inverse circuits) and exact
identities (parameter shift, the sin(h)/h law of central differences on a
sinusoid).  Each test is chosen so that a plausible slip in the oracle
(a transposed operand, a wrong sign or bit index, a dropped term) fails it.
"""
import math

import numpy as np
import pytest
import scipy.linalg

import oracle
from workloads import (Gate, ghz_circuit, w_circuit, qft_circuit,
                       random_mixed_circuit, layered_u3_cz,
                       hardware_efficient_ansatz, random_pauli_sum)

X = np.array([[0, 1], [1, 0]], dtype=complex)
Y = np.array([[0, -1j], [1j, 0]], dtype=complex)
Z = np.array([[1, 0], [0, -1]], dtype=complex)
I2 = np.eye(2, dtype=complex)


# ---------------------------------------------------------------- matrices
@pytest.mark.parametrize("name,G", [("rx", X), ("ry", Y), ("rz", Z)])
def test_rotations_are_exponentials(name, G):
    for th in np.linspace(-7, 7, 11):
        got = oracle.gate_matrix(Gate(name, (0,), (), (th,)))
        assert np.allclose(got, scipy.linalg.expm(-0.5j * th * G), atol=1e-14)


def test_rzz_is_exponential():
    for th in (0.3, 2.0, -5.0):
        got = oracle.gate_matrix(Gate("rzz", (0, 1), (), (th,)))
        assert np.allclose(got, scipy.linalg.expm(-0.5j * th * np.kron(Z, Z)), atol=1e-14)


def test_fixed_gates():
    m = lambda n: oracle.gate_matrix(Gate(n, (0,)))
    H = m("h")
    assert np.allclose(H @ H, I2)
    assert np.allclose(H @ Z @ H, X)
    assert np.allclose(m("x"), X) and np.allclose(m("y"), Y) and np.allclose(m("z"), Z)
    assert np.allclose(m("s") @ m("s"), Z)
    assert np.allclose(m("t") @ m("t"), m("s"))
    assert np.allclose(m("sdg") @ m("s"), I2) and np.allclose(m("tdg") @ m("t"), I2)
    sw = oracle.gate_matrix(Gate("swap", (0, 1)))
    # SWAP exchanges |01> and |10> (bit r of the index <-> targets[r])
    e = np.eye(4)
    assert np.allclose(sw @ e[:, 1], e[:, 2]) and np.allclose(sw @ e[:, 2], e[:, 1])


def test_u3_decomposition():
    # OpenQASM 2: U3(t, p, l) = e^{i(p+l)/2} RZ(p) RY(t) RZ(l)
    rng = np.random.default_rng(7)
    for _ in range(10):
        t, p, l = rng.uniform(-7, 7, 3)
        got = oracle.gate_matrix(Gate("u3", (0,), (), (t, p, l)))
        rz = lambda a: scipy.linalg.expm(-0.5j * a * Z)
        ry = scipy.linalg.expm(-0.5j * t * Y)
        assert np.allclose(got, np.exp(0.5j * (p + l)) * rz(p) @ ry @ rz(l), atol=1e-13)
    # phase gate P(t) = e^{it/2} RZ(t)
    got = oracle.gate_matrix(Gate("p", (0,), (), (0.7,)))
    assert np.allclose(got, np.exp(0.35j) * scipy.linalg.expm(-0.35j * Z))


# ------------------------------------------------------- gate application
def tensor_apply(psi, n, U, targets, controls):
    """Independent reference: view the state as an n-axis tensor (axis a is
    qubit n-1-a in C order), contract U on the target axes, and restrict to
    the slice where every control axis is 1."""
    T = psi.reshape((2,) * n).copy()
    ax = lambda q: n - 1 - q
    k = len(targets)
    sl = [slice(None)] * n
    for c in controls:
        sl[ax(c)] = 1
    sub = T[tuple(sl)]
    # axes of `sub` after removing control axes
    rem = [a for a in range(n) if a not in {ax(c) for c in controls}]
    tax = [rem.index(ax(t)) for t in targets]
    # U acts on the combined index j = sum_r bit_r 2^r with bit r <-> targets[r]
    Ut = U.reshape((2,) * (2 * k))            # row bits then col bits, MSB first
    # Ut axes: out bits (k-1..0), in bits (k-1..0); target r <-> bit r
    in_axes = [2 * k - 1 - r for r in range(k)]
    out_axes = [k - 1 - r for r in range(k)]
    res = np.tensordot(Ut, sub, axes=(in_axes, tax))
    # res axes: out bits (k-1..0 order as in Ut) followed by remaining sub axes
    rest = [a for a in range(sub.ndim) if a not in tax]
    perm_src = list(range(k)) + list(range(k, k + len(rest)))
    dest = [tax[k - 1 - i] for i in range(k)] + rest
    res = np.moveaxis(res, perm_src, dest)
    T[tuple(sl)] = res
    return T.reshape(-1)


@pytest.mark.parametrize("seed", range(6))
def test_apply_matches_tensor_contraction(seed):
    n = 7
    gates = random_mixed_circuit(n, 40, seed, kmax=3, max_ctrl=2)
    rng = np.random.default_rng(seed)
    psi = rng.standard_normal(1 << n) + 1j * rng.standard_normal(1 << n)
    ref = psi.copy()
    for g in gates:
        oracle.apply_matrix(psi, n, oracle.gate_matrix(g), g.targets, g.controls)
        ref = tensor_apply(ref, n, oracle.gate_matrix(g), g.targets, g.controls)
        assert np.allclose(psi, ref, atol=1e-12), g


def test_apply_full_matrix_kron():
    # single-target uncontrolled gates against the Kronecker product
    n = 5
    rng = np.random.default_rng(3)
    psi = rng.standard_normal(1 << n) + 1j * rng.standard_normal(1 << n)
    for q in range(n):
        U = oracle.gate_matrix(Gate("u3", (q,), (), tuple(rng.uniform(0, 6, 3))))
        ops = [I2] * n
        ops[n - 1 - q] = U          # kron order: most significant qubit first
        full = ops[0]
        for o in ops[1:]:
            full = np.kron(full, o)
        want = full @ psi
        got = psi.copy()
        oracle.apply_matrix(got, n, U, (q,))
        assert np.allclose(got, want, atol=1e-13)


def test_circuit_then_inverse_is_identity():
    n = 6
    gates = random_mixed_circuit(n, 60, 11)
    psi = oracle.simulate(n, gates, init=13)
    for g in reversed(gates):
        oracle.apply_matrix(psi, n, oracle.gate_matrix(g).conj().T, g.targets, g.controls)
    want = np.zeros(1 << n, complex)
    want[13] = 1
    assert np.allclose(psi, want, atol=1e-12)


def test_norm_preserved_and_run_packed_agrees():
    n = 10
    gates = layered_u3_cz(n, 8, 5)
    a = oracle.simulate(n, gates)
    b = oracle.run_packed(n, gates)
    assert np.array_equal(a, b)
    assert abs(oracle.norm2(a) - 1) < 1e-13


# ---------------------------------------------------------- closed forms
@pytest.mark.parametrize("n", [2, 5, 9])
def test_ghz(n):
    psi = oracle.simulate(n, ghz_circuit(n))
    want = np.zeros(1 << n, complex)
    want[0] = want[-1] = 1 / math.sqrt(2)
    assert np.max(np.abs(psi - want)) < 1e-15


@pytest.mark.parametrize("n", [2, 3, 6, 10])
def test_w(n):
    psi = oracle.simulate(n, w_circuit(n))
    want = np.zeros(1 << n, complex)
    for q in range(n):
        want[1 << q] = 1 / math.sqrt(n)
    assert np.max(np.abs(psi - want)) < 1e-14


@pytest.mark.parametrize("n", [3, 6, 10])
def test_qft_is_inverse_fft(n):
    N = 1 << n
    rng = np.random.default_rng(n)
    v = rng.standard_normal(N) + 1j * rng.standard_normal(N)
    v /= np.linalg.norm(v)
    psi = v.copy()
    oracle.apply_gates(psi, n, qft_circuit(n))
    assert np.max(np.abs(psi - math.sqrt(N) * np.fft.ifft(v))) < 1e-13


def test_qft_basis_closed_form():
    n = 12
    N = 1 << n
    x = 2741
    psi = oracle.simulate(n, qft_circuit(n), init=x)
    y = np.arange(N)
    want = np.exp(2j * np.pi * ((x * y) % N) / N) / math.sqrt(N)
    assert np.max(np.abs(psi - want)) < 1e-13


# ------------------------------------------------- readout: probabilities
def test_probabilities_and_marginals():
    n = 8
    psi = oracle.simulate(n, random_mixed_circuit(n, 50, 3))
    p = oracle.probabilities(psi)
    assert np.allclose(p, np.abs(psi) ** 2, atol=1e-16)
    qs = [5, 1, 6]
    m = oracle.marginal(psi, qs)
    # independent: reshape to a tensor and sum the other axes
    T = (np.abs(psi) ** 2).reshape((2,) * n)
    keep = [n - 1 - q for q in qs]
    S = T.sum(axis=tuple(a for a in range(n) if a not in keep))
    # S axes are in increasing axis order; reorder to (q2, q1, q0) MSB-first
    order = sorted(keep)
    S = np.transpose(S, [order.index(a) for a in reversed(keep)])
    assert np.allclose(m, S.reshape(-1), atol=1e-15)
    assert abs(m.sum() - 1) < 1e-14


# --------------------------------------------------- readout: expectation
def pauli_dense(n, x, z):
    ops = []
    for q in range(n - 1, -1, -1):
        bx, bz = (x >> q) & 1, (z >> q) & 1
        ops.append(Y if (bx and bz) else X if bx else Z if bz else I2)
    full = ops[0]
    for o in ops[1:]:
        full = np.kron(full, o)
    return full


def test_pauli_expectation_dense():
    n = 6
    psi = oracle.simulate(n, random_mixed_circuit(n, 40, 9))
    xs, zs, cs, labels = random_pauli_sum(n, 30, 4, wmin=1, wmax=6)
    for x, z in zip(xs, zs):
        want = np.vdot(psi, pauli_dense(n, int(x), int(z)) @ psi)
        re, im = oracle.expect_pauli(psi, int(x), int(z))
        assert abs(re - want.real) < 1e-13 and abs(im) < 1e-13
    lam = oracle.apply_pauli_sum(psi, xs, zs, cs)
    H = sum(c * pauli_dense(n, int(x), int(z)) for x, z, c in zip(xs, zs, cs))
    assert np.allclose(lam, H @ psi, atol=1e-13)


def test_z_expectation_product_state():
    n = 5
    th = np.array([0.1, 1.2, 2.3, -0.7, 3.0])
    gates = [Gate("ry", (q,), (), (float(th[q]),)) for q in range(n)]
    psi = oracle.simulate(n, gates)
    assert np.allclose(oracle.expect_z_all(psi), np.cos(th), atol=1e-14)
    # <X_q> = sin(theta_q) and <Y_q> = 0 for RY on |0>
    for q in range(n):
        assert abs(oracle.expect_pauli(psi, 1 << q, 0)[0] - math.sin(th[q])) < 1e-14
        assert abs(oracle.expect_pauli(psi, 1 << q, 1 << q)[0]) < 1e-14
    zz = oracle.expect_zz(psi, [(0, 1), (3, 4)])
    assert np.allclose(zz, [math.cos(th[0]) * math.cos(th[1]), math.cos(th[3]) * math.cos(th[4])])


# ------------------------------------------------------------- sampling
def test_sampling_matches_searchsorted():
    n = 9
    psi = oracle.simulate(n, random_mixed_circuit(n, 40, 2))
    u = np.random.default_rng(0).random(2000)
    idx, margin = oracle.sample(psi, u)
    cdf = np.cumsum(np.abs(psi) ** 2)
    ref = np.searchsorted(cdf, u * cdf[-1], side="right")
    close = margin < 1e-12
    assert np.array_equal(idx[~close], ref[~close])
    assert np.all(np.abs(idx[close].astype(np.int64) - ref[close]) <= 1)


def test_sampling_chi_square():
    n = 6
    psi = oracle.simulate(n, random_mixed_circuit(n, 30, 8))
    p = np.abs(psi) ** 2
    u = np.random.default_rng(1).random(100000)
    idx, _ = oracle.sample(psi, u)
    counts = np.bincount(idx.astype(np.int64), minlength=1 << n)
    exp = p * u.size
    mask = exp > 5
    chi2 = np.sum((counts[mask] - exp[mask]) ** 2 / exp[mask])
    dof = mask.sum() - 1
    p_value = 1 - scipy.stats.chi2.cdf(chi2, dof)
    assert p_value > 1e-4


# ------------------------------------------------------------- adjoint
def _hea_problem(n=4, layers=3, seed=0):
    gates, P = hardware_efficient_ansatz(n, layers)
    xs, zs, cs, _ = random_pauli_sum(n, 6, seed + 100)
    th = np.random.default_rng(seed).uniform(0, 2 * math.pi, P)
    return gates, P, xs, zs, cs, th


def test_adjoint_matches_parameter_shift():
    n = 4
    gates, P, xs, zs, cs, th = _hea_problem(n)
    f, g = oracle.adjoint(n, gates, th, xs, zs, cs)
    assert abs(f - oracle.energy(n, gates, th, xs, zs, cs)) < 1e-13
    for p in range(P):
        tp, tm = th.copy(), th.copy()
        tp[p] += math.pi / 2
        tm[p] -= math.pi / 2
        ps = 0.5 * (oracle.energy(n, gates, tp, xs, zs, cs) - oracle.energy(n, gates, tm, xs, zs, cs))
        assert abs(g[p] - ps) < 1e-12


def test_adjoint_matches_central_difference_sinusoid_law():
    # along one coordinate f = A cos t + B sin t + C, so the central
    # difference with step h equals f'(t) sin(h)/h exactly
    n = 5
    gates, P, xs, zs, cs, th = _hea_problem(n, 2, seed=3)
    f, g = oracle.adjoint(n, gates, th, xs, zs, cs)
    h = 1e-3
    scale = np.sum(np.abs(cs))
    for p in range(0, P, 3):
        tp, tm = th.copy(), th.copy()
        tp[p] += h
        tm[p] -= h
        fd = (oracle.energy(n, gates, tp, xs, zs, cs) - oracle.energy(n, gates, tm, xs, zs, cs)) / (2 * h)
        assert abs(fd / (math.sin(h) / h) - g[p]) < 1e-9 * scale


def test_adjoint_controlled_rotation():
    n = 3
    gates = [Gate("h", (0,)), Gate("h", (1,)),
             Gate("ry", (2,), (0,), (0.0,), pidx=0), Gate("rx", (1,), (2,), (0.0,), pidx=1),
             Gate("rz", (0,), (1, 2), (0.0,), pidx=2)]
    xs = np.array([0b100, 0b011], np.uint64)
    zs = np.array([0b001, 0b110], np.uint64)
    cs = np.array([0.8, -1.3])
    th = np.array([0.7, 1.9, -2.2])
    f, g = oracle.adjoint(n, gates, th, xs, zs, cs)
    for p in range(3):
        tp, tm = th.copy(), th.copy()
        tp[p] += math.pi / 2
        tm[p] -= math.pi / 2
        # a controlled rotation is not a pure sinusoid of period 2pi with the
        # shift rule, so compare with a high-order central difference instead
        h = 1e-4
        t1, t2 = th.copy(), th.copy()
        t1[p] += h
        t2[p] -= h
        fd = (oracle.energy(n, gates, t1, xs, zs, cs) - oracle.energy(n, gates, t2, xs, zs, cs)) / (2 * h)
        assert abs(fd - g[p]) < 1e-7


# ------------------------------------------------------------- fusion
def test_block_matrix_equals_unfused():
    n = 7
    gates = random_mixed_circuit(n, 30, 21, kmax=2, max_ctrl=1)
    qs = sorted({q for g in gates[:6] for q in g.qubits()})
    M = oracle.block_matrix(gates[:6], qs)
    assert np.allclose(M @ M.conj().T, np.eye(M.shape[0]), atol=1e-12)
    rng = np.random.default_rng(0)
    psi = rng.standard_normal(1 << n) + 1j * rng.standard_normal(1 << n)
    a = psi.copy()
    oracle.apply_gates(a, n, gates[:6])
    b = psi.copy()
    oracle.apply_matrix(b, n, M, qs)
    assert np.allclose(a, b, atol=1e-12)


def test_plan_validator():
    gates = [Gate("h", (0,)), Gate("x", (1,), (0,)), Gate("h", (2,)), Gate("z", (2,), (1,))]
    assert oracle.validate_plan(gates, [[0, 1], [2, 3]], 3)[0]
    assert oracle.validate_plan(gates, [[2], [0, 1], [3]], 2)[0]
    assert not oracle.validate_plan(gates, [[1, 0], [2, 3]], 3)[0]      # order on qubit 0
    assert not oracle.validate_plan(gates, [[0, 1, 2, 3]], 2)[0]        # too wide
    assert not oracle.validate_plan(gates, [[0, 1], [3]], 3)[0]         # gate missing
    assert not oracle.validate_plan(gates, [[3], [0, 1, 2]], 3)[0]      # z before h on qubit 2


def test_plan_validator_diagonal_commutation():
    """Diagonal gates may trade places between the same non-diagonal gates;
    every order the validator accepts gives the program-order state (brute
    force over random orders of small circuits rich in diagonal gates)."""
    g = [Gate("h", (0,)), Gate("z", (1,), (0,)), Gate("rz", (1,), (), (0.4,)), Gate("t", (0,)),
         Gate("x", (1,))]
    assert oracle.validate_plan(g, [[0], [3], [2], [1], [4]], 2)[0]
    assert not oracle.validate_plan(g, [[0], [1], [4], [2], [3]], 2)[0]   # x(1) before rz(1)
    assert not oracle.validate_plan(g, [[3], [0], [1], [2], [4]], 2)[0]   # t(0) before h(0)
    assert not oracle.validate_plan(g, [[0], [4], [1], [2], [3]], 2)[0]   # x(1) before cz
    n = 4
    rng = np.random.default_rng(11)
    psi = rng.standard_normal(1 << n) + 1j * rng.standard_normal(1 << n)
    accepted = 0
    for trial in range(30):
        gates = []
        for _ in range(9):
            a, b = (int(v) for v in rng.choice(n, 2, replace=False))
            kind = int(rng.integers(0, 6))
            gates.append([Gate("h", (a,)), Gate("z", (a,), (b,)), Gate("rz", (a,), (), (float(rng.uniform(0, 6)),)),
                          Gate("p", (a,), (b,), (float(rng.uniform(0, 6)),)), Gate("rzz", (a, b), (), (0.7,)),
                          Gate("x", (a,), (b,))][kind])
        want = oracle.apply_gates(psi.copy(), n, gates)
        for _ in range(40):
            perm = [int(v) for v in rng.permutation(len(gates))]
            if not oracle.validate_plan(gates, [[i] for i in perm], n)[0]:
                continue
            accepted += perm != sorted(perm)
            got = oracle.apply_gates(psi.copy(), n, [gates[i] for i in perm])
            assert np.max(np.abs(got - want)) < 1e-12
    assert accepted >= 10


# ------------------------------------------------------------- cost-model MLP
def test_mlp_backward_matches_central_differences():
    from oracle import mlp
    from workloads import mlp_init
    rng = np.random.default_rng(0)
    d, H, B = 5, 7, 9
    params = mlp_init(d, H, 3)
    for p in params:                      # nonzero biases so every term is exercised
        p += 0.1 * rng.standard_normal(p.shape)
    X = rng.standard_normal((B, d))
    t = rng.standard_normal(B)
    L0, grads = mlp.backward(params, X, t)
    assert abs(L0 - mlp.loss(params, X, t)) < 1e-15
    h = 1e-6
    for pi, (p, g) in enumerate(zip(params, grads)):
        flat, gflat = p.reshape(-1), g.reshape(-1)
        for idx in range(0, flat.size, max(1, flat.size // 6)):
            old = flat[idx]
            flat[idx] = old + h
            lp = mlp.loss(params, X, t)
            flat[idx] = old - h
            lm = mlp.loss(params, X, t)
            flat[idx] = old
            assert abs((lp - lm) / (2 * h) - gflat[idx]) < 1e-7 * (1 + abs(gflat[idx])), (pi, idx)


def test_adam_first_step_closed_form():
    # with bias correction the first step moves each parameter by
    # -lr * g / (|g| + eps)
    from oracle import mlp
    rng = np.random.default_rng(1)
    p = [rng.standard_normal(6)]
    g = [rng.standard_normal(6)]
    m, v = [np.zeros(6)], [np.zeros(6)]
    p0 = p[0].copy()
    mlp.adam_step(p, g, m, v, 1, 0.01)
    assert np.allclose(p[0], p0 - 0.01 * g[0] / (np.abs(g[0]) + 1e-8), atol=1e-15)
