"""Kraus trajectories (paper, "Noise simulation method"): the FP64 oracle
pinned to the mathematics of quantum channels, and the product's host-side
channel tables checked against it.

Pins: every Kraus set is complete (sum K^dag K = I); each channel's action on
a density matrix matches its closed form (depolarizing shrinks the Bloch
vector by 1 - p, damping moves population p from |1> to |0>, decoherence
decays the excited population as exp(-t/T1) and the coherence as
exp(-t/T2), ...); enumerating every branch of a trajectory step with its
weight reproduces the channel exactly; deterministic cases (full damping,
zero error rate) give known states.
"""
import math

import numpy as np
import pytest

import oracle
from oracle import noise as onoise
from workloads import Gate, random_mixed_circuit

KINDS = ["damping", "dephasing", "phase_flip", "depolarizing", "bit_phase_flip", "bit_flip",
         "phase_damping"]
DECO = {"t1": 50.0, "t2": 70.0, "tgate": 4.0}


def params(kind, p):
    return dict(DECO) if kind == "decoherence" else {"p": p}


def rand_rho(rng, n=1):
    a = rng.standard_normal((1 << n, 1 << n)) + 1j * rng.standard_normal((1 << n, 1 << n))
    r = a @ a.conj().T
    return r / np.trace(r)


@pytest.mark.parametrize("kind", KINDS + ["decoherence"])
def test_kraus_sets_are_complete(kind):
    for p in (0.0, 0.13, 0.5, 1.0):
        ops = onoise.kraus(kind, **params(kind, p))
        s = sum(K.conj().T @ K for K in ops)
        assert np.allclose(s, np.eye(2), atol=1e-14), (kind, p)


def test_channel_closed_forms():
    rng = np.random.default_rng(3)
    for trial in range(5):
        r = rand_rho(rng)
        p = float(rng.uniform(0.05, 0.95))
        ch = lambda kind, **kw: onoise.channel(r, 1, 0, onoise.kraus(kind, **kw))
        # depolarizing: (1 - p) rho + p I / 2
        assert np.allclose(ch("depolarizing", p=p), (1 - p) * r + p * np.eye(2) / 2, atol=1e-14)
        # amplitude damping
        want = np.array([[r[0, 0] + p * r[1, 1], math.sqrt(1 - p) * r[0, 1]],
                         [math.sqrt(1 - p) * r[1, 0], (1 - p) * r[1, 1]]])
        assert np.allclose(ch("damping", p=p), want, atol=1e-14)
        # dephasing: populations kept, coherences times 1 - 2p
        want = np.array([[r[0, 0], (1 - 2 * p) * r[0, 1]], [(1 - 2 * p) * r[1, 0], r[1, 1]]])
        assert np.allclose(ch("dephasing", p=p), want, atol=1e-14)
        # phase damping: coherences times sqrt(1 - p)
        want = np.array([[r[0, 0], math.sqrt(1 - p) * r[0, 1]],
                         [math.sqrt(1 - p) * r[1, 0], r[1, 1]]])
        assert np.allclose(ch("phase_damping", p=p), want, atol=1e-14)
        # bit flip: (1 - p) rho + p X rho X, X rho X swaps both indices
        assert np.allclose(ch("bit_flip", p=p), (1 - p) * r + p * r[::-1, ::-1], atol=1e-14)
        # bit-phase flip: Y rho Y = [[r11, -r10], [-r01, r00]]
        yry = np.array([[r[1, 1], -r[1, 0]], [-r[0, 1], r[0, 0]]])
        assert np.allclose(ch("bit_phase_flip", p=p), (1 - p) * r + p * yry, atol=1e-14)
        # decoherence: excited population decays as exp(-t/T1), coherence as exp(-t/T2)
        t1, t2, tg = 40.0 + 10 * trial, 55.0 + 5 * trial, 3.0 + trial
        d = ch("decoherence", t1=t1, t2=t2, tgate=tg)
        assert abs(d[1, 1] - math.exp(-tg / t1) * r[1, 1]) < 1e-14
        assert abs(d[0, 1] - math.exp(-tg / t2) * r[0, 1]) < 1e-14
        assert abs(np.trace(d) - 1) < 1e-14


@pytest.mark.parametrize("kind", KINDS + ["decoherence"])
def test_trajectory_branches_reproduce_the_channel(kind):
    """Sum over branches j of (weight_j / total) |psi_j><psi_j| equals the
    channel applied to |psi><psi| (each branch selected by a uniform inside
    its cumulative interval)."""
    n = 3
    rng = np.random.default_rng(11)
    psi = rng.standard_normal(1 << n) + 1j * rng.standard_normal(1 << n)
    psi /= np.linalg.norm(psi)
    ops = onoise.kraus(kind, **params(kind, 0.3))
    for q in range(n):
        w = onoise.branch_weights(psi, n, q, ops)
        cum = np.concatenate([[0.0], np.cumsum(w)])
        total = cum[-1]
        rho = np.zeros((1 << n, 1 << n), complex)
        for j in range(len(ops)):
            if w[j] == 0:
                continue
            u = (cum[j] + 0.5 * w[j]) / total
            phi, jj, _ = onoise.trajectory_step(psi, n, q, ops, u)
            assert jj == j
            assert abs(np.linalg.norm(phi) - 1) < 1e-13
            rho += (w[j] / total) * np.outer(phi, phi.conj())
        want = onoise.channel(np.outer(psi, psi.conj()), n, q, ops)
        assert np.max(np.abs(rho - want)) < 1e-13, (kind, q)


def test_noisy_run_special_cases():
    n = 3
    # full damping after X: every excitation decays, branch K2 every time
    gates = [Gate("x", (q,)) for q in range(n)]
    psi, br, _ = onoise.noisy_run(n, gates, [("x", "damping", {"p": 1.0})], np.full(n, 0.5))
    assert br == [1] * n and abs(psi[0]) == pytest.approx(1.0, abs=1e-15)
    # zero error rate: the noiseless state, the identity branch every time
    gates = random_mixed_circuit(n, 30, 4, kmax=2, max_ctrl=1)
    model = [(onoise.gate_type(g), "depolarizing", {"p": 0.0}) for g in gates]
    u = np.random.default_rng(0).uniform(size=400)
    psi, br, _ = onoise.noisy_run(n, gates, model, u)
    assert set(br) <= {0}
    assert np.allclose(psi, oracle.simulate(n, gates), atol=1e-14)
    # uniforms are consumed per gate, per channel entry, per qubit (targets then controls)
    g = [Gate("x", (1,), (0,))]
    psi, br, _ = onoise.noisy_run(2, g, [("cnot", "bit_flip", {"p": 0.5}),
                                         ("cnot", "bit_flip", {"p": 0.5})], [0.9, 0.1, 0.9, 0.1])
    assert br == [1, 0, 1, 0]
    # an "x" entry does not match a controlled X
    psi, br, _ = onoise.noisy_run(2, g, [("x", "bit_flip", {"p": 0.5})], [])
    assert br == []


def test_product_channel_tables_match_the_oracle():
    """Two independent transcriptions of the paper's equations agree."""
    pytest.importorskip("torch")
    from paper_2212_14201_amd import noise
    for kind in KINDS + ["decoherence"]:
        for p in (0.0, 0.21, 1.0):
            a = noise.kraus_ops(kind, **params(kind, p))
            b = onoise.kraus(kind, **params(kind, p))
            assert len(a) == len(b)
            for x, y in zip(a, b):
                assert np.allclose(x, y, atol=1e-15), kind
    with pytest.raises(ValueError):
        noise.kraus_ops("damping", p=1.5)
    with pytest.raises(ValueError):
        noise.kraus_ops("decoherence", t1=10.0, t2=30.0, tgate=1.0)   # T2 > 2 T1
    with pytest.raises(ValueError):
        noise.kraus_ops("nonsense", p=0.1)


def test_noise_model_counts_branchings():
    pytest.importorskip("torch")
    from paper_2212_14201_amd import noise
    m = noise.NoiseModel([("cz", "depolarizing", {"p": 0.01}), ("h", "damping", {"p": 0.02}),
                          ("cz", "phase_damping", {"p": 0.03}), ("x", "bit_flip", {"p": 0.1})])
    gates = [Gate("h", (0,)), Gate("z", (1,), (0,)), Gate("rx", (2,), (), (0.3,)),
             Gate("x", (2,), (0, 1)), Gate("x", (1,))]
    assert m.branchings(gates) == 1 + 2 * 2 + 0 + 0 + 1
    for g in gates:
        assert noise.gate_type(g) == onoise.gate_type(g)
