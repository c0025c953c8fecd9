"""The full-size complex64 checks can fail: on the CPU, with the FP64 oracle
alone, a state that misses one gate of the workload's circuit fails each of
them.

The full-size tests compare the GPU's complex64 state with stored oracle
values by (a) the relative 2-norm error over a gathered set of amplitudes,
(b) <Z_q> within 2 tau + tau^2 and (c) samples inside the CDF window widened
by the stated cumulative-probability bound, all with the tau of the largest
full-size plan.  Here the oracle's own result with one gate dropped stands
in for a wrong GPU result, on the same generators at 14 qubits (the full
sizes take the oracle minutes per run): for gates spread over the circuit
and covering every gate kind, (a) and (b) fail by orders of magnitude and
(c) rejects some of the samples.
"""
import numpy as np
import pytest

import oracle
from tests.util import c64_bound, cdf_eps, cdf_window, gate_ks
from workloads import config_circuit, layered_u3_cz, qft_then_brick, uniform_stream


def full_size_tau():
    """The largest tau any full-size complex64 check uses: the plain path on
    the 28-qubit workload (one pass per gate)."""
    return c64_bound(gate_ks(config_circuit("layered28")["gates"]))


def rel2(got, want):
    return float(np.linalg.norm(got - want) / np.linalg.norm(want))


def dropped_indices(gates, count):
    """Gate indices spread evenly over the circuit plus the first gate of
    every kind."""
    idx = set(np.linspace(0, len(gates) - 1, count).astype(int).tolist())
    seen = {}
    for i, g in enumerate(gates):
        seen.setdefault((g.name, len(g.controls)), i)
    return sorted(idx | set(seen.values()))


@pytest.mark.parametrize("family", ["layered", "qft_brick"])
def test_missing_gate_fails_full_size_checks(family):
    """For every dropped gate whose effect on the state is above the stated
    bound (2-norm change > 10 tau), the sampled amplitude check fails; for
    every one that changes the probabilities by more than 100 eps in total
    variation, the <Z> check fails and some samples leave the CDF window.
    Gates below those sizes (diagonal gates at the end of the circuit leave
    every probability unchanged; the QFT's controlled phases of angle
    pi/2^13 change the state by ~5e-4) are counted, and must be few; gates
    that are the identity on their input (a controlled phase whose control
    is still a 0 basis bit) change nothing any check could see."""
    n = 14
    if family == "layered":
        x, gates = 0, layered_u3_cz(n, 40, 2801)
    else:
        x, gates = qft_then_brick(n, 30, 3001)
    tau = full_size_tau()
    assert 1e-5 < tau < 1e-4
    rng = np.random.Generator(np.random.PCG64(14))
    S = rng.integers(0, 1 << n, 2048)
    u = uniform_stream(2803, 1024)
    psi = oracle.run_packed(n, gates, x)
    p = oracle.probabilities(psi)
    z = oracle.expect_z_all(psi)
    cdf = np.cumsum(p)
    eps = cdf_eps(tau)
    # the reference passes its own checks
    ok, _ = cdf_window(oracle.sample(psi, u)[0], cdf, u, eps)
    assert ok.all()
    small_amp, small_prob, identity, tested = [], [], [], 0
    for j in dropped_indices(gates, 60):
        bad = oracle.run_packed(n, gates[:j] + gates[j + 1:], x)
        tested += 1
        change = float(np.linalg.norm(bad - psi))
        if change < 1e-12:
            # a controlled phase whose control is still a 0 basis bit (the
            # QFT on a basis state): the gate is the identity on its input
            assert oracle.is_diagonal(gates[j]), (j, gates[j])
            identity.append(j)
            continue
        if change > 10 * tau:
            r2 = rel2(bad[S], psi[S])
            assert r2 > tau, (j, gates[j], r2)
        else:
            small_amp.append(j)
        if np.sum(np.abs(oracle.probabilities(bad) - p)) > 100 * eps:
            dz = float(np.max(np.abs(oracle.expect_z_all(bad) - z)))
            assert dz > 2 * tau + tau * tau, (j, gates[j], dz)
            ok, _ = cdf_window(oracle.sample(bad, u)[0], cdf, u, eps)
            assert not ok.all(), (j, gates[j])
        else:
            small_prob.append(j)
    print(f"{family}: tau {tau:.1e}, eps {eps:.1e}; {tested} dropped gates; below the amplitude "
          f"bound: {[str(gates[j].name) + str(gates[j].targets) for j in small_amp]}; "
          f"probabilities unchanged within 100 eps: {len(small_prob)}; identity on their input: "
          f"{len(identity)}")
    assert len(small_amp) <= 3 and len(small_prob) <= 12
