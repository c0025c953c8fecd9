"""Full-size parity: the 28-qubit layered workload (plain and fused, both
dtypes) and the 30-qubit QFT + brick workload (in the configuration
bench.py times) against values the FP64 oracle stored in tests/golden/
(written by make_golden.py), and the largest state the library accepts (34
qubits) against the oracle's result on the qubits its circuit touches."""
import json
import math
import os

import numpy as np
import pytest

import oracle
from tests.util import C128_TOL, U32, c64_bound, cdf_eps, cdf_window, gate_ks
from workloads import Gate, config_circuit, random_mixed_circuit

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

qvm = pytest.importorskip("paper_2212_14201_amd.qvm")
HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(autouse=True)
def _gpu(require_gpu):
    pass


def golden(name):
    with open(os.path.join(HERE, "golden", name + ".json")) as fh:
        return json.load(fh)


def plan_bound(plan):
    st = plan.stats()
    s = sum((1 << plan.block(b)["k"]) + 4 for b in range(st["blocks"])) + 5 * st["diag_ops"]
    return 10.0 * math.sqrt(s) * U32


def rel2(got, want):
    """Relative 2-norm error over a gathered set of amplitudes: the stated
    complex64 bound tau bounds the error's 2-norm over the whole (unit)
    state, and rounding errors spread over the amplitudes like the
    amplitudes themselves, so it bounds this ratio too, whereas a single
    amplitude of a 2^28-amplitude state (~2^-14) is below tau."""
    return float(np.linalg.norm(got - want) / np.linalg.norm(want))


def check_samples(got, g, dtype, cdf=None, tau=None):
    """complex128: the oracle's bin except where the target lies within
    1e-12 of a CDF boundary (then a neighbour).  complex64: each sample s
    must satisfy C(s-1) - eps <= u C(N-1) <= C(s) + eps, with C the FP64
    cumulative probability of a reference state and eps = 2 (2 tau + tau^2)
    the stated bound on the cumulative-probability error (sum |dp_i| <=
    2 |dpsi|_2 + |dpsi|_2^2, once for C(s) and once for the total), plus
    1e-12 for the reference's own error."""
    want = np.asarray(g["samples"], dtype=np.int64)
    got = got.astype(np.int64)
    if dtype == "c128":
        close = np.asarray(g["sample_margin"]) <= 1e-12
        assert np.array_equal(got[~close], want[~close])
        assert np.all(np.abs(got[close] - want[close]) <= 1)
        return f"{int(close.sum())} on a CDF boundary"
    eps = cdf_eps(tau) + 1e-12
    ok, slack = cdf_window(got, cdf, np.asarray(g["uniforms"]), eps)
    d = np.abs(got - want)
    assert ok.all(), (int((~ok).sum()), float(slack.min()), eps)
    return (f"all within the CDF window (eps {eps:.1e}, smallest slack {float(slack.min()):.1e}); "
            f"bin distance to the oracle's median {int(np.median(d))}, max {int(d.max())}, "
            f"exact {int(np.sum(d == 0))}")


@pytest.fixture(scope="module")
def cdf28():
    """FP64 cumulative probabilities of the 28-qubit layered workload's state
    from the plain complex128 path, which is first checked against the
    oracle's stored amplitudes, <Z_q> and samples."""
    g = golden("layered28")
    cfg = config_circuit("layered28")
    n = cfg["n"]
    sv = qvm.StateVector(n, "c128", init=0)
    sv.run(cfg["gates"])
    idx = np.asarray(g["amp_index"], dtype=np.uint64)
    want = np.asarray(g["amp_re"]) + 1j * np.asarray(g["amp_im"])
    assert float(np.max(np.abs(sv.gather(idx) - want))) <= C128_TOL
    assert float(np.max(np.abs(sv.expect_z_all() - g["z"]))) <= 1e-12
    check_samples(sv.sample(cfg["uniforms"]), g, "c128")
    c = np.cumsum(sv.probabilities())
    del sv
    return c


@pytest.mark.parametrize("path", ["plain_c128", "plain_c64", "fused_c64", "fused_c128"])
def test_layered_28_qubits(path, request):
    g = dict(golden("layered28"))
    cfg = config_circuit("layered28")
    n, gates = cfg["n"], cfg["gates"]
    g["uniforms"] = cfg["uniforms"]
    dtype = "c128" if path.endswith("c128") else "c64"
    cdf = request.getfixturevalue("cdf28") if dtype == "c64" else None
    print(f"case {path}", flush=True)
    sv = qvm.StateVector(n, dtype, init=0)
    if path.startswith("plain"):
        sv.run(gates)
        tol = C128_TOL if dtype == "c128" else c64_bound(gate_ks(gates))
    else:
        plan = qvm.Plan(gates, n, dtype, k_max=4, tile_qubits=13 if dtype == "c64" else 12)
        plan.run(sv)
        tol = plan_bound(plan) if dtype == "c64" else C128_TOL
    idx = np.asarray(g["amp_index"], dtype=np.uint64)
    want = np.asarray(g["amp_re"]) + 1j * np.asarray(g["amp_im"])
    got = sv.gather(idx)
    err = float(np.max(np.abs(got - want)))
    r2 = rel2(got, want)
    ptol = 1e-13 if dtype == "c128" else 2 * tol + tol * tol
    z = sv.expect_z_all()
    zz, _ = sv.expect_pauli(np.zeros(n - 1, np.uint64),
                            np.array([(1 << q) | (1 << (q + 1)) for q in range(n - 1)], np.uint64))
    zerr = float(np.max(np.abs(z - g["z"])))
    zzerr = float(np.max(np.abs(zz - g["zz"])))
    samp = check_samples(sv.sample(cfg["uniforms"]), g, dtype, cdf, tol)
    print(f"{path}: amp max-abs err {err:.2e}, relative 2-norm {r2:.2e} (tol {tol:.1e}), "
          f"<Z> err {zerr:.2e}, <ZZ> err {zzerr:.2e}, samples: {samp}")
    if dtype == "c128":
        assert err <= tol
    else:
        assert r2 <= tol
    assert zerr <= ptol and zzerr <= ptol


def bench_plan(gates, n):
    """The plan bench.py times: the shipped learned planner's choice, or the
    greedy planner with 3-qubit blocks in 13-qubit tiles without a model."""
    from paper_2212_14201_amd import learned_planner
    planner = learned_planner.load_default()
    ga = qvm.GateArray(gates)
    if planner is None:
        return qvm.Plan(ga, n, "c64", k_max=3, tile_qubits=13)
    return planner.choose(ga, n, "c64")[1]


def test_qft_brick_30_qubits_bench_configuration():
    """The bench's fused complex64 plan and the plain complex128 path on the
    30-qubit workload."""
    g = golden("qft30")
    cfg = config_circuit("qft30")
    n, x, gates = cfg["n"], cfg["init"], cfg["gates"]
    assert x == g["x"]
    idx = np.asarray(g["amp_index"], dtype=np.uint64)
    want = np.asarray(g["amp_re"]) + 1j * np.asarray(g["amp_im"])
    fused = qvm.StateVector(n, "c64", init=x)
    plan = bench_plan(gates, n)
    plan.run(fused)
    fgot = fused.gather(idx)
    ferr = float(np.max(np.abs(fgot - want)))
    fr2 = rel2(fgot, want)
    fz = float(np.max(np.abs(fused.expect_z_all() - g["z"])))
    del fused
    plain = qvm.StateVector(n, "c128", init=x)
    plain.run(gates)
    perr = float(np.max(np.abs(plain.gather(idx) - want)))
    pz = float(np.max(np.abs(plain.expect_z_all() - g["z"])))
    tol = plan_bound(plan)
    print(f"fused c64 amp max-abs err {ferr:.2e}, relative 2-norm {fr2:.2e} (tol {tol:.1e}) "
          f"<Z> {fz:.2e}; plain c128 amp err {perr:.2e} <Z> {pz:.2e}")
    assert perr <= C128_TOL and pz <= 1e-12
    assert fr2 <= tol and fz <= 2 * tol + tol * tol


@pytest.mark.parametrize("path", ["plain", "fused"])
def test_maximum_size_34_qubits(path):
    """The largest state the library accepts (34 qubits, complex64, 128 GiB):
    a circuit on qubits 0, 11, 22 and 33 of a seeded basis state leaves the
    state the product of the oracle's 4-qubit result and the fixed bits, so
    every nonzero amplitude, every <Z_q> and the fixed bits of every sample
    are known exactly."""
    n, S = 34, (0, 11, 22, 33)
    rng = np.random.Generator(np.random.PCG64(3434))
    x = int(rng.integers(0, 1 << n))
    for q in S:
        x &= ~(1 << q)
    small = random_mixed_circuit(4, 40, 3435, kmax=2, max_ctrl=1)
    big = [Gate(g.name, tuple(S[t] for t in g.targets), tuple(S[c] for c in g.controls),
                g.params, g.pidx, g.matrix) for g in small]
    a = oracle.simulate(4, small)
    sv = qvm.StateVector(n, "c64", init=x)
    print(f"path={path} x={x:#x}", flush=True)
    if path == "plain":
        sv.run(big)
        tol = c64_bound(gate_ks(small))
    else:
        plan = qvm.Plan(big, n, "c64", k_max=3, tile_qubits=13)
        plan.run(sv)
        sv.reset_layout()
        tol = plan_bound(plan)
    idx = np.array([x | sum(((j >> r) & 1) << S[r] for r in range(4)) for j in range(16)],
                   dtype=np.uint64)
    got = sv.gather(idx)
    err = float(np.max(np.abs(got - a)))
    others = np.array([(int(i) ^ (1 << 5)) for i in idx[:4]] + [int(x) ^ (1 << 30)], dtype=np.uint64)
    zero = float(np.max(np.abs(sv.gather(others))))
    print(f"path={path} err={err:.2e} tol={tol:.2e} off-support={zero:.1e}")
    assert err <= tol and zero == 0.0
    z = sv.expect_z_all()
    pz = np.abs(a) ** 2
    for q in range(n):
        if q in S:
            r = S.index(q)
            want = sum(pz[j] * (1 - 2 * ((j >> r) & 1)) for j in range(16))
        else:
            want = 1.0 - 2.0 * ((x >> q) & 1)
        assert abs(z[q] - want) <= 1e-5, q
    smp = sv.sample(np.linspace(0.01, 0.99, 64))
    fixed = ~sum(1 << q for q in S) & ((1 << n) - 1)
    assert all((int(s) & fixed) == (x & fixed) for s in smp)
