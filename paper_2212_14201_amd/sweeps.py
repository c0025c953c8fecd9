"""The paper's own benchmark shapes, run on the library with seeded
synthetic inputs (the paper prints no numbers for them, so these are
context curves, not targets):

  gates    time per gate of RX, RY, CNOT, Toffoli and random 1-, 2- and
           3-qubit unitaries on the plain per-gate path over qubit counts,
           complex128 and complex64 (the paper's basic-gate performance
           comparison, "Performance of basic gates");
  circuit  the paper's random circuit, a rotation layer (RX, RY, RZ on every
           qubit) and a CNOT layer (target i, control (i+1) mod n) repeated,
           over qubit counts: plain complex128 against the fused complex64
           path with the shipped learned planner (the greedy planner at its
           fallback setting if no model is present), planning included.

    python -m paper_2212_14201_amd.sweeps gates --n 16 20 24 28 30
    python -m paper_2212_14201_amd.sweeps circuit --n 16 20 24 28 30 --layers 10
    python -m paper_2212_14201_amd.sweeps simplify

The third compares the fused path with and without the peephole pre-pass
(qvm_simplify) on circuits of the planner workload.

One JSON object per measurement on stdout.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))

GATE_KINDS = ("rx", "ry", "cnot", "toffoli", "u1q", "u2q", "u3q")


def _unitary(rng, k):
    z = rng.standard_normal((1 << k, 1 << k)) + 1j * rng.standard_normal((1 << k, 1 << k))
    q, r = np.linalg.qr(z)
    return q * (np.diag(r) / np.abs(np.diag(r)))


def gate_list(kind, n, count, seed):
    """`count` gates of one kind on seeded random distinct qubits."""
    from workloads import Gate
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for _ in range(count):
        if kind in ("rx", "ry"):
            out.append(Gate(kind, (int(rng.integers(0, n)),), (), (float(rng.uniform(0, 2 * np.pi)),)))
        elif kind == "cnot":
            t, c = (int(v) for v in rng.choice(n, 2, replace=False))
            out.append(Gate("x", (t,), (c,)))
        elif kind == "toffoli":
            t, c1, c2 = (int(v) for v in rng.choice(n, 3, replace=False))
            out.append(Gate("x", (t,), (c1, c2)))
        else:
            k = int(kind[1])
            qs = tuple(int(v) for v in rng.choice(n, k, replace=False))
            out.append(Gate("unitary", qs, (), (), -1, _unitary(rng, k)))
    return out


def touched_fraction(kind):
    """Share of the amplitudes a gate of this kind must change."""
    return {"cnot": 0.5, "toffoli": 0.25}.get(kind, 1.0)


def _events():
    import torch
    return torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)


def sweep_gates(ns, dtypes=("c128", "c64"), count=32, seed=7):
    import torch
    from . import qvm
    for dtype in dtypes:
        eb = 16 if dtype == "c128" else 8
        for n in ns:
            sv = qvm.StateVector(n, dtype, init=0)
            for kind in GATE_KINDS:
                ga = qvm.GateArray(gate_list(kind, n, count, seed + n))
                sv.run(ga)                                  # warm-up
                e0, e1 = _events()
                e0.record()
                sv.run(ga)
                e1.record()
                torch.cuda.synchronize()
                ms = e0.elapsed_time(e1) / count
                gbs = 2.0 * (1 << n) * eb * touched_fraction(kind) / (ms / 1e3) / 1e9
                yield {"sweep": "gates", "dtype": dtype, "n": n, "gate": kind, "ms_per_gate": ms,
                       "effective_GBs": gbs}
            del sv
            torch.cuda.empty_cache()


def sweep_circuit(ns, layers=10, seed=11):
    import torch
    from . import learned_planner, qvm
    from workloads import rotation_cnot_circuit
    planner = learned_planner.load_default()
    for n in ns:
        gates = rotation_cnot_circuit(n, layers, seed + n)
        ga = qvm.GateArray(gates)
        rec = {"sweep": "circuit", "n": n, "layers": layers, "gates": len(gates)}
        plain = qvm.StateVector(n, "c128", init=0)
        plain.run(ga)
        plain.init_basis(0)
        e0, e1 = _events()
        e0.record()
        plain.run(ga)
        e1.record()
        torch.cuda.synchronize()
        rec["plain_c128_ms"] = e0.elapsed_time(e1)
        del plain
        torch.cuda.empty_cache()
        fused = qvm.StateVector(n, "c64", init=0)
        for rep in range(2):                                # the second one is reported
            fused.init_basis(0)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            if planner is not None:
                cand, plan, _ = planner.choose(ga, n, "c64")
                rec["planner"] = "learned: %s, k_max %d, tile %d" % cand
            else:
                plan = learned_planner.build_plan(ga, n, "c64", learned_planner.FALLBACK)
                rec["planner"] = "greedy: %s, k_max %d, tile %d" % learned_planner.FALLBACK
            t1 = time.perf_counter()
            plan.run(fused)
            torch.cuda.synchronize()
            t2 = time.perf_counter()
        rec["fused_c64_plan_ms"] = (t1 - t0) * 1e3
        rec["fused_c64_end_to_end_ms"] = (t2 - t0) * 1e3
        rec["passes"] = plan.stats()["passes"]
        rec["speedup"] = rec["plain_c128_ms"] / rec["fused_c64_end_to_end_ms"]
        del fused
        torch.cuda.empty_cache()
        yield rec


def sweep_simplify(first=100_000, count=20, n_range=(26, 28)):
    """The peephole pre-pass on planner-workload circuits: gate counts and the
    fused complex64 run time (greedy, 3-qubit blocks in 13-qubit tiles)
    without and with it."""
    import torch
    from . import qvm
    from workloads import random_planner_circuit
    sv = None
    for s in range(first, first + count):
        n, gates = random_planner_circuit(s, n_range=n_range, g_range=(100, 500))
        ga = qvm.GateArray(gates)
        t0 = time.perf_counter()
        sa = qvm.simplify(ga, n)
        ts = (time.perf_counter() - t0) * 1e3
        if sv is None or sv.n != n:
            sv = None
            torch.cuda.empty_cache()
            sv = qvm.StateVector(n, "c64", init=0)
        rec = {"sweep": "simplify", "seed": s, "n": n, "gates": ga.n, "kept": sa.n, "simplify_ms": ts}
        for tag, arr in (("original", ga), ("simplified", sa)):
            plan = qvm.Plan(arr, n, "c64", k_max=3, tile_qubits=13)
            sv.init_basis(0)
            plan.run(sv)
            sv.init_basis(0)
            e0, e1 = _events()
            e0.record()
            plan.run(sv)
            e1.record()
            torch.cuda.synchronize()
            rec[tag + "_ms"] = e0.elapsed_time(e1)
        yield rec


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("what", choices=["gates", "circuit", "simplify"])
    ap.add_argument("--n", type=int, nargs="+", default=[16, 20, 24, 28, 30])
    ap.add_argument("--layers", type=int, default=10)
    ap.add_argument("--dtype", nargs="+", default=["c128", "c64"])
    a = ap.parse_args()
    if a.what == "gates":
        it = sweep_gates(a.n, a.dtype)
    elif a.what == "circuit":
        it = sweep_circuit(a.n, a.layers)
    else:
        it = sweep_simplify()
    for rec in it:
        print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
