#!/usr/bin/env python3
"""Benchmark of the full-amplitude state-vector hot path on one MI355X.

Workload: 30 qubits, a seeded random basis state |x>, the quantum Fourier
transform, then 30 layers of random U3 on every qubit plus a CZ brick
(1,815 gates).  One step runs the whole path on it:

  fused complex64:  plan (lowering + fusion, host) -> init |x> -> fused tile
                    passes (MFMA blocks, diagonal runs, remapping) ->
                    <Z_q> for all q, <Z_q Z_q+1>, an 8-qubit marginal,
                    1,024 samples, renormalisation (FP64 readouts)
  plain complex128: init |x> -> one kernel per gate -> <Z_q> for all q

The reported value is the fused complex64 path's end-to-end gates/s
(planning included, as the paper adds optimisation time to the total).
Beside it: both paths' effective bandwidth, the speed-up, the dominant
kernel's roofline fraction from live per-launch HIP events, and the FP64
CPU oracle's throughput on a bounded sample of the same workload.
"""
import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "effective HBM GB/s + gates/s, 30-qubit statevector, fused c64 vs plain c128"
HBM_PEAK_GBS = 8000.0
MFMA_PEAK = {"f32": 157.3e12, "f64": 78.6e12}


def plain_bytes(gates, n, elem_bytes):
    """Algorithmic bytes of the plain per-gate path: every amplitude a gate
    changes is read and written once (dense: all; X/CNOT/SWAP moves: half;
    phase gates: the matching quarter; 2^-c for c controls)."""
    N = float(1 << n)
    tot = 0.0
    for g in gates:
        c = len(g.controls)
        if g.name in ("z", "s", "t", "sdg", "tdg", "p"):
            f = 0.5 ** (1 + c)            # one phase entry on the target's 1 half
        elif g.name == "swap":
            f = 0.5 * 0.5 ** c
        elif g.name == "x" and c:
            f = 0.5 ** c                  # pairs where the controls are set
        else:
            f = 0.5 ** c
        tot += 2.0 * N * elem_bytes * f
    return tot


def src_digest(files):
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


KERNEL_SOURCES = {
    "dense1": ["paper_2212_14201_amd/csrc/gates.hip"],
    "phase": ["paper_2212_14201_amd/csrc/gates.hip"],
    "swappair": ["paper_2212_14201_amd/csrc/gates.hip"],
    "tile": ["paper_2212_14201_amd/csrc/tile.hip", "paper_2212_14201_amd/csrc/tile.hpp"],
}


def stored_traffic(kernel, launches_bytes):
    """HBM bytes per launch from committed rocprofv3 counter runs, scaled by
    the copy-kernel factor; None when absent or when the kernel source has
    changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path) or kernel not in KERNEL_SOURCES:
        return None
    with open(path) as fh:
        data = json.load(fh)
    rec = data.get(kernel)
    if not rec or rec.get("src_sha") != src_digest(KERNEL_SOURCES[kernel]):
        return None
    return rec.get("bytes_per_launch")


def host_description():
    """Host CPU model and core counts of the machine the oracle runs on."""
    model = None
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count()
    return {"cpu_model": model, "nproc": avail, "logical_cpus": os.cpu_count()}


def cpu_baseline(n, x, gates, budget_s, plain_bytes_fn):
    """The FP64 oracle on the host cores: a strided sample of the workload's
    gates (every 25th, in order) applied to the 30-qubit state, until the
    sample or the time budget runs out; once with every thread OpenMP is
    given, then single-threaded on the next gates of the same sample."""
    import oracle
    sample = gates[::25]
    psi = oracle.basis_state(n, x)
    all_threads = oracle.max_threads()

    def leg(start, threads, seconds):
        oracle.set_threads(threads)
        done = []
        t0 = time.perf_counter()
        for g in sample[start:]:
            oracle.apply_matrix(psi, n, oracle.gate_matrix(g), g.targets, g.controls)
            done.append(g)
            if time.perf_counter() - t0 > seconds:
                break
        return done, time.perf_counter() - t0

    done, dt = leg(0, all_threads, budget_s * 0.6)
    one, dt1 = leg(len(done), 1, budget_s * 0.4)
    oracle.set_threads(all_threads)
    del psi
    host = host_description()
    out = {"value": len(done) / dt, "unit": "gates/s", "cores": all_threads, "kind": "oracle",
           "sample": f"{len(done)} gates (every 25th gate of the workload, in order) applied "
                     f"in complex128 to the {n}-qubit state by the FP64 oracle in {dt:.1f} s "
                     f"on {all_threads} threads",
           "effective_GBs": plain_bytes_fn(done, n, 16) / dt / 1e9,
           "single_thread": {"value": len(one) / dt1, "unit": "gates/s", "cores": 1,
                             "sample": f"the next {len(one)} gates of the same sample in "
                                       f"{dt1:.1f} s on one thread",
                             "effective_GBs": plain_bytes_fn(one, n, 16) / dt1 / 1e9}}
    out.update(host)
    return out


U32 = 2.0 ** -24


def golden(name):
    """Values the FP64 oracle stored for a workload (tests/golden/, written
    by make_golden.py, which calls only the oracle)."""
    with open(os.path.join(ROOT, "tests", "golden", name + ".json")) as fh:
        return json.load(fh)


def tau_of_ks(ks):
    """Stated complex64 bound on the state's 2-norm error after passes whose
    matrices are 2^k x 2^k (a diagonal term counts k = 0): (2^k + 4)
    roundings of size 2^-24 per pass, summed in quadrature, safety factor
    10."""
    return 10.0 * math.sqrt(max(sum((1 << k) + 4 for k in ks), 1)) * U32


def plan_ks(plan):
    st = plan.stats()
    return [plan.block(b)["k"] for b in range(st["blocks"])] + [0] * st["diag_ops"]


def errors_vs_oracle(sv, g, n, zz=False):
    """Errors of a state's results against the oracle's stored values:
    max-abs and relative 2-norm error of the stored amplitudes (all of them,
    or those at the stored seeded indices), max-abs error of <Z_q> (and of
    <Z_q Z_q+1> when stored)."""
    import numpy as np
    if "amp_index" in g:
        idx = np.asarray(g["amp_index"], dtype=np.uint64)
        got = sv.gather(idx)
    else:
        got = sv.amplitudes()
    want = np.asarray(g["amp_re"]) + 1j * np.asarray(g["amp_im"])
    out = {"amplitudes_compared": int(want.size),
           "amp_max_abs": float(np.max(np.abs(got - want))),
           "amp_rel_2norm": float(np.linalg.norm(got - want) / np.linalg.norm(want)),
           "z_max_abs": float(np.max(np.abs(sv.expect_z_all() - np.asarray(g["z"]))))}
    if "prob" in g:
        out["prob_max_abs"] = float(np.max(np.abs(sv.probabilities() - np.asarray(g["prob"]))))
    if zz and "zz" in g:
        zx = np.zeros(n - 1, dtype=np.uint64)
        zm = np.array([(1 << q) | (1 << (q + 1)) for q in range(n - 1)], dtype=np.uint64)
        v, _ = sv.expect_pauli(zx, zm)
        out["zz_max_abs"] = float(np.max(np.abs(v - np.asarray(g["zz"]))))
    return out, got


def time_path(torch, sv, init, runner, reps):
    """Mean run time (s) of `runner()` on a state reset to |init> before each
    rep (after one untimed rep), from HIP events on the state's stream, plus
    the host wall time per rep (launch-bound paths)."""
    sv.init_basis(init)
    runner()
    torch.cuda.synchronize()
    times = []
    t0 = time.perf_counter()
    for _ in range(reps):
        sv.init_basis(init)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        runner()
        e1.record()
        torch.cuda.synchronize()
        times.append(e0.elapsed_time(e1) / 1e3)
    wall = (time.perf_counter() - t0) / reps
    return float(sum(times) / len(times)), wall


def progress(msg):
    print(f"bench: {msg}", file=sys.stderr, flush=True)


def layered_configs(torch, planner, records):
    """The two layered U3 + CZ workloads, outside the timed steps: 12 qubits,
    20 layers (launch-bound) and 28 qubits, 40 layers (both dtypes), on the
    plain path and the fused path, with errors against the oracle's stored
    values."""
    import numpy as np
    from paper_2212_14201_amd import qvm
    from workloads import SEEDS, config_circuit
    out = {}
    for name, reps in (("layered12", 50), ("layered28", 2)):
        cfg = config_circuit(name)
        n, gates = cfg["n"], cfg["gates"]
        ga = qvm.GateArray(gates)
        g = golden(name)
        G = len(gates)
        layers = {"layered12": 20, "layered28": 40}[name]
        res = {"workload": f"{n} qubits, {layers} layers of U3 + CZ brick from |0..0>, {G} gates",
               "n_qubits": n, "gates": G}
        ref = None
        for path in ("plain_c128", "plain_c64", "fused_c64", "fused_c128"):
            dtype = path.split("_")[1]
            progress(f"{name} {path}")
            sv = qvm.StateVector(n, dtype, init=0)
            if path.startswith("plain"):
                runner = lambda: sv.run(ga)
                extra = {}
                tau = tau_of_ks([len(gg.targets) for gg in gates])
            else:
                if planner is not None and dtype == "c64" and n >= 20:
                    cand, plan, _ = planner.choose(ga, n, dtype)
                    setting = "%s, k_max %d, tile %d" % tuple(cand)
                else:
                    tile = min(n, 13 if dtype == "c64" else 12)
                    plan = qvm.Plan(ga, n, dtype, k_max=3, tile_qubits=tile)
                    setting = f"tile, k_max 3, tile {tile}"
                runner = lambda: plan.run(sv)
                st = plan.stats()
                extra = {"setting": setting, "passes": st["passes"], "blocks": st["blocks"]}
                tau = tau_of_ks(plan_ks(plan))
            secs, wall = time_path(torch, sv, 0, runner, reps)
            err, got = errors_vs_oracle(sv, g, n, zz=True)
            err["bound"] = 1e-12 if dtype == "c128" else tau
            if path == "plain_c128":
                ref = got
            elif ref is not None:
                err["amp_max_abs_vs_plain_c128"] = float(np.max(np.abs(got - ref)))
            rec = {"run_ms": secs * 1e3, "host_ms_per_call": wall * 1e3, "gates_per_s": G / secs,
                   "error_vs_oracle": err}
            if path.startswith("plain"):
                gb = plain_bytes(gates, n, 8 if dtype == "c64" else 16)
                rec["effective_GBs"] = gb / secs / 1e9
                rec["frac_of_hbm_peak"] = rec["effective_GBs"] / HBM_PEAK_GBS
            else:
                rec["effective_GBs"] = extra["passes"] * 2.0 * (1 << n) * (8 if dtype == "c64" else 16) / secs / 1e9
            rec.update(extra)
            if name == "layered28":
                t0 = time.perf_counter()
                sv.sample(cfg["uniforms"])
                rec["sample_1024_ms"] = (time.perf_counter() - t0) * 1e3
            res[path] = rec
            records.append({"config": name, "seed": SEEDS[name], "path": path, "dtype": dtype,
                            "n": n, "gates": G, "passes": extra.get("passes", G), "ms": secs * 1e3,
                            "GBs": rec["effective_GBs"],
                            "hbm_frac": rec["effective_GBs"] / HBM_PEAK_GBS,
                            "error_vs_oracle": err})
            del sv
            torch.cuda.empty_cache()
        out[name] = res
    return out


def copy_bandwidth(torch, nbytes, reps=3):
    """The library's streaming device copy (qvm_stream_copy) of nbytes, read
    plus written, in GB/s: the measured streaming reference beside the 8 TB/s
    peak."""
    from paper_2212_14201_amd import qvm
    src = torch.zeros(nbytes // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    stream = torch.cuda.current_stream().cuda_stream
    qvm.stream_copy(dst, src, stream)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        qvm.stream_copy(dst, src, stream)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del src, dst
    torch.cuda.empty_cache()
    return 2.0 * nbytes / (ms / 1e3) / 1e9


def adjoint_measure(torch, reps=2):
    """Batched adjoint gradients: 20 qubits, complex64, 16 layers of RY, RZ
    and a CNOT ladder (640 parameters, 944 gates), a 40-term Pauli sum, a
    batch of 64 parameter vectors.  Algorithmic bytes per batch element:
    start state (1 write), forward gates (read + write of what each
    changes), the Pauli sum (read psi, write lambda), the value (read both)
    and the reverse sweep (read + write of psi and lambda per gate)."""
    import numpy as np
    from paper_2212_14201_amd import adjoint
    from workloads import SEEDS, hardware_efficient_ansatz, random_pauli_sum
    n, layers, B = 20, 16, 64
    gates, P = hardware_efficient_ansatz(n, layers)
    xs, zs, cs, _ = random_pauli_sum(n, 40, SEEDS["pauli20"])
    theta = np.random.Generator(np.random.PCG64(SEEDS["hea20"])).uniform(0, 2 * math.pi, (B, P))
    prob = adjoint.AdjointProblem(n, gates, P, xs, zs, cs, B, "c64")
    prob.run(theta)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        prob.run(theta)
    dt = (time.perf_counter() - t0) / reps
    S = float(1 << n) * 8
    per_gate = 5.0 * S
    for g in gates:
        per_gate += 6.0 * S * 0.5 ** len(g.controls)
    # executed passes: the start state (write), each gate group forward
    # (read + write psi) and in reverse (read + write psi and lambda), the
    # Pauli sum (read psi, write lambda) and the value (read both)
    groups = prob.group_count()
    executed = S + groups * 2.0 * S + 2.0 * S + 2.0 * S + groups * 4.0 * S
    return {"workload": "20 qubits, complex64, 944 gates (640 RY/RZ + 304 CNOT), 40 Pauli terms, "
                        "batch 64", "ms_per_batch": dt * 1e3, "gradients_per_s": B * P / dt,
            "gate_groups": groups,
            "effective_GBs": executed * B / dt / 1e9, "frac_of_hbm_peak": executed * B / dt / 1e9 / HBM_PEAK_GBS,
            "per_gate_equivalent_GB_per_batch": per_gate * B / 1e9}


def noise_measure(torch, reps=3):
    """Kraus trajectories: 26 qubits, complex64, 4 layers of RY + RZ on every
    qubit, a CNOT / CZ brick and an H (262 gates), with depolarizing noise
    after every RY, amplitude damping on both qubits of every CNOT, phase
    damping after every RZ and bit flips after every H.  Each branching is
    one FP64 pass for the qubit's reduced density matrix plus the chosen
    operator's plain-kernel pass."""
    import numpy as np
    from paper_2212_14201_amd import noise, profiling, qvm
    from workloads import noisy_layers, uniform_stream
    n, layers = 26, 4
    gates = noisy_layers(n, layers, 2600)
    model = noise.NoiseModel([("ry", "depolarizing", {"p": 0.01}), ("cnot", "damping", {"p": 0.02}),
                              ("rz", "phase_damping", {"p": 0.02}), ("h", "bit_flip", {"p": 0.01})])
    nb = model.branchings(gates)
    sv = qvm.StateVector(n, "c64")
    u = uniform_stream(2601, nb * (reps + 1))
    noise.run_trajectory(sv, gates, model, u[:nb])
    torch.cuda.synchronize()
    profiling.begin(sv)
    t0 = time.perf_counter()
    for r in range(reps):
        noise.run_trajectory(sv, gates, model, u[nb * (r + 1): nb * (r + 2)])
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    st = profiling.end(sv).get("rdm1", {})
    ms = st.get("total_ms", 0.0)
    gbs = st["bytes"] / (ms / 1e3) / 1e9 if ms else None
    return {"workload": f"{n} qubits, complex64, {len(gates)} gates, {nb} Kraus branchings "
                        "(depolarizing, damping, phase damping, bit flip)",
            "ms_per_trajectory": dt * 1e3, "trajectories_per_s": 1.0 / dt,
            "branchings_per_s": nb / dt,
            "rdm1_kernel": {"launches": st.get("launches"), "avg_launch_ms":
                            ms / st["launches"] if ms else None, "GBs": gbs,
                            "frac_of_hbm_peak": gbs / HBM_PEAK_GBS if gbs else None}}


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--planner", choices=["learned", "fixed"], default="learned",
                    help="learned: the cost-model MLP picks among candidate plans (falls back to "
                         "'fixed' when no trained model is present); fixed: --k-max/--tile")
    ap.add_argument("--k-max", type=int, default=3)
    ap.add_argument("--tile", type=int, default=13, help="tile qubits per pass (0: one block per pass)")
    ap.add_argument("--no-adjoint", action="store_true", help="skip the adjoint-gradient workload")
    ap.add_argument("--no-noise", action="store_true", help="skip the Kraus-trajectory workload")
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-plain", action="store_true", help="skip the complex128 comparison path")
    ap.add_argument("--no-configs", action="store_true",
                    help="skip the 12- and 28-qubit layered workloads")
    ap.add_argument("--records", default=None,
                    help="append one JSON record per measured workload and path to this file")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(the state would shard by its top qubits across GPUs; not built).", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2212_14201_amd import qvm, profiling
    from workloads import SEEDS, config_circuit, uniform_stream

    cfg = config_circuit("qft30")
    n, x, gates = cfg["n"], cfg["init"], cfg["gates"]
    ga = qvm.GateArray(gates)
    uniforms = uniform_stream(3002, 1024)
    zz_x = np.zeros(n - 1, dtype=np.uint64)
    zz_z = np.array([(1 << q) | (1 << (q + 1)) for q in range(n - 1)], dtype=np.uint64)
    planner = None
    if args.planner == "learned":
        from paper_2212_14201_amd import learned_planner
        planner = learned_planner.load_default()
    fused = qvm.StateVector(n, "c64", init=None)
    plain = None if args.no_plain else qvm.StateVector(n, "c128", init=None)
    torch.cuda.synchronize()

    def step():
        r = {}
        t0 = time.perf_counter()
        if planner is not None:
            r["choice"], plan, r["predicted_ms"] = planner.choose(ga, n, "c64")
        else:
            plan = qvm.Plan(ga, n, "c64", k_max=args.k_max, tile_qubits=args.tile, defer_narrow=args.tile > 0)
        t1 = time.perf_counter()
        fused.init_basis(x)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        plan.run(fused)
        e1.record()
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        r["plan_s"] = t1 - t0
        r["fused_run_s"] = e0.elapsed_time(e1) / 1e3
        r["fused_e2e_s"] = t2 - t0
        r["stats"] = plan.stats()
        r["plan"] = plan
        t3 = time.perf_counter()
        r["z"] = fused.expect_z_all()
        r["zz"], _ = fused.expect_pauli(zz_x, zz_z)
        r["marg"] = fused.probabilities(list(range(8)))
        r["samples"] = fused.sample(uniforms)
        r["norm_before"] = fused.renormalize()
        r["readout_s"] = time.perf_counter() - t3
        if plain is not None:
            plain.init_basis(x)
            e2 = torch.cuda.Event(enable_timing=True)
            e3 = torch.cuda.Event(enable_timing=True)
            e2.record()
            plain.run(ga)
            e3.record()
            r["z128"] = plain.expect_z_all()
            r["plain_run_s"] = e2.elapsed_time(e3) / 1e3
        return r

    for i in range(args.warmup):
        step()
        progress(f"warmup step {i + 1} done")
    profiling.begin(fused)
    if plain is not None:
        profiling.begin(plain)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    recs = []
    for i in range(args.steps):
        recs.append(step())
        progress(f"step {i + 1} done")
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kstats = {"c64:" + k: v for k, v in profiling.end(fused).items()}
    if plain is not None:
        kstats.update({"c128:" + k: v for k, v in profiling.end(plain).items()})

    G = len(gates)
    fused_run = float(np.mean([r["fused_run_s"] for r in recs]))
    fused_e2e = float(np.mean([r["fused_e2e_s"] for r in recs]))
    st = recs[-1]["stats"]
    N = 1 << n
    fused_info = {
        "run_ms": fused_run * 1e3, "plan_ms": float(np.mean([r["plan_s"] for r in recs])) * 1e3,
        "end_to_end_ms": fused_e2e * 1e3,
        "readout_ms": float(np.mean([r["readout_s"] for r in recs])) * 1e3,
        "gates_per_s": G / fused_run, "gates_per_s_end_to_end": G / fused_e2e,
        "effective_GBs": st["passes"] * 2.0 * N * 8 / fused_run / 1e9,
        "unfused_equivalent_GB_per_run": plain_bytes(gates, n, 8) / 1e9,
        "passes": st["passes"], "blocks": st["blocks"], "blocks_by_k": st["blocks_by_k"],
        "diag_ops": st["diag_ops"], "tile_qubits": st["tile_qubits"],
        "norm_before_renormalize": float(recs[-1]["norm_before"]),
    }
    if planner is not None:
        fused_info["planner"] = "learned"
        fused_info["choice"] = "%s, k_max %d, tile %d" % tuple(recs[-1]["choice"])
        fused_info["predicted_ms"] = recs[-1]["predicted_ms"]
    else:
        fused_info["planner"] = f"greedy, k_max {args.k_max}, tile {args.tile}"
    fused_info["tile_TFLOPs"] = None
    if "c64:tile" in kstats and kstats["c64:tile"]["total_ms"]:
        kt = kstats["c64:tile"]
        fused_info["tile_TFLOPs"] = kt["flops"] / (kt["total_ms"] / 1e3) / 1e12
        fused_info["tile_frac_of_mfma_peak"] = fused_info["tile_TFLOPs"] / (MFMA_PEAK["f32"] / 1e12)
    out = {"metric": METRIC, "value": G / fused_e2e, "unit": "gates/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": wall / args.steps * 1e3,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
           "data": "synthetic",
           "config": {"workload": "qft30: QFT on a seeded basis state then 30 layers of random U3 + "
                                  "CZ brick, 30 qubits, 1815 gates",
                      "n_qubits": n, "gates": G, "fused_dtype": "complex64",
                      "plain_dtype": "complex128", "planner": fused_info["planner"]},
           "fused_c64": fused_info}
    if plain is not None:
        prun = float(np.mean([r["plain_run_s"] for r in recs]))
        pbytes = plain_bytes(gates, n, 16)
        out["plain_c128"] = {"run_ms": prun * 1e3, "gates_per_s": G / prun,
                             "effective_GBs": pbytes / prun / 1e9,
                             "frac_of_hbm_peak": pbytes / prun / 1e9 / HBM_PEAK_GBS}
        out["speedup_fused_c64_vs_plain_c128"] = prun / fused_run
        z64, z128 = recs[-1]["z"], recs[-1]["z128"]
        out["fused_c64_max_abs_z_error_vs_c128"] = float(np.max(np.abs(z64 - z128)))
    # errors of both paths' final states against the oracle's stored values
    # for this workload (amplitudes at 4,096 seeded indices, every <Z_q>)
    gq = golden("qft30")
    last_plan = recs[-1]["plan"]
    err, got64 = errors_vs_oracle(fused, gq, n)
    err["bound"] = tau_of_ks(plan_ks(last_plan))
    out["fused_c64"]["error_vs_oracle"] = err
    if plain is not None:
        err, got128 = errors_vs_oracle(plain, gq, n)
        err["bound"] = 1e-12
        out["plain_c128"]["error_vs_oracle"] = err
        out["fused_c64"]["error_vs_oracle"]["amp_max_abs_vs_plain_c128"] = float(np.max(np.abs(got64 - got128)))
    # roofline of the kernel class with the largest share of the timed region
    dom_name, dom = max(kstats.items(), key=lambda kv: kv[1]["total_ms"])
    per_launch_s = dom["total_ms"] / dom["launches"] / 1e3
    bpl = dom["bytes"] / dom["launches"]
    fpl = dom["flops"] / dom["launches"]
    prec = "f32" if dom_name.startswith("c64") else "f64"
    if fpl / max(bpl, 1.0) > MFMA_PEAK[prec] / (HBM_PEAK_GBS * 1e9):
        ach = fpl / per_launch_s / 1e12
        roof = {"bound": "mfma", "achieved": ach, "peak": MFMA_PEAK[prec] / 1e12, "unit": "TFLOP/s",
                "frac": ach / (MFMA_PEAK[prec] / 1e12)}
    else:
        ach = bpl / per_launch_s / 1e9
        roof = {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": ach / HBM_PEAK_GBS}
    roof["kernel"] = dom_name
    roof["launches_timed"] = dom["launches"]
    roof["avg_launch_ms"] = per_launch_s * 1e3
    roof["algorithmic_bytes_per_launch"] = bpl
    roof["traffic"] = stored_traffic(dom_name.split(":")[1], bpl)
    out["roofline"] = roof
    out["kernels"] = {k: {"launches": v["launches"], "total_ms": v["total_ms"],
                          "GBs": v["bytes"] / (v["total_ms"] / 1e3) / 1e9 if v["total_ms"] else None,
                          "TFLOPs": v["flops"] / (v["total_ms"] / 1e3) / 1e12 if v["total_ms"] else None}
                      for k, v in kstats.items()}
    # outside the timed steps: the greedy planner without the model, at the
    # setting it falls back to (3-qubit blocks in 13-qubit tiles, narrow
    # trailing blocks deferred) and at the classic fused-gate setting (one
    # 5-qubit block per pass), beside the learned choice
    if planner is not None:
        from paper_2212_14201_amd import learned_planner
        base = {}
        for label, cand in (("fallback", learned_planner.FALLBACK), ("classic", learned_planner.CLASSIC)):
            gplan = learned_planner.build_plan(ga, n, "c64", cand)
            secs, _ = time_path(torch, fused, x, lambda: gplan.run(fused), 2)
            base[label] = {"setting": "%s, k_max %d, tile %d" % cand, "run_ms": secs * 1e3,
                           "learned_speedup": secs / fused_run}
        out["fused_c64"]["greedy_fallback"] = base["fallback"]
        out["fused_c64"]["greedy_classic"] = base["classic"]
    del fused, plain
    torch.cuda.empty_cache()
    out["hbm_copy_GBs"] = copy_bandwidth(torch, 1 << 33)
    out["fused_c64"]["effective_frac_of_copy"] = out["fused_c64"]["effective_GBs"] / out["hbm_copy_GBs"]
    if "plain_c128" in out:
        out["plain_c128"]["frac_of_copy"] = out["plain_c128"]["effective_GBs"] / out["hbm_copy_GBs"]
    records = [{"config": "qft30", "seed": SEEDS["qft30"], "path": "fused_c64", "dtype": "c64", "n": n,
                "gates": G, "passes": st["passes"], "ms": fused_run * 1e3,
                "GBs": out["fused_c64"]["effective_GBs"],
                "hbm_frac": out["fused_c64"]["effective_GBs"] / HBM_PEAK_GBS,
                "mfma_frac": out["fused_c64"].get("tile_frac_of_mfma_peak"),
                "error_vs_oracle": out["fused_c64"]["error_vs_oracle"]}]
    if "plain_c128" in out:
        records.append({"config": "qft30", "seed": SEEDS["qft30"], "path": "plain_c128", "dtype": "c128",
                        "n": n, "gates": G, "passes": G, "ms": out["plain_c128"]["run_ms"],
                        "GBs": out["plain_c128"]["effective_GBs"],
                        "hbm_frac": out["plain_c128"]["frac_of_hbm_peak"],
                        "error_vs_oracle": out["plain_c128"]["error_vs_oracle"]})
    if not args.no_configs:
        out["configs"] = layered_configs(torch, planner, records)
    if not args.no_adjoint:
        progress("adjoint workload")
        out["adjoint_c64"] = adjoint_measure(torch)
    if not args.no_noise:
        progress("Kraus-trajectory workload")
        out["noise_c64"] = noise_measure(torch)
    if not args.no_cpu_baseline:
        progress("oracle on the host cores")
        out["cpu_baseline"] = cpu_baseline(n, x, gates, args.cpu_seconds, plain_bytes)
    if args.records:
        with open(args.records, "a") as fh:
            for r in records:
                fh.write(json.dumps(r) + "\n")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
