"""Launch one kernel class a few times at a given size, for counter runs.

Used under ``rocprofv3 --pmc`` to read HBM traffic (FETCH_SIZE, WRITE_SIZE)
of a single kernel class, and with ``--kernel copy`` to read the same
counters for a plain device copy of known size (the scale factor).

    python -m paper_2212_14201_amd.microbench --kernel dense1 --n 30 --dtype c128
    python -m paper_2212_14201_amd.microbench --kernel tile --n 30 --dtype c64 --defer
    python -m paper_2212_14201_amd.microbench --kernel copy --n 30 --dtype c128
    python -m paper_2212_14201_amd.microbench --kernel stream --n 30 --launches 5
    python -m paper_2212_14201_amd.microbench --kernel blocks --k 4 --blocks 32 --n 30 --launches 2
    python -m paper_2212_14201_amd.microbench --kernel phase --qubits 0 1 --n 30 --dtype c128
    python -m paper_2212_14201_amd.microbench --kernel adjoint --launches 3
"""
import argparse
import os
import sys

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--kernel", choices=["dense1", "phase", "tile", "copy", "stream", "blocks", "adjoint"],
                    required=True)
    ap.add_argument("--qubits", type=int, nargs=2, default=(0, 1), help="phase: the CZ's control and target")
    ap.add_argument("--k", type=int, default=4, help="blocks: block width in qubits")
    ap.add_argument("--blocks", type=int, default=32, help="blocks: fused blocks in the one tile pass")
    ap.add_argument("--tile", type=int, default=13, help="blocks: tile qubits of the pass")
    ap.add_argument("--classic", action="store_true",
                    help="tile: the classic plan (one 5-qubit block per pass) instead of 3-qubit blocks in tiles")
    ap.add_argument("--defer", action="store_true",
                    help="tile: passes leave narrow trailing blocks to a later pass (the learned planner's "
                         "choice for the 30-qubit workload)")
    ap.add_argument("--n", type=int, default=30)
    ap.add_argument("--dtype", default="c128")
    ap.add_argument("--launches", type=int, default=3)
    a = ap.parse_args()
    import torch
    from paper_2212_14201_amd import qvm
    from workloads import Gate, config_circuit

    if a.kernel == "stream":
        # streaming rates: qvm_stream_copy, a plain U3 on complex128 and an
        # almost empty tile pass on complex64, each at 2^n amplitudes
        def timed(fn, reps):
            fn()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(reps):
                fn()
            e1.record()
            torch.cuda.synchronize()
            return e0.elapsed_time(e1) / reps
        nb = 16 << a.n
        src = torch.zeros(nb // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        ms = timed(lambda: qvm.stream_copy(dst, src), a.launches)
        print(f"qvm_stream_copy {nb >> 30} GiB: {ms:.3f} ms, {2 * nb / ms / 1e6:.0f} GB/s", flush=True)
        ms = timed(lambda: dst.copy_(src), a.launches)
        print(f"torch device copy {nb >> 30} GiB: {ms:.3f} ms, {2 * nb / ms / 1e6:.0f} GB/s", flush=True)
        del src, dst
        torch.cuda.empty_cache()
        sv = qvm.StateVector(a.n, "c128", init=0)
        for t in (0, a.n // 3, a.n - 1):
            g = qvm.GateArray([Gate("u3", (t,), (), (0.3, 0.2, 0.1))])
            ms = timed(lambda: sv.run(g), a.launches)
            print(f"plain u3 complex128 target {t}: {ms:.3f} ms, {2 * 16 * 2**a.n / ms / 1e6:.0f} GB/s", flush=True)
        del sv
        torch.cuda.empty_cache()
        sv = qvm.StateVector(a.n, "c64", init=0)
        plan = qvm.Plan([Gate("z", (a.n - 1,), (a.n - 2,))], a.n, "c64", k_max=3, tile_qubits=13)
        def run():
            sv.init_basis(0)
            plan.run(sv)
        ms = timed(run, a.launches) - timed(lambda: sv.init_basis(0), a.launches)
        print(f"tile pass complex64 (one CZ): {ms:.3f} ms, {2 * 8 * 2**a.n / ms / 1e6:.0f} GB/s", flush=True)
        return
    if a.kernel == "adjoint":
        # the batched adjoint workload: 20 qubits, complex64, 16 layers of
        # RY, RZ and a CNOT ladder (944 gates), 40 Pauli terms, batch 64
        import math
        import numpy as np
        from paper_2212_14201_amd import adjoint
        from workloads import SEEDS, hardware_efficient_ansatz, random_pauli_sum
        gates, P = hardware_efficient_ansatz(20, 16)
        xs, zs, cs, _ = random_pauli_sum(20, 40, SEEDS["pauli20"])
        theta = np.random.Generator(np.random.PCG64(SEEDS["hea20"])).uniform(0, 2 * math.pi, (64, P))
        prob = adjoint.AdjointProblem(20, gates, P, xs, zs, cs, 64, "c64")
        for _ in range(a.launches):
            prob.run(theta)
        torch.cuda.synchronize()
        print(f"adjoint batch 64 x {a.launches}", flush=True)
        return
    if a.kernel == "blocks":
        # one complex64 tile pass (tiles of `tile` qubits) holding `blocks` random
        # k-qubit unitaries on overlapping windows of the tile qubits (so
        # that none fuse): the block kernel's cost in isolation
        import numpy as np
        rng = np.random.Generator(np.random.PCG64(17))
        gates = []
        for i in range(a.blocks):
            z = rng.standard_normal((2 ** a.k, 2 ** a.k)) + 1j * rng.standard_normal((2 ** a.k, 2 ** a.k))
            q, r = np.linalg.qr(z)
            lo = i % (a.tile - a.k + 1)
            gates.append(Gate("unitary", tuple(range(lo, lo + a.k)), (), (), -1, q))
        sv = qvm.StateVector(a.n, "c64", init=0)
        plan = qvm.Plan(gates, a.n, "c64", k_max=a.k, tile_qubits=a.tile)
        assert plan.stats()["passes"] == 1 and plan.stats()["blocks"] == a.blocks
        for _ in range(a.launches):
            sv.init_basis(0)
            plan.run(sv)
        torch.cuda.synchronize()
        print(f"blocks k={a.k} x {a.blocks} n={a.n} x {a.launches}", flush=True)
        return
    if a.kernel == "copy":
        real = torch.float32 if a.dtype == "c64" else torch.float64
        src = torch.zeros(2 << a.n, dtype=real, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(a.launches):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(f"copy of {src.numel() * src.element_size()} bytes x {a.launches}", flush=True)
        return
    sv = qvm.StateVector(a.n, a.dtype, init=0)
    if a.kernel in ("dense1", "phase"):
        # dense1: a U3 on qubit n/3; phase: one CZ (a phase on the quarter of
        # the amplitudes with both bits set)
        g = (Gate("u3", (a.n // 3,), (), (0.3, 0.2, 0.1)) if a.kernel == "dense1"
             else Gate("z", (a.qubits[1],), (a.qubits[0],)))
        for _ in range(a.launches):
            sv.apply(g)
    else:
        cfg = config_circuit("qft30") if a.n == 30 else None
        gates = cfg["gates"] if cfg else [Gate("h", (q,)) for q in range(a.n)]
        plan = (qvm.Plan(gates, a.n, a.dtype, k_max=5, tile_qubits=0) if a.classic
                else qvm.Plan(gates, a.n, a.dtype, k_max=3, tile_qubits=13 if a.dtype == "c64" else 12,
                              defer_narrow=a.defer))
        for _ in range(a.launches):
            sv.init_basis(0)
            plan.run(sv)
    torch.cuda.synchronize()
    print(f"{a.kernel} n={a.n} {a.dtype} x {a.launches}", flush=True)


if __name__ == "__main__":
    main()
