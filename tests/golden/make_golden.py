"""Write the stored expected values for the full-size parity tests.

Calls only the FP64 oracle (oracle/) on the seeded inputs of workloads/:

  layered12.json  12 qubits, 20 layers of U3 + CZ brick from |0..0>: all
                  4,096 amplitudes, all probabilities, <Z_q> for all q.
  layered28.json  28 qubits, 40 layers of U3 + CZ brick from |0..0>:
                  <Z_q> for all q, <Z_q Z_q+1>, 1,024 samples (with their
                  distance to the nearest CDF boundary), amplitudes at 2,048
                  seeded indices, the norm.
  qft30.json      30 qubits, QFT on the seeded basis state then 30 brick
                  layers: amplitudes at 4,096 seeded indices, <Z_q> for all q.

Run from the repository root:  python tests/golden/make_golden.py [name ...]
(tens of minutes per file on a few host cores; needs 4 GiB / 16 GiB of RAM).
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

import oracle  # noqa: E402
from workloads import config_circuit  # noqa: E402


def sample_indices(n, count, seed):
    return np.random.Generator(np.random.PCG64(seed)).integers(0, 1 << n, count, dtype=np.uint64)


def layered12():
    cfg = config_circuit("layered12")
    n = cfg["n"]
    t0 = time.time()
    psi = oracle.run_packed(n, cfg["gates"], cfg["init"])
    return {"n": n, "gates": len(cfg["gates"]), "z": oracle.expect_z_all(psi).tolist(),
            "amp_re": psi.real.tolist(), "amp_im": psi.imag.tolist(),
            "prob": oracle.probabilities(psi).tolist(),
            "norm2": oracle.norm2(psi), "oracle_seconds": time.time() - t0,
            "oracle_threads": oracle.max_threads()}


def layered28():
    cfg = config_circuit("layered28")
    n = cfg["n"]
    t0 = time.time()
    psi = oracle.run_packed(n, cfg["gates"], cfg["init"])
    z = oracle.expect_z_all(psi)
    zz = oracle.expect_zz(psi, [(q, q + 1) for q in range(n - 1)])
    samples, margin = oracle.sample(psi, cfg["uniforms"])
    idx = sample_indices(n, 2048, 2804)
    amp = psi[idx.astype(np.int64)]
    return {"n": n, "gates": len(cfg["gates"]), "z": z.tolist(), "zz": zz.tolist(),
            "samples": samples.tolist(), "sample_margin": margin.tolist(),
            "amp_index": idx.tolist(), "amp_re": amp.real.tolist(), "amp_im": amp.imag.tolist(),
            "norm2": oracle.norm2(psi), "oracle_seconds": time.time() - t0,
            "oracle_threads": oracle.max_threads()}


def qft30():
    cfg = config_circuit("qft30")
    n = cfg["n"]
    t0 = time.time()
    psi = oracle.run_packed(n, cfg["gates"], cfg["init"])
    z = oracle.expect_z_all(psi)
    idx = sample_indices(n, 4096, 3003)
    amp = psi[idx.astype(np.int64)]
    return {"n": n, "gates": len(cfg["gates"]), "x": cfg["init"], "z": z.tolist(),
            "amp_index": idx.tolist(), "amp_re": amp.real.tolist(), "amp_im": amp.imag.tolist(),
            "norm2": oracle.norm2(psi), "oracle_seconds": time.time() - t0,
            "oracle_threads": oracle.max_threads()}


def main():
    names = sys.argv[1:] or ["layered12", "layered28", "qft30"]
    for name in names:
        data = {"layered12": layered12, "layered28": layered28, "qft30": qft30}[name]()
        data["source"] = "FP64 oracle (oracle/qvm_oracle.c) via tests/golden/make_golden.py"
        with open(os.path.join(HERE, name + ".json"), "w") as fh:
            json.dump(data, fh)
        print(name, "done in", round(data["oracle_seconds"]), "s", flush=True)


if __name__ == "__main__":
    main()
