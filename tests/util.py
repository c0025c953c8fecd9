"""Shared helpers for the test suite (tolerances, oracle shortcuts)."""
import math
import os
import re

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

U32 = 2.0 ** -24          # unit roundoff of binary32

C128_TOL = 1e-12          # max-abs amplitude error allowed in complex128


def c64_bound(ks):
    """Stated per-result bound for complex64 amplitudes after passes whose
    matrices are 2^k x 2^k: probabilistic rounding-error model, each pass
    contributing (2^k + 4) roundings of size u, summed in quadrature, with a
    safety factor of 10."""
    s = sum((1 << k) + 4 for k in ks)
    return 10.0 * math.sqrt(max(s, 1)) * U32


def gate_ks(gates):
    return [len(g.targets) for g in gates]


def header_functions():
    """Every function declared in include/*.h."""
    names = []
    inc = os.path.join(ROOT, "include")
    for f in sorted(os.listdir(inc)):
        if f.endswith(".h"):
            txt = open(os.path.join(inc, f)).read()
            txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
            names += re.findall(r"\b(qvm_[a-z0-9_]+)\s*\(", txt)
    return sorted(set(names))
