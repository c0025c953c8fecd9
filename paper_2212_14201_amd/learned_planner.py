"""Learned fusion planner driven by the cost-model MLP.

The greedy planner (``qvm_plan_greedy``) builds a plan for a given block
width k_max and execution mode: one fused block per HBM pass (``tile = 0``)
or tile passes that hold many blocks (``tile = L``).  Which choice is fastest
depends on the circuit.  The learned planner builds every candidate plan on
the host, predicts each pass's time with the MLP (features from
``qvm_plan_pass_features``), and runs the candidate with the smallest
predicted total.  The greedy planner alone stays as the fallback (when no
trained model is present), and at its classic setting (5-qubit blocks, one
pass each) as the baseline that plan quality is measured against; all
candidates compute the same state up to rounding.

The MLP is trained on pass timings the simulator measures itself (per-launch
HIP events of the tile kernel), on a seeded mixture of circuit families
(``workloads.planner_mix_circuit``: random gates from {H, T, RX, RZ, RZZ, CNOT,
CZ, Toffoli}, layered U3 + CZ bricks, QFT prefixes, rotation + CNOT layers;
26-32 qubits).  Features are clamped to the training range when predicting.

    python -m paper_2212_14201_amd.learned_planner collect  --first 0 --count 2000 --no-mix --out R.npz
    python -m paper_2212_14201_amd.learned_planner collect  --first 0 --count 1000 --out X.npz
    python -m paper_2212_14201_amd.learned_planner combine  --data R.npz X.npz --out D.npz
    python -m paper_2212_14201_amd.learned_planner train    --data D.npz --model M.npz
    python -m paper_2212_14201_amd.learned_planner evaluate --model M.npz --first 100000 --count 200
    python -m paper_2212_14201_amd.learned_planner explain  --model M.npz --workload qft30
"""
from __future__ import annotations

import argparse
import ctypes
import json
import math
import os
import sys
import time

import numpy as np

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))

from . import qvm  # noqa: E402
from .qvm import _i32p, _vp, check, lib  # noqa: E402

NFEAT = 23
# the trained cost model shipped with the package (complex64 pass timings)
DEFAULT_MODEL = os.path.join(os.path.dirname(os.path.abspath(__file__)), "data", "costmodel_c64.npz")
CANDIDATES = [("block", 2, 0), ("block", 3, 0), ("block", 4, 0), ("block", 5, 0), ("block", 6, 0),
              ("tile", 3, 13), ("tile", 4, 13), ("tile", 5, 13),
              ("tile", 3, 12), ("tile", 4, 12), ("tile", 5, 12), ("tile", 3, 11)]
# tile settings whose passes leave narrow trailing blocks to a later pass
# (QVM_PLAN_DEFER_NARROW): scored beside the others; the model sees their
# passes as it sees any pass
DEFER_CANDIDATES = [("tiled", 3, 13), ("tiled", 4, 13), ("tiled", 3, 12)]
# the setting used without a model: 3-qubit blocks in 13-qubit tiles with
# narrow trailing blocks deferred (the fastest fixed setting on held-out
# random and mixture circuits and on the 30-qubit workload)
FALLBACK = ("tiled", 3, 13)
# the settings the planner scores: 2-qubit blocks one per pass are left out
# (every pass streams the whole state for a 2-qubit block; on the 30-qubit
# workload 436 passes, 8.4x the fallback's time, and the slowest candidate
# to plan); the fallback is planned in full while the others are scored
SCORED = [c for c in CANDIDATES if c != ("block", 2, 0)] + DEFER_CANDIDATES
CLASSIC = ("block", 5, 0)      # the classic fused-gate simulator: 5-qubit blocks, one pass each
# tile widths at which the model also picks the block width of every pass
ADAPTIVE_TILES = (13, 12)
ADAPTIVE_K = (3, 4, 5)
TILE_KIND = 6                  # kernel class index of the tile kernel in the profiler


def _declare():
    L = lib()
    L.qvm_plan_pass_features.argtypes = [_vp, ctypes.POINTER(ctypes.c_float), ctypes.c_size_t, _i32p]
    L.qvm_plan_pass_features.restype = ctypes.c_int
    L.qvm_profile_launches.argtypes = [_vp, ctypes.POINTER(ctypes.c_double), _i32p, ctypes.c_int32, _i32p]
    L.qvm_profile_launches.restype = ctypes.c_int
    return L


_POOL = None


def _pool():
    """The host threads that plan the candidates (kept between calls)."""
    global _POOL
    if _POOL is None:
        from concurrent.futures import ThreadPoolExecutor
        _POOL = ThreadPoolExecutor(max_workers=min(len(SCORED), os.cpu_count() or 1))
    return _POOL


def cand_for_dtype(c, dtype):
    mode, k, tile = c
    if dtype == "c128" and tile > 12:
        tile = 12
    return mode, k, tile


def build_plan(ga, n, dtype, cand, image=True, k_of_pass=None):
    """A candidate plan: (mode, k_max, tile) of the greedy planner ("tiled":
    tile passes that leave narrow trailing blocks to a later pass), or
    ("adaptive", k, tile) with the per-pass block widths k_of_pass."""
    mode, k, tile = cand_for_dtype(cand, dtype)
    try:
        if mode == "adaptive":
            return qvm.Plan(ga, n, dtype, tile_qubits=tile, image=image, k_of_pass=k_of_pass)
        return qvm.Plan(ga, n, dtype, k_max=k, tile_qubits=tile, image=image, defer_narrow=mode == "tiled")
    except qvm.QvmError:
        return None        # e.g. a Toffoli does not fit 2-qubit blocks


def cand_name(cand):
    return "%s-%d-%d" % tuple(cand)


def plan_features(plan) -> np.ndarray:
    L = _declare()
    npass = ctypes.c_int32()
    check(L.qvm_plan_pass_features(plan._h, None, 0, ctypes.byref(npass)))
    out = np.zeros(npass.value * NFEAT, dtype=np.float32)
    check(L.qvm_plan_pass_features(plan._h, out.ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
                                   out.size, ctypes.byref(npass)))
    return out.reshape(npass.value, NFEAT)


def tile_launch_ms(sv) -> np.ndarray:
    L = _declare()
    cnt = ctypes.c_int32()
    check(L.qvm_profile_launches(sv.handle, None, None, 0, ctypes.byref(cnt)))
    ms = np.zeros(cnt.value, dtype=np.float64)
    kind = np.zeros(cnt.value, dtype=np.int32)
    check(L.qvm_profile_launches(sv.handle, ms.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                 kind.ctypes.data_as(_i32p), cnt.value, ctypes.byref(cnt)))
    return ms[kind == TILE_KIND]


class StatePool:
    """One state per (n, dtype) at a time (large states are freed first)."""

    def __init__(self):
        self.key, self.sv = None, None

    def get(self, n, dtype):
        import torch
        if self.key != (n, dtype):
            self.sv = None
            torch.cuda.empty_cache()
            self.sv = qvm.StateVector(n, dtype, init=0)
            self.key = (n, dtype)
        return self.sv


def time_plan(sv, plan, x=0):
    """Run a plan once with per-launch events; returns (total ms, pass ms)."""
    from . import profiling
    sv.init_basis(x)
    profiling.begin(sv)
    plan.run(sv)
    profiling.end(sv)
    ms = tile_launch_ms(sv)
    return float(ms.sum()), ms


def planner_circuit(seed, n_range=(26, 32), g_range=(100, 500)):
    from workloads import random_planner_circuit
    return random_planner_circuit(seed, n_range=n_range, g_range=g_range)


# circuits longer than this are timed with tile-pass candidates only (one
# block per pass would take seconds per circuit); block passes are covered
# by the shorter circuits, and a block pass looks the same in either
LONG_CIRCUIT = 600


# ------------------------------------------------------------------ collect
def collect(first, count, out_path, dtype="c64", seed=0, n_range=(26, 32), g_range=(100, 500), mix=True):
    """Time candidate plans of each circuit; save every pass's features and
    measured milliseconds (npz: features, ms, seed, cand).  Each circuit
    draws a setting at random: a tile width, whose candidates at every block
    width are all timed (their pass i holds the same gates, so the model
    learns the per-pass width choice from paired samples), or one block-per-
    pass candidate.  mix: circuits from the mixture of families
    (``workloads.planner_mix_circuit``), else the random planner workload
    with the given ranges."""
    from workloads import planner_mix_circuit
    rng = np.random.Generator(np.random.PCG64(seed + first))
    tile_ls = sorted({c[2] for c in CANDIDATES if c[0] == "tile"}, reverse=True)
    blocks = [c for c in CANDIDATES if c[0] == "block"]
    jobs = []
    for s in range(first, first + count):
        if mix:
            n, gates, _ = planner_mix_circuit(s)
        else:
            n, gates = planner_circuit(s, n_range, g_range)
        # tile settings three times as often as block settings; long
        # circuits take tile settings only (one block per pass would take
        # seconds per circuit; a block pass looks the same in either)
        if len(gates) > LONG_CIRCUIT or rng.random() < 0.75:
            L = tile_ls[int(rng.integers(0, len(tile_ls)))]
            cands = [c for c in CANDIDATES if c[0] == "tile" and c[2] == L]
        else:
            cands = [blocks[int(rng.integers(0, len(blocks)))]]
        jobs.append((n, s, gates, cands))
    jobs.sort(key=lambda j: j[0])          # group by size to reuse the state buffer
    pool = StatePool()
    F, T, S, C = [], [], [], []
    t0 = time.time()
    for i, (n, s, gates, cands) in enumerate(jobs):
        ga = qvm.GateArray(gates)
        for cand in cands:
            plan = build_plan(ga, n, dtype, cand)
            if plan is None:
                cand = ("block", 3, 0)
                plan = build_plan(ga, n, dtype, cand)
            sv = pool.get(n, dtype)
            _, ms = time_plan(sv, plan)
            feats = plan_features(plan)
            F.append(feats)
            T.append(ms)
            S.append(np.full(len(ms), s, dtype=np.int32))
            C.append(np.full(len(ms), CANDIDATES.index(cand), dtype=np.int32))
        if (i + 1) % 100 == 0:
            print(f"collect: {i + 1}/{len(jobs)} circuits, {sum(len(t) for t in T)} passes, "
                  f"{time.time() - t0:.0f} s", flush=True)
        if (i + 1) % 500 == 0 or i + 1 == len(jobs):
            # rewritten as it grows, so that a cut-short run keeps what it measured
            np.savez_compressed(out_path, features=np.concatenate(F), ms=np.concatenate(T),
                                seed=np.concatenate(S), cand=np.concatenate(C))
    return sum(len(t) for t in T)


def refeature(in_path, out_path, mix=False, n_range=(26, 32), g_range=(100, 500), dtype="c64"):
    """Recompute the pass features of collected timings with the current
    planner (host only): each (circuit seed, candidate) group of rows is
    planned again for scoring and its features replace the stored ones.  The
    timings stay valid as long as the kernels are unchanged; the schedule
    must match pass for pass (same pass count, same features in the columns
    both layouts share)."""
    from workloads import planner_mix_circuit
    z = np.load(in_path, allow_pickle=False)
    F, T, S, C = z["features"], z["ms"], z["seed"], z["cand"]
    out = np.zeros((len(F), NFEAT), dtype=np.float32)
    shared = min(F.shape[1], NFEAT)
    i = 0
    while i < len(F):
        j = i
        while j < len(F) and S[j] == S[i] and C[j] == C[i] and (j == i or F[j, 0] == F[i, 0]):
            j += 1
        seed, cand = int(S[i]), CANDIDATES[int(C[i])]
        if mix:
            n, gates, _ = planner_mix_circuit(seed)
        else:
            n, gates = planner_circuit(seed, n_range, g_range)
        plan = build_plan(qvm.GateArray(gates), n, dtype, cand, image=False)
        f = plan_features(plan)
        # a group may hold several timed runs of one candidate back to back
        reps = (j - i) // len(f)
        if reps < 1 or (j - i) % len(f) or not np.allclose(np.tile(f[:, :shared], (reps, 1)), F[i:j, :shared]):
            raise ValueError(f"rows {i}..{j}: seed {seed} {cand_name(cand)} does not match the plan")
        out[i:j] = np.tile(f, (reps, 1))
        i = j
    np.savez_compressed(out_path, features=out, ms=T, seed=S, cand=C)
    return len(out)


# -------------------------------------------------------------------- model
ADAPTIVE_MARGIN = 0.03


class LearnedPlanner:
    def __init__(self, net, mu, sd, lo=None, hi=None, adaptive_margin=ADAPTIVE_MARGIN):
        self.net, self.mu, self.sd = net, mu, sd
        self.lo, self.hi = lo, hi
        self.adaptive_margin = adaptive_margin

    def predict_pass_ms(self, feats):
        """Predicted ms per pass.  Features are clamped to the range seen in
        training, so a pass beyond it is predicted like the nearest trained
        one instead of by the network's extrapolation."""
        import torch
        if self.lo is not None:
            feats = np.clip(feats, self.lo, self.hi)
        X = torch.tensor((feats - self.mu) / self.sd, dtype=torch.float32, device=self.net.device)
        y = self.net.predict(X).cpu().numpy().astype(np.float64)
        return np.exp(y)

    def predict_plan_ms(self, plan):
        return float(self.predict_pass_ms(plan_features(plan)).sum())

    def choose(self, ga, n, dtype="c64"):
        """Returns (candidate, plan, predicted ms) with the smallest prediction.

        The candidates are planned for scoring only (no block matrices or
        device image) on host threads (the library's planner is reentrant and
        ctypes releases the GIL), all their passes are scored in one MLP
        forward, and only the winner is then built in full (the fallback
        setting is built in full while the others are scored, as it often
        wins).  The fixed settings (SCORED) include tile settings that leave
        narrow trailing blocks to a later pass (DEFER_CANDIDATES).  Beside them, at each tile width of
        ADAPTIVE_TILES the model picks every
        pass's block width: a tile pass takes the same gates whatever its
        width, so pass i of the fixed-width candidates are alternatives for
        the same work and the pass with the smallest prediction is taken
        (candidate ("adaptive", widest k, tile); the widths are in
        plan.k_of_pass)."""
        def scored(c):
            p = build_plan(ga, n, dtype, c, image=c == FALLBACK)
            return (c, p, plan_features(p)) if p is not None else None
        done = [r for r in _pool().map(scored, SCORED) if r is not None]
        live = [(c, p) for c, p, _ in done]
        feats = [f for _, _, f in done]
        rows = np.concatenate(feats)
        if len(rows) == 0:                   # nothing to run: every plan is empty
            c0 = live[0][0]
            return c0, build_plan(ga, n, dtype, c0), 0.0
        ms = self.predict_pass_ms(rows)
        per, o = {}, 0
        for (c, _), f in zip(live, feats):
            per[c] = ms[o:o + len(f)]
            o += len(f)
        options = [(float(v.sum()), c, None) for c, v in per.items()]
        for L in ADAPTIVE_TILES:
            group = [c for c in per if c[0] == "tile" and cand_for_dtype(c, dtype)[2] == L and c[1] in ADAPTIVE_K]
            if len(group) < 2 or len({len(per[c]) for c in group}) != 1 or len(per[group[0]]) == 0:
                continue
            P = np.stack([per[c] for c in group])
            pick = P.argmin(axis=0)
            ks = [group[i][1] for i in pick]
            options.append((float(P.min(axis=0).sum()), ("adaptive", max(ks), L), ks))
        # the per-pass minimum over several predictions is biased low by the
        # model's error: an adaptive plan must beat the fixed settings by a
        # margin to be taken
        pred, cand, ks = min(options, key=lambda t: t[0] * (1.0 + self.adaptive_margin if t[2] else 1.0))
        if cand == FALLBACK and ks is None:
            plan = dict(live)[cand]          # built in full while the others were scored
            plan.k_of_pass = None
            return cand, plan, pred
        plan = build_plan(ga, n, dtype, cand, k_of_pass=ks)
        plan.k_of_pass = ks
        return cand, plan, pred

    def save(self, path):
        extra = {"mu": self.mu, "sd": self.sd}
        if self.lo is not None:
            extra.update(lo=self.lo, hi=self.hi)
        self.net.save(path, extra=extra)

    @classmethod
    def load(cls, path, device="cuda"):
        from .costmodel import CostMLP
        net, z = CostMLP.load(path, device)
        if net.d != NFEAT:
            raise ValueError(f"{path}: model takes {net.d} features, the planner emits {NFEAT}")
        lo = z["lo"] if "lo" in z.files else None
        hi = z["hi"] if "hi" in z.files else None
        return cls(net, z["mu"], z["sd"], lo, hi)


def load_default(device="cuda"):
    """The shipped trained planner, or None when no model file is present or
    it was trained on a different feature layout."""
    if not os.path.exists(DEFAULT_MODEL):
        return None
    with np.load(DEFAULT_MODEL, allow_pickle=False) as z:
        if int(z["d"]) != NFEAT:
            return None
    return LearnedPlanner.load(DEFAULT_MODEL, device)


def combine(paths, out_path):
    """Concatenate collected timing files into one training set; `source`
    gives each row's file index."""
    parts = [np.load(p, allow_pickle=False) for p in paths]
    cols = {k: np.concatenate([z[k] for z in parts]) for k in ("features", "ms", "seed", "cand")}
    cols["source"] = np.concatenate([np.full(len(z["ms"]), i, dtype=np.int32) for i, z in enumerate(parts)])
    if cols["features"].shape[1] != NFEAT:
        raise ValueError(f"features have {cols['features'].shape[1]} columns, the planner emits {NFEAT}")
    np.savez_compressed(out_path, **cols)
    return len(cols["ms"])


def load_rows(*paths):
    F, T = [], []
    for p in paths:
        z = np.load(p, allow_pickle=False)
        F.append(z["features"])
        T.append(z["ms"])
    return np.concatenate(F).astype(np.float32), np.concatenate(T).astype(np.float64)


def train(F, T, epochs=60, batch=4096, lr=2e-3, hidden=128, seed=0, device="cuda", log=True):
    """Fit log(ms) with the HIP MLP; returns (planner, history)."""
    import torch
    from workloads import mlp_init
    from .costmodel import CostMLP
    mu = F.mean(axis=0)
    sd = F.std(axis=0) + 1e-6
    X = torch.tensor((F - mu) / sd, dtype=torch.float32, device=device)
    t = torch.tensor(np.log(T), dtype=torch.float32, device=device)
    net = CostMLP(F.shape[1], hidden, init=mlp_init(F.shape[1], hidden, seed), device=device)
    rng = np.random.Generator(np.random.PCG64(seed))
    hist = []
    nb = max(1, (len(F) + batch - 1) // batch)
    for ep in range(epochs):
        perm = torch.tensor(rng.permutation(len(F)), device=device)
        tot = 0.0
        for b in range(nb):
            idx = perm[b * batch:(b + 1) * batch]
            step_lr = lr * 0.5 * (1 + math.cos(math.pi * (ep * nb + b) / (epochs * nb)))
            tot += float(net.train_step(X[idx].contiguous(), t[idx].contiguous(), step_lr).cpu())
        hist.append(tot / nb)
        if log and (ep % 10 == 0 or ep == epochs - 1):
            print(f"train: epoch {ep} loss {hist[-1]:.4f}", flush=True)
    return LearnedPlanner(net, mu, sd, F.min(axis=0), F.max(axis=0)), hist


# ----------------------------------------------------------------- evaluate
def max_abs_vs_c128(fused, plain, chunk=1 << 26):
    """Max-abs difference of two states over every amplitude (both in the
    identity layout), in chunks."""
    import torch
    n = 1 << fused.n
    worst = 0.0
    for o in range(0, n, chunk):
        m = min(chunk, n - o)
        a = fused.amps[2 * o: 2 * (o + m)].to(torch.float64)
        b = plain.amps[2 * o: 2 * (o + m)]
        d = (a - b).view(m, 2)
        worst = max(worst, float(torch.sqrt((d * d).sum(dim=1)).max()))
    return worst


# fixed settings timed beside the learned choice on held-out circuits: every
# tile setting (the fallback among them) and the classic one block per pass
EVAL_CANDIDATES = [c for c in CANDIDATES if c[0] == "tile"] + DEFER_CANDIDATES + [CLASSIC]


def evaluate(planner, first, count, dtype="c64", reps=2, check=True, n_range=(26, 32),
             g_range=(100, 500), mix=False, log=True, cand_reps=2, cands=None, report=None):
    """Held-out circuits: measured time of the learned choice (best of
    `reps` runs) and of every fixed setting in `cands` (EVAL_CANDIDATES by
    default, best of `cand_reps` runs; the fallback tile-3-13 among them),
    and, with check, the learned plan's whole final state against the plain
    complex128 path.  mix: circuits from the family mixture instead of the
    random planner workload.  report: a JSON file rewritten every ten
    circuits (a cut-short run keeps what it measured)."""
    cands = EVAL_CANDIDATES if cands is None else cands
    import torch
    from workloads import planner_mix_circuit
    if mix:
        jobs = [(planner_mix_circuit(s)[:2], s) for s in range(first, first + count)]
    else:
        jobs = [(planner_circuit(s, n_range, g_range), s) for s in range(first, first + count)]
    jobs.sort(key=lambda j: j[0][0])
    recs = []
    t0 = time.time()
    cur_n, sv = None, None
    for i, ((n, gates), s) in enumerate(jobs):
        if n != cur_n:
            sv = None
            torch.cuda.empty_cache()
            sv = qvm.StateVector(n, dtype, init=0)
            cur_n = n
        ga = qvm.GateArray(gates)
        tp = time.perf_counter()
        cand, plan, pred = planner.choose(ga, n, dtype)
        plan_ms = (time.perf_counter() - tp) * 1e3
        best = lambda p, r: min(time_plan(sv, p)[0] for _ in range(r))
        rec = {"seed": s, "n": n, "gates": len(gates), "choice": cand_name(cand), "pred_ms": pred,
               "plan_ms": plan_ms, "learned_ms": best(plan, reps)}
        if plan.k_of_pass is not None:
            rec["k_of_pass"] = [int(k) for k in plan.k_of_pass]
        allm = {}
        for c in cands:
            p = build_plan(ga, n, dtype, c)
            if p is not None:
                allm[cand_name(c)] = best(p, cand_reps)
        rec["all_ms"] = allm
        if check:
            # the learned plan's whole state against the unfused complex128 path
            sv.init_basis(0)
            plan.run(sv)
            sv.reset_layout()
            plain = qvm.StateVector(n, "c128", init=0)
            plain.run(ga)
            rec["max_abs_err_vs_c128"] = max_abs_vs_c128(sv, plain)
            del plain
            torch.cuda.empty_cache()
        recs.append(rec)
        if (i + 1) % 10 == 0 or i + 1 == len(jobs):
            if report:
                with open(report, "w") as fh:
                    json.dump({"records": recs}, fh)
            if log:
                print(f"evaluate: {i + 1}/{len(jobs)} circuits, {time.time() - t0:.0f} s", flush=True)
    return recs


def _ratios(num, den):
    r = np.asarray(num, dtype=np.float64) / np.asarray(den, dtype=np.float64)
    return {"wins": int(np.sum(r > 1.01)), "losses": int(np.sum(r < 0.99)),
            "ties_within_1pct": int(np.sum((r >= 0.99) & (r <= 1.01))),
            "median_speedup": float(np.median(r)), "geomean_speedup": float(np.exp(np.mean(np.log(r)))),
            "min_speedup": float(r.min()), "max_speedup": float(r.max())}


def summarize(recs):
    """Speed-ups of the learned choice (time of the other / learned time):
    over the fallback setting, over the single fixed setting with the
    smallest total time on these circuits, over the classic one block per
    pass, and the learned time over the best candidate of each circuit."""
    learned = [r["learned_ms"] for r in recs]
    keys = set.intersection(*(set(r["all_ms"]) for r in recs))
    best_fixed = min(keys, key=lambda k: sum(r["all_ms"][k] for r in recs))
    fb, cl = cand_name(FALLBACK), cand_name(CLASSIC)
    out = {"circuits": len(recs),
           "choices": {c: sum(r["choice"] == c for r in recs) for c in sorted({r["choice"] for r in recs})},
           "learned_total_ms": float(sum(learned)),
           "vs_fallback": dict(setting=fb, total_ms=float(sum(r["all_ms"][fb] for r in recs)),
                               **_ratios([r["all_ms"][fb] for r in recs], learned)),
           "vs_best_fixed": dict(setting=best_fixed,
                                 total_ms=float(sum(r["all_ms"][best_fixed] for r in recs)),
                                 **_ratios([r["all_ms"][best_fixed] for r in recs], learned)),
           "learned_over_best_candidate_geomean": float(np.exp(np.mean(np.log(
               [r["learned_ms"] / min(r["all_ms"].values()) for r in recs])))),
           "mean_plan_ms": float(np.mean([r["plan_ms"] for r in recs]))}
    if cl in keys:
        out["vs_classic"] = dict(setting=cl, **_ratios([r["all_ms"][cl] for r in recs], learned))
    errs = [r["max_abs_err_vs_c128"] for r in recs if "max_abs_err_vs_c128" in r]
    if errs:
        out["amplitude_checks"] = len(errs)
        out["max_abs_err_vs_c128"] = float(max(errs))
        out["within_1e-5"] = int(sum(e <= 1e-5 for e in errs))
    return out


def explain(planner, n, gates, x=0, dtype="c64", measure=True):
    """Every candidate's predicted (and, if `measure`, measured) time for one
    circuit; returns (choice, rows)."""
    ga = qvm.GateArray(gates)
    cand, chosen, pred = planner.choose(ga, n, dtype)
    rows = []
    sv = qvm.StateVector(n, dtype, init=0) if measure else None
    for c in CANDIDATES + DEFER_CANDIDATES:
        p = build_plan(ga, n, dtype, c)
        if p is None:
            continue
        rows.append({"candidate": cand_name(c), "predicted_ms": planner.predict_plan_ms(p),
                     "measured_ms": time_plan(sv, p, x)[0] if measure else None})
    choice = {"choice": cand_name(cand), "predicted_ms": pred,
              "measured_ms": time_plan(sv, chosen, x)[0] if measure else None}
    if chosen.k_of_pass is not None:
        choice["k_of_pass"] = chosen.k_of_pass
    return choice, rows


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("cmd", choices=["collect", "refeature", "combine", "train", "evaluate", "explain", "summarize"])
    ap.add_argument("--workload", default="qft30", help="explain: a named workload of workloads.config_circuit")
    ap.add_argument("--first", type=int, default=0)
    ap.add_argument("--count", type=int, default=2000)
    ap.add_argument("--out", default="gpurun_out/planner_train.npz")
    ap.add_argument("--data", nargs="+", default=["gpurun_out/planner_train.npz"])
    ap.add_argument("--model", default="gpurun_out/costmodel.npz")
    ap.add_argument("--epochs", type=int, default=60)
    ap.add_argument("--no-check", action="store_true", help="evaluate: skip the complex128 comparison")
    ap.add_argument("--reports", nargs="+", default=[], help="summarize: evaluation reports to merge")
    ap.add_argument("--report", default="gpurun_out/planner_eval.json")
    ap.add_argument("--no-mix", action="store_true", help="collect: the random planner workload only")
    ap.add_argument("--mix", action="store_true", help="evaluate: circuits from the family mixture")
    a = ap.parse_args()
    if a.cmd == "collect":
        rows = collect(a.first, a.count, a.out, mix=not a.no_mix)
        print(f"collected {rows} pass timings", flush=True)
    elif a.cmd == "refeature":
        rows = refeature(a.data[0], a.out, mix=not a.no_mix)
        print(f"recomputed features of {rows} pass timings", flush=True)
    elif a.cmd == "combine":
        print(f"combined {combine(a.data, a.out)} pass timings", flush=True)
    elif a.cmd == "train":
        F, T = load_rows(*a.data)
        planner, hist = train(F, T, epochs=a.epochs)
        planner.save(a.model)
        print(json.dumps({"rows": len(F), "final_loss": hist[-1]}), flush=True)
    elif a.cmd == "explain":
        from workloads import config_circuit
        cfg = config_circuit(a.workload)
        choice, rows = explain(LearnedPlanner.load(a.model), cfg["n"], cfg["gates"], cfg["init"])
        print(json.dumps(choice), flush=True)
        for r in rows:
            print(json.dumps(r), flush=True)
    elif a.cmd == "evaluate":
        planner = LearnedPlanner.load(a.model)
        recs = evaluate(planner, a.first, a.count, mix=a.mix, check=not a.no_check, report=a.report)
        print(json.dumps(summarize(recs)), flush=True)
    elif a.cmd == "summarize":
        recs = []
        for path in a.reports:
            with open(path) as fh:
                recs += json.load(fh)["records"]
        print(json.dumps(summarize(recs), indent=1), flush=True)


if __name__ == "__main__":
    main()
