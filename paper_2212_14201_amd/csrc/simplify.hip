// Peephole pre-pass before fusion (paper, "Quantum circuit optimization",
// first layer): identity pairs are removed and consecutive rotations about
// the same axis are merged into one rotation by the sum of their angles,
// any number of them in a row.
//
// Two gates are consecutive when they act on the same qubits (targets and
// controls) and no gate between them touches any of those qubits.  Rules,
// for gates with identical targets and identical controls:
//   cancel   H H, X X, Y Y, Z Z, SWAP SWAP (either target order), S SDG,
//            SDG S, T TDG, TDG T; I is dropped
//   merge    RX RX, RY RY, RZ RZ, P P, RZZ RZZ (either target order):
//            angles add; a sum of exactly 0 drops the gate
//   combine  T T -> S, TDG TDG -> SDG, S S -> Z, SDG SDG -> Z
// A combined or merged gate is compared again with the gate before it, so
// chains collapse (H S S H -> H Z H; RZ(a) RZ(-a) X X -> nothing).  Every
// rule is an exact matrix identity; merged angles are rounded sums.
#include <algorithm>
#include <cstring>
#include <string>
#include <vector>

#include "internal.hpp"

namespace qvm {
namespace {

uint64_t qubits_of(const qvm_gate& g) {
    uint64_t m = g.ctrl_mask;
    for (int r = 0; r < g.k; ++r) m |= 1ull << g.targets[r];
    return m;
}

bool same_targets(const qvm_gate& a, const qvm_gate& b, bool unordered) {
    if (a.k != b.k || a.ctrl_mask != b.ctrl_mask) return false;
    if (a.k == 2 && unordered)
        return (a.targets[0] == b.targets[0] && a.targets[1] == b.targets[1]) ||
               (a.targets[0] == b.targets[1] && a.targets[1] == b.targets[0]);
    for (int r = 0; r < a.k; ++r)
        if (a.targets[r] != b.targets[r]) return false;
    return true;
}

enum class Pair { none, cancel, merge, become };

// What the consecutive pair (a, b) (a first) reduces to; for `become`,
// *kind receives the single gate's kind.
Pair rule(const qvm_gate& a, const qvm_gate& b, int32_t* kind) {
    const int ka = a.kind, kb = b.kind;
    const bool sym = ka == QVM_G_SWAP || ka == QVM_G_RZZ;
    if (!same_targets(a, b, sym)) return Pair::none;
    if (ka == kb) {
        switch (ka) {
            case QVM_G_H: case QVM_G_X: case QVM_G_Y: case QVM_G_Z: case QVM_G_SWAP:
                return Pair::cancel;
            case QVM_G_RX: case QVM_G_RY: case QVM_G_RZ: case QVM_G_P: case QVM_G_RZZ:
                return Pair::merge;
            case QVM_G_T: *kind = QVM_G_S; return Pair::become;
            case QVM_G_TDG: *kind = QVM_G_SDG; return Pair::become;
            case QVM_G_S: case QVM_G_SDG: *kind = QVM_G_Z; return Pair::become;
            default: return Pair::none;
        }
    }
    if ((ka == QVM_G_S && kb == QVM_G_SDG) || (ka == QVM_G_SDG && kb == QVM_G_S) ||
        (ka == QVM_G_T && kb == QVM_G_TDG) || (ka == QVM_G_TDG && kb == QVM_G_T))
        return Pair::cancel;
    return Pair::none;
}

}  // namespace
}  // namespace qvm

using namespace qvm;

extern "C" qvm_status qvm_simplify(const qvm_gate* in, size_t n_in, int n_qubits, qvm_gate* out,
                                   size_t* n_out) {
    if (!n_out) return fail(QVM_EARG, "NULL n_out");
    *n_out = 0;
    if (n_qubits < 1 || n_qubits > QVM_MAX_QUBITS) return fail(QVM_EARG, "n_qubits outside 1..34");
    if (n_in && (!in || !out)) return fail(QVM_EARG, "NULL gate array");
    try {
        for (size_t i = 0; i < n_in; ++i) {
            qvm_status st = validate_gate(in[i], n_qubits, true);
            if (st) return fail(st, "gate " + std::to_string(i) + ": " + std::string(qvm_last_error()));
        }
        std::vector<qvm_gate> g;                   // kept gates, in order (dead ones marked k = -1)
        g.reserve(n_in);
        std::vector<std::vector<int>> top(n_qubits);   // per qubit: kept gates touching it, in order
        auto last_on = [&](uint64_t mask) -> int {
            int j = -2;                            // -2: unset, -1: qubits disagree or none
            for (int q = 0; q < n_qubits; ++q) {
                if (!((mask >> q) & 1)) continue;
                const int t = top[q].empty() ? -1 : top[q].back();
                if (j == -2) j = t;
                else if (j != t) return -1;
            }
            return j < 0 ? -1 : j;
        };
        auto push = [&](const qvm_gate& x) {
            g.push_back(x);
            const uint64_t m = qubits_of(x);
            for (int q = 0; q < n_qubits; ++q)
                if ((m >> q) & 1) top[q].push_back((int)g.size() - 1);
        };
        auto pop = [&](int j) {
            const uint64_t m = qubits_of(g[j]);
            for (int q = 0; q < n_qubits; ++q)
                if ((m >> q) & 1) top[q].pop_back();
            g[j].k = -1;
        };
        for (size_t i = 0; i < n_in; ++i) {
            qvm_gate cur = in[i];
            if (cur.kind == QVM_G_I) continue;
            for (;;) {
                const uint64_t m = qubits_of(cur);
                const int j = last_on(m);
                if (j < 0 || qubits_of(g[j]) != m) {
                    push(cur);
                    break;
                }
                int32_t kind = 0;
                const Pair p = rule(g[j], cur, &kind);
                if (p == Pair::none) {
                    push(cur);
                    break;
                }
                qvm_gate prev = g[j];
                pop(j);
                if (p == Pair::cancel) break;
                if (p == Pair::merge) {
                    prev.params[0] += cur.params[0];
                    if (prev.params[0] == 0.0) break;
                    cur = prev;                    // compare the merged gate with the one before
                } else {
                    prev.kind = kind;
                    cur = prev;
                }
            }
        }
        size_t o = 0;
        for (const qvm_gate& x : g)
            if (x.k >= 0) out[o++] = x;
        *n_out = o;
        return QVM_OK;
    } catch (const std::exception& e) {
        return fail(QVM_ENOMEM, e.what());
    }
}
