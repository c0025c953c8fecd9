// C ABI entry points: validation, gate lowering, state handles, dispatch.
//
// Gate lowering evaluates angles on the host in double precision with the
// system libm and classifies each gate exactly (from exact zeros and ones of
// its matrix) so that the cheapest kernel that is still exact is chosen:
// phase-only, diagonal, amplitude move (X, CNOT, Toffoli, SWAP: the paper's
// "memory operation" gates in "Performance of basic gates"), or dense.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "internal.hpp"

namespace qvm {

static thread_local std::string g_err;

void set_error(const std::string& msg) { g_err = msg; }

qvm_status fail(qvm_status st, const std::string& msg) {
    g_err = msg;
    return st;
}

qvm_status device_fail(qvm_sv* sv, hipError_t e, const char* where) {
    if (sv) sv->failed = true;
    g_err = std::string("HIP error '") + hipGetErrorString(e) + "' in " + where;
    return QVM_EDEVICE;
}

WorkLayout work_layout(int n, qvm_dtype) {
    WorkLayout L{};
    auto al = [](size_t v) { return (v + 255) & ~size_t(255); };
    size_t off = 0;
    L.red_off = off;
    L.red_bytes = al(sizeof(double) * (size_t)(kRedBlocks + 1) * kRedSlots);
    off += L.red_bytes;
    L.chunk_log = std::max(12, n - 18);
    if (L.chunk_log > n) L.chunk_log = n;
    size_t nchunks = (size_t)1 << (n - L.chunk_log);
    L.chunk_off = off;
    L.chunk_bytes = al(sizeof(double) * (2 * nchunks + 2));
    off += L.chunk_bytes;
    L.io_off = off;
    L.io_bytes = (size_t)16 << 20;
    off += L.io_bytes;
    L.plan_off = off;
    L.plan_bytes = (size_t)32 << 20;
    off += L.plan_bytes;
    L.total = off;
    return L;
}

uint64_t phys_mask(const qvm_sv* sv, uint64_t m) {
    uint64_t r = 0;
    for (int q = 0; q < sv->n; ++q)
        if ((m >> q) & 1) r |= 1ull << sv->perm[q];
    return r;
}

uint64_t phys_index(const qvm_sv* sv, uint64_t l) { return phys_mask(sv, l); }

// ----------------------------------------------------------------- lowering
static int kind_arity(int kind) {
    switch (kind) {
        case QVM_G_RZZ:
        case QVM_G_SWAP: return 2;
        case QVM_G_MATRIX: return 0;
        default: return 1;
    }
}

qvm_status validate_gate(const qvm_gate& g, int n, bool allow_k_gt3) {
    if (g.kind < QVM_G_MATRIX || g.kind > QVM_G_SWAP)
        return fail(QVM_EARG, "unknown gate kind " + std::to_string(g.kind));
    int ar = kind_arity(g.kind);
    if (g.k < 1 || g.k > QVM_MAX_K)
        return fail(QVM_EARG, "gate k=" + std::to_string(g.k) + " outside 1..6");
    if (ar && g.k != ar)
        return fail(QVM_EARG, "gate kind " + std::to_string(g.kind) + " takes " +
                                  std::to_string(ar) + " targets, got " + std::to_string(g.k));
    if (!allow_k_gt3 && g.k > 3)
        return fail(QVM_EUNSUPPORTED, "plain path applies k <= 3; fuse larger blocks");
    if (g.kind == QVM_G_MATRIX && !g.u) return fail(QVM_EARG, "matrix gate with NULL u");
    if (g.kind != QVM_G_MATRIX && g.u) return fail(QVM_EARG, "named gate with non-NULL u");
    uint64_t tm = 0;
    for (int r = 0; r < g.k; ++r) {
        int t = g.targets[r];
        if (t < 0 || t >= n)
            return fail(QVM_ERANGE, "target " + std::to_string(t) + " outside 0.." + std::to_string(n - 1));
        if (tm & (1ull << t)) return fail(QVM_EARG, "duplicate target " + std::to_string(t));
        tm |= 1ull << t;
    }
    if (n < 64 && (g.ctrl_mask >> n))
        return fail(QVM_ERANGE, "control mask names a qubit >= n");
    if (g.ctrl_mask & tm) return fail(QVM_EARG, "control overlaps a target");
    return QVM_OK;
}

qvm_status gate_matrix(const qvm_gate& g, std::vector<cd>& u) {
    const cd I(0.0, 1.0);
    int k = g.kind == QVM_G_MATRIX ? g.k : kind_arity(g.kind);
    int dim = 1 << k;
    u.assign((size_t)dim * dim, cd(0.0, 0.0));
    auto at = [&](int r, int c) -> cd& { return u[(size_t)r * dim + c]; };
    const double th = g.params[0];
    switch (g.kind) {
        case QVM_G_MATRIX:
            for (int i = 0; i < dim * dim; ++i) u[i] = cd(g.u[2 * i], g.u[2 * i + 1]);
            break;
        case QVM_G_I: at(0, 0) = 1.0; at(1, 1) = 1.0; break;
        case QVM_G_H: {
            double h = 1.0 / std::sqrt(2.0);
            at(0, 0) = h; at(0, 1) = h; at(1, 0) = h; at(1, 1) = -h;
            break;
        }
        case QVM_G_X: at(0, 1) = 1.0; at(1, 0) = 1.0; break;
        case QVM_G_Y: at(0, 1) = -I; at(1, 0) = I; break;
        case QVM_G_Z: at(0, 0) = 1.0; at(1, 1) = -1.0; break;
        case QVM_G_S: at(0, 0) = 1.0; at(1, 1) = I; break;
        case QVM_G_SDG: at(0, 0) = 1.0; at(1, 1) = -I; break;
        case QVM_G_T: at(0, 0) = 1.0; at(1, 1) = std::polar(1.0, M_PI / 4); break;
        case QVM_G_TDG: at(0, 0) = 1.0; at(1, 1) = std::polar(1.0, -M_PI / 4); break;
        case QVM_G_RX: {   // cos(t/2) I - i sin(t/2) X
            double c = std::cos(th / 2), s = std::sin(th / 2);
            at(0, 0) = c; at(1, 1) = c; at(0, 1) = cd(0, -s); at(1, 0) = cd(0, -s);
            break;
        }
        case QVM_G_RY: {   // cos(t/2) I - i sin(t/2) Y
            double c = std::cos(th / 2), s = std::sin(th / 2);
            at(0, 0) = c; at(1, 1) = c; at(0, 1) = -s; at(1, 0) = s;
            break;
        }
        case QVM_G_RZ:     // diag(e^{-it/2}, e^{it/2})
            at(0, 0) = std::polar(1.0, -th / 2); at(1, 1) = std::polar(1.0, th / 2);
            break;
        case QVM_G_P: at(0, 0) = 1.0; at(1, 1) = std::polar(1.0, th); break;
        case QVM_G_U3: {
            double c = std::cos(th / 2), s = std::sin(th / 2);
            double phi = g.params[1], lam = g.params[2];
            at(0, 0) = c;
            at(0, 1) = -std::polar(s, lam);
            at(1, 0) = std::polar(s, phi);
            at(1, 1) = std::polar(c, phi + lam);
            break;
        }
        case QVM_G_RZZ:    // e^{-it/2} on even parity, e^{+it/2} on odd parity
            for (int j = 0; j < 4; ++j)
                at(j, j) = std::polar(1.0, (((j ^ (j >> 1)) & 1) ? th : -th) / 2);
            break;
        case QVM_G_SWAP:
            at(0, 0) = 1.0; at(1, 2) = 1.0; at(2, 1) = 1.0; at(3, 3) = 1.0;
            break;
        default:
            return fail(QVM_EARG, "unknown gate kind");
    }
    return QVM_OK;
}

LOp classify(int k, const int* t, uint64_t cmask, const std::vector<cd>& u) {
    LOp op{};
    op.k = k;
    op.cmask = cmask;
    for (int r = 0; r < k; ++r) op.t[r] = t[r];
    int dim = 1 << k;
    auto at = [&](int r, int c) { return u[(size_t)r * dim + c]; };
    const cd one(1.0, 0.0), zero(0.0, 0.0);
    uint64_t tmask = 0;
    for (int r = 0; r < k; ++r) tmask |= 1ull << t[r];
    auto scatter = [&](int j) {     // local index -> physical bit pattern
        uint64_t v = 0;
        for (int r = 0; r < k; ++r)
            if ((j >> r) & 1) v |= 1ull << t[r];
        return v;
    };
    bool diag = true;
    for (int r = 0; r < dim && diag; ++r)
        for (int c = 0; c < dim; ++c)
            if (r != c && at(r, c) != zero) { diag = false; break; }
    if (diag) {
        int nonunit = 0, last = -1;
        for (int j = 0; j < dim; ++j)
            if (at(j, j) != one) { ++nonunit; last = j; }
        if (nonunit <= 1) {
            op.cls = OP_PHASE;
            op.cond_mask = cmask | tmask;
            op.cond_val = cmask | (last >= 0 ? scatter(last) : 0);
            op.phase = last >= 0 ? at(last, last) : one;
            return op;
        }
        op.cls = OP_DIAG;
        op.m.resize(dim);
        for (int j = 0; j < dim; ++j) op.m[j] = at(j, j);
        return op;
    }
    // permutation with unit entries?
    std::vector<int> sigma(dim, -1);   // column c -> row sigma[c]
    bool perm = true;
    for (int c = 0; c < dim && perm; ++c) {
        int cnt = 0;
        for (int r = 0; r < dim; ++r) {
            cd v = at(r, c);
            if (v == zero) continue;
            if (v != one) { perm = false; break; }
            ++cnt;
            sigma[c] = r;
        }
        if (cnt != 1) perm = false;
    }
    if (perm) {
        std::vector<int> moved;
        for (int c = 0; c < dim; ++c)
            if (sigma[c] != c) moved.push_back(c);
        // (a) one transposition
        if (moved.size() == 2 && sigma[moved[0]] == moved[1] && sigma[moved[1]] == moved[0]) {
            int a = moved[0], b = moved[1];
            int xm = a ^ b, h = __builtin_ctz(xm);
            if ((a >> h) & 1) std::swap(a, b);
            op.cls = OP_SWAPPAIR;
            op.xmask = scatter(xm);
            op.cond_mask = cmask | (tmask & ~(1ull << t[h]));
            op.cond_val = cmask | (scatter(a) & ~(1ull << t[h]));
            op.hbit = 1ull << t[h];
            return op;
        }
        // (b) j -> j ^ xm for every j
        int xm = sigma[0];
        bool full = xm != 0;
        for (int c = 0; c < dim && full; ++c)
            if (sigma[c] != (c ^ xm)) full = false;
        if (full) {
            op.cls = OP_SWAPPAIR;
            op.xmask = scatter(xm);
            op.cond_mask = cmask;
            op.cond_val = cmask;
            op.hbit = op.xmask & (~op.xmask + 1);
            return op;
        }
    }
    op.cls = OP_DENSE;
    op.m = u;
    return op;
}

LOp lower(const qvm_sv* sv, const qvm_gate& g, const std::vector<cd>& u) {
    int pt[QVM_MAX_K];
    for (int r = 0; r < g.k; ++r) pt[r] = sv->perm[g.targets[r]];
    return classify(g.k, pt, phys_mask(sv, g.ctrl_mask), u);
}

}  // namespace qvm

using namespace qvm;

#define QVM_CHECK_SV(sv)                                                         \
    do {                                                                         \
        if (!(sv)) return fail(QVM_EARG, "NULL state handle");                   \
        if ((sv)->failed) return fail(QVM_ESTATE, "state handle failed earlier"); \
    } while (0)

extern "C" {

const char* qvm_last_error(void) { return g_err.c_str(); }

qvm_status qvm_gate_matrix(const qvm_gate* g, double* u_out) {
    if (!g || !u_out) return fail(QVM_EARG, "NULL argument");
    qvm_status st = validate_gate(*g, QVM_MAX_QUBITS, true);
    if (st) return st;
    std::vector<cd> u;
    st = gate_matrix(*g, u);
    if (st) return st;
    for (size_t i = 0; i < u.size(); ++i) {
        u_out[2 * i] = u[i].real();
        u_out[2 * i + 1] = u[i].imag();
    }
    return QVM_OK;
}

size_t qvm_workspace_bytes(int n, qvm_dtype dt) {
    if (n < 1 || n > QVM_MAX_QUBITS) return 0;
    return work_layout(n, dt).total;
}

qvm_status qvm_sv_create(int n, qvm_dtype dt, void* amps, void* work, size_t work_bytes,
                         void* stream, qvm_sv** out) {
    if (!out) return fail(QVM_EARG, "NULL out");
    *out = nullptr;
    if (n < 1 || n > QVM_MAX_QUBITS) return fail(QVM_EARG, "n_qubits outside 1..34");
    if (dt != QVM_C64 && dt != QVM_C128) return fail(QVM_EARG, "unknown dtype");
    if (!amps || !work) return fail(QVM_EARG, "NULL device buffer");
    if (((uintptr_t)amps & 255) || ((uintptr_t)work & 255))
        return fail(QVM_EARG, "device buffers must be 256-byte aligned");
    WorkLayout L = work_layout(n, dt);
    if (work_bytes < L.total)
        return fail(QVM_ENOMEM, "workspace has " + std::to_string(work_bytes) + " bytes, needs " +
                                    std::to_string(L.total));
    qvm_sv* sv = new (std::nothrow) qvm_sv();
    if (!sv) return fail(QVM_ENOMEM, "host allocation failed");
    sv->n = n;
    sv->dt = dt;
    sv->amps = amps;
    sv->work = (char*)work;
    sv->work_bytes = work_bytes;
    sv->stream = (hipStream_t)stream;
    for (int q = 0; q < QVM_MAX_QUBITS; ++q) sv->perm[q] = q;
    sv->failed = false;
    sv->lay = L;
    *out = sv;
    return QVM_OK;
}

qvm_status qvm_sv_destroy(qvm_sv* sv) {
    if (sv)
        for (hipEvent_t e : sv->prof.events) (void)hipEventDestroy(e);
    delete sv;
    return QVM_OK;
}

qvm_status qvm_sv_set_stream(qvm_sv* sv, void* stream) {
    QVM_CHECK_SV(sv);
    sv->stream = (hipStream_t)stream;
    return QVM_OK;
}

qvm_status qvm_init_basis(qvm_sv* sv, uint64_t index) {
    QVM_CHECK_SV(sv);
    if (sv->n < 64 && (index >> sv->n)) return fail(QVM_ERANGE, "basis index >= 2^n");
    for (int q = 0; q < QVM_MAX_QUBITS; ++q) sv->perm[q] = q;
    return launch_init_basis(sv, index);
}

qvm_status qvm_apply(qvm_sv* sv, const qvm_gate* g) {
    QVM_CHECK_SV(sv);
    if (!g) return fail(QVM_EARG, "NULL gate");
    qvm_status st = validate_gate(*g, sv->n, false);
    if (st) return st;
    std::vector<cd> u;
    st = gate_matrix(*g, u);
    if (st) return st;
    return launch_op(sv, lower(sv, *g, u));
}

qvm_status qvm_kraus_ops(qvm_channel kind, double p, double t1, double t2, double tgate,
                         double* ops_out, int32_t* n_ops) {
    if (!ops_out || !n_ops) return fail(QVM_EARG, "NULL output");
    using M2 = std::array<cd, 4>;                     // row-major 2x2
    const cd I(0, 1);
    auto pauli = [&](char c, double s) -> M2 {
        switch (c) {
            case 'X': return {0, s, s, 0};
            case 'Y': return {0, -I * s, I * s, 0};
            case 'Z': return {s, 0, 0, -s};
            default: return {s, 0, 0, s};
        }
    };
    auto damping = [](double q) -> std::vector<M2> {
        return {M2{1, 0, 0, std::sqrt(1.0 - q)}, M2{0, std::sqrt(q), 0, 0}};
    };
    auto dephasing = [&](double q) -> std::vector<M2> {
        return {pauli('I', std::sqrt(1.0 - q)), pauli('Z', std::sqrt(q))};
    };
    std::vector<M2> ops;
    if (kind == QVM_K_DECOHERENCE) {
        if (!(t1 > 0 && t2 > 0 && tgate >= 0))
            return fail(QVM_EARG, "decoherence needs T1 > 0, T2 > 0, tgate >= 0");
        if (t2 > 2 * t1) return fail(QVM_EARG, "decoherence needs T2 <= 2 T1 (a non-negative dephasing rate)");
        const double p1 = 1.0 - std::exp(-tgate / t1);
        const double p2 = 0.5 * (1.0 - std::exp(-(tgate / t2 - tgate / (2.0 * t1))));
        for (const M2& a : damping(p1))
            for (const M2& b : dephasing(p2))
                ops.push_back(M2{a[0] * b[0] + a[1] * b[2], a[0] * b[1] + a[1] * b[3],
                                 a[2] * b[0] + a[3] * b[2], a[2] * b[1] + a[3] * b[3]});
    } else {
        if (!(p >= 0.0 && p <= 1.0)) return fail(QVM_ERANGE, "error rate outside [0, 1]");
        switch (kind) {
            case QVM_K_DAMPING: ops = damping(p); break;
            case QVM_K_DEPHASING: ops = dephasing(p); break;
            case QVM_K_DEPOLARIZING:
                ops = {pauli('I', std::sqrt(1.0 - 0.75 * p)), pauli('X', 0.5 * std::sqrt(p)),
                       pauli('Y', 0.5 * std::sqrt(p)), pauli('Z', 0.5 * std::sqrt(p))};
                break;
            case QVM_K_BIT_PHASE_FLIP: ops = {pauli('I', std::sqrt(1.0 - p)), pauli('Y', std::sqrt(p))}; break;
            case QVM_K_BIT_FLIP: ops = {pauli('I', std::sqrt(1.0 - p)), pauli('X', std::sqrt(p))}; break;
            case QVM_K_PHASE_DAMPING: ops = {M2{1, 0, 0, std::sqrt(1.0 - p)}, M2{0, 0, 0, std::sqrt(p)}}; break;
            default: return fail(QVM_EARG, "unknown channel kind");
        }
    }
    for (size_t i = 0; i < ops.size(); ++i)
        for (int e = 0; e < 4; ++e) {
            ops_out[8 * i + 2 * e] = ops[i][e].real();
            ops_out[8 * i + 2 * e + 1] = ops[i][e].imag();
        }
    *n_ops = (int32_t)ops.size();
    return QVM_OK;
}

qvm_status qvm_apply_kraus(qvm_sv* sv, int32_t qubit, int32_t n_ops, const double* ops, double u,
                           int32_t* chosen, double* probs) {
    QVM_CHECK_SV(sv);
    if (qubit < 0 || qubit >= sv->n) return fail(QVM_ERANGE, "qubit >= n");
    if (n_ops < 1 || n_ops > QVM_MAX_KRAUS) return fail(QVM_EARG, "n_ops outside 1..16");
    if (!ops) return fail(QVM_EARG, "NULL Kraus operators");
    if (!(u >= 0.0 && u < 1.0)) return fail(QVM_EARG, "u outside [0, 1)");
    // reduced density matrix of the qubit: rho = [[r00, r01], [conj(r01), r11]]
    double r[4];
    qvm_status st = rd_rdm1(sv, sv->perm[qubit], r);
    if (st) return st;
    const cd r01(r[2], r[3]);
    // p_i = ||K_i psi||^2 = Tr(K_i^dag K_i rho)
    double w[QVM_MAX_KRAUS], total = 0;
    for (int i = 0; i < n_ops; ++i) {
        const double* k = ops + 8 * i;
        const cd a(k[0], k[1]), b(k[2], k[3]), c(k[4], k[5]), d(k[6], k[7]);
        const double m00 = std::norm(a) + std::norm(c), m11 = std::norm(b) + std::norm(d);
        const cd m01 = std::conj(a) * b + std::conj(c) * d;          // (K^dag K)_{01}
        // Tr(M rho) = m00 r00 + m11 r11 + 2 Re(m01 conj(r01))
        w[i] = std::max(0.0, m00 * r[0] + m11 * r[1] + 2.0 * (m01 * std::conj(r01)).real());
        total += w[i];
    }
    if (!(total > 0.0)) return fail(QVM_EARG, "every Kraus branch has zero weight");
    int j = 0;
    for (double acc = w[0]; j < n_ops - 1 && !(acc > u * total); acc += w[++j]) {}
    while (w[j] == 0.0 && j > 0) --j;                 // rounding at the top end
    const double f = std::sqrt(total / w[j]);        // keeps the state's norm
    std::vector<cd> m(4);
    for (int e = 0; e < 4; ++e) m[e] = f * cd(ops[8 * j + 2 * e], ops[8 * j + 2 * e + 1]);
    qvm_gate g{};
    g.kind = QVM_G_MATRIX;
    g.k = 1;
    g.targets[0] = qubit;
    st = launch_op(sv, lower(sv, g, m));
    if (st) return st;
    if (chosen) *chosen = j;
    if (probs)
        for (int i = 0; i < n_ops; ++i) probs[i] = w[i] / total;
    return QVM_OK;
}

qvm_status qvm_run(qvm_sv* sv, const qvm_gate* gates, size_t n_gates) {
    QVM_CHECK_SV(sv);
    if (n_gates && !gates) return fail(QVM_EARG, "NULL gate list");
    for (size_t i = 0; i < n_gates; ++i) {
        qvm_status st = validate_gate(gates[i], sv->n, false);
        if (st) return fail(st, "gate " + std::to_string(i) + ": " + g_err);
    }
    std::vector<cd> u;
    for (size_t i = 0; i < n_gates; ++i) {
        qvm_status st = gate_matrix(gates[i], u);
        if (st) return st;
        st = launch_op(sv, lower(sv, gates[i], u));
        if (st) return st;
    }
    return QVM_OK;
}

qvm_status qvm_get_layout(const qvm_sv* sv, int32_t* perm_out) {
    if (!sv || !perm_out) return fail(QVM_EARG, "NULL argument");
    for (int q = 0; q < sv->n; ++q) perm_out[q] = sv->perm[q];
    return QVM_OK;
}

qvm_status qvm_reset_layout(qvm_sv* sv) {
    QVM_CHECK_SV(sv);
    // selection-sort the layout with physical bit swaps
    for (int q = 0; q < sv->n; ++q) {
        if (sv->perm[q] == q) continue;
        int other = -1;
        for (int r = 0; r < sv->n; ++r)
            if (sv->perm[r] == q) other = r;
        int a = sv->perm[q], b = q;         // physical bits to exchange
        qvm_status st = launch_swap_bits(sv, a, b);
        if (st) return st;
        sv->perm[other] = a;
        sv->perm[q] = b;
    }
    return QVM_OK;
}

qvm_status qvm_norm(qvm_sv* sv, double* out) {
    QVM_CHECK_SV(sv);
    if (!out) return fail(QVM_EARG, "NULL out");
    return rd_norm(sv, out);
}

qvm_status qvm_renormalize(qvm_sv* sv, double* norm_before) {
    QVM_CHECK_SV(sv);
    double nrm = 0;
    qvm_status st = rd_norm(sv, &nrm);
    if (st) return st;
    if (norm_before) *norm_before = nrm;
    if (!(nrm > 0) || !std::isfinite(nrm)) return fail(QVM_ESTATE, "norm is zero or not finite");
    return rd_scale(sv, 1.0 / std::sqrt(nrm));
}

qvm_status qvm_expect_z_all(qvm_sv* sv, double* out) {
    QVM_CHECK_SV(sv);
    if (!out) return fail(QVM_EARG, "NULL out");
    double total = 0, bit[64];
    qvm_status st = rd_z_all(sv, &total, bit);
    if (st) return st;
    for (int q = 0; q < sv->n; ++q) out[q] = total - 2.0 * bit[sv->perm[q]];
    return QVM_OK;
}

qvm_status qvm_expect_pauli(qvm_sv* sv, size_t nt, const uint64_t* x, const uint64_t* z,
                            const double* coeff, double* out_terms, double* out_sum) {
    QVM_CHECK_SV(sv);
    if (nt && (!x || !z)) return fail(QVM_EARG, "NULL mask array");
    if (out_sum && nt && !coeff) return fail(QVM_EARG, "NULL coefficients");
    uint64_t lim = sv->n >= 64 ? ~0ull : ((1ull << sv->n) - 1);
    for (size_t t = 0; t < nt; ++t)
        if ((x[t] & ~lim) || (z[t] & ~lim)) return fail(QVM_ERANGE, "Pauli mask names a qubit >= n");
    std::vector<double> vals(nt, 0.0);
    std::vector<bool> done(nt, false);
    for (size_t t = 0; t < nt; ++t) {
        if (done[t]) continue;
        // group all terms with this x mask
        std::vector<size_t> grp;
        for (size_t u = t; u < nt; ++u)
            if (!done[u] && x[u] == x[t]) grp.push_back(u);
        uint64_t xp = phys_mask(sv, x[t]);
        for (size_t s = 0; s < grp.size(); s += 32) {
            int cnt = (int)std::min<size_t>(32, grp.size() - s);
            uint64_t zp[32];
            double res[32];
            for (int i = 0; i < cnt; ++i) zp[i] = phys_mask(sv, z[grp[s + i]]);
            qvm_status st = rd_pauli_group(sv, xp, cnt, zp, res);
            if (st) return st;
            for (int i = 0; i < cnt; ++i) vals[grp[s + i]] = res[i];
        }
        for (size_t u : grp) done[u] = true;
    }
    if (out_terms)
        for (size_t t = 0; t < nt; ++t) out_terms[t] = vals[t];
    if (out_sum) {
        double s = 0;
        for (size_t t = 0; t < nt; ++t) s += coeff[t] * vals[t];
        *out_sum = s;
    }
    return QVM_OK;
}

qvm_status qvm_probabilities(qvm_sv* sv, int m, const int32_t* qubits, double* out) {
    QVM_CHECK_SV(sv);
    if (!out) return fail(QVM_EARG, "NULL out");
    if (!qubits) {
        if (m != sv->n) return fail(QVM_EARG, "qubits = NULL requires m = n");
        return rd_probs_full(sv, out);
    }
    if (m < 1 || m > sv->n) return fail(QVM_EARG, "m outside 1..n");
    uint64_t seen = 0;
    int pq[QVM_MAX_QUBITS];
    bool ident = (m == sv->n);
    for (int r = 0; r < m; ++r) {
        int q = qubits[r];
        if (q < 0 || q >= sv->n) return fail(QVM_ERANGE, "qubit outside 0..n-1");
        if (seen & (1ull << q)) return fail(QVM_EARG, "duplicate qubit");
        seen |= 1ull << q;
        pq[r] = sv->perm[q];
        if (q != r) ident = false;
    }
    if (ident) return rd_probs_full(sv, out);
    if (m > 20) return fail(QVM_EUNSUPPORTED, "marginals over more than 20 qubits");
    return rd_marginal(sv, m, pq, out);
}

qvm_status qvm_sample(qvm_sv* sv, size_t ns, const double* u, uint64_t* out) {
    QVM_CHECK_SV(sv);
    if (ns && (!u || !out)) return fail(QVM_EARG, "NULL argument");
    for (size_t s = 0; s < ns; ++s)
        if (!(u[s] >= 0.0 && u[s] < 1.0)) return fail(QVM_ERANGE, "uniform outside [0,1)");
    return rd_sample(sv, ns, u, out);
}

qvm_status qvm_copy_amplitudes(qvm_sv* sv, uint64_t first, uint64_t count, double* out) {
    QVM_CHECK_SV(sv);
    if (count && !out) return fail(QVM_EARG, "NULL out");
    uint64_t N = 1ull << sv->n;
    if (first > N || count > N - first) return fail(QVM_ERANGE, "range outside the state");
    return rd_copy(sv, first, count, out);
}

qvm_status qvm_gather_amplitudes(qvm_sv* sv, size_t count, const uint64_t* idx, double* out) {
    QVM_CHECK_SV(sv);
    if (count && (!idx || !out)) return fail(QVM_EARG, "NULL argument");
    uint64_t N = 1ull << sv->n;
    for (size_t i = 0; i < count; ++i)
        if (idx[i] >= N) return fail(QVM_ERANGE, "index >= 2^n");
    return rd_gather(sv, count, idx, out);
}

}  // extern "C"
