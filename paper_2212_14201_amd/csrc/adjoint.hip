// Batched adjoint (reverse-sweep) gradient of f(theta) = <psi(theta)|H|psi(theta)>
// for circuits of one-target gates (any controls) whose trainable gates are
// RX/RY/RZ rotations U = exp(-i theta G / 2), G in {X, Y, Z} (the paper's
// variational circuits, "Variational quantum circuit"; the method is the
// published reverse sweep of Jones & Gacon, arXiv:2009.02823):
//   psi_L = U_L ... U_1 |0>,  lambda_L = H psi_L,  f = Re <psi_L|lambda_L>,
//   for l = L .. 1:  df/dtheta_l = Im <lambda_l| G_l |psi_l>   (trainable l),
//                    psi <- U_l^dagger psi,  lambda <- U_l^dagger lambda.
// A controlled rotation's generator acts only where its controls are 1.
//
// All batch elements advance together: one launch per gate group covers the
// whole batch (blockIdx.y = batch element).  In the reverse sweep a launch
// reads each amplitude of psi and lambda once, and for every gate of its
// group, last to first, accumulates the gradient term in double precision
// and applies U^dagger to both; then writes them back.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "internal.hpp"

namespace qvm {

template <typename R> struct AC2;
template <> struct AC2<float> { using T = float2; };
template <> struct AC2<double> { using T = double2; };

constexpr int kAdjBlocks = 64;        // blocks per batch element (and reduction partials per row)

__device__ __forceinline__ uint64_t adep(uint64_t w, uint64_t fixed) {
    while (fixed) {
        uint64_t low = fixed & (~fixed + 1);
        uint64_t lo = w & (low - 1);
        w = ((w - lo) << 1) | lo;
        fixed ^= low;
    }
    return w;
}

__device__ double adj_block_sum(double v, double* sh) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) sh[wid] = v;
    __syncthreads();
    return (sh[0] + sh[1]) + (sh[2] + sh[3]);
}

// Gate groups.  The host splits the gate sequence into groups whose gates
// target at most r qubits (the group's slots; controls may sit on any
// qubit) and keeps, for every qubit, the program order of the gates that
// touch it.  A thread owns one item: the 2^r amplitudes of psi (and lambda)
// that differ only in the slot bits, held in registers for the whole group,
// so a group costs one read and one write of each state however many gates
// it holds.  Controls on slot bits are tests of the register index, controls
// on other bits one test of the item's base index.
constexpr int kAdjMaxTrain = 64;      // trainable gates per group
constexpr int kAdjMaxOps = 512;       // gates per group
constexpr int kAdjThreads = 256;

struct AdjOpDev {
    uint64_t cout;     // control bits outside the slots
    int32_t slot;      // target slot
    int32_t cj;        // control bits among the slots, as a mask over slots
    int32_t gate;      // row of the matrix tables
    int32_t gen;       // reverse sweep: 1/2/3 = X/Y/Z generator of a trainable gate, 0 fixed
    int32_t tix;       // index among the group's trainable gates
    int32_t pad;
};

struct AdjGroupArgs {
    uint64_t tbit[4];  // slot s <-> bit tbit[s] of the amplitude index
    uint64_t tmask;    // OR of the slot bits
    int32_t first, count;
    int32_t n_train, row0;   // trainable gates; gradient row of the first one
};

// Im( conj(l0) (G p)_0 + conj(l1) (G p)_1 ) in double for G = X, Y, Z.
template <typename T>
__device__ __forceinline__ double gen_term(int gen, const T& a0, const T& a1, const T& l0, const T& l1) {
    const double p0r = a0.x, p0i = a0.y, p1r = a1.x, p1i = a1.y;
    const double q0r = l0.x, q0i = l0.y, q1r = l1.x, q1i = l1.y;
    if (gen == 1) return (q0r * p1i - q0i * p1r) + (q1r * p0i - q1i * p0r);   // X: (p1, p0)
    if (gen == 2) return -(q0r * p1r + q0i * p1i) + (q1r * p0r + q1i * p0i);  // Y: (-i p1, i p0)
    return (q0r * p0i - q0i * p0r) - (q1r * p1i - q1i * p1r);                  // Z: (p0, -p1)
}

template <typename R, typename T>
__device__ __forceinline__ void mul2(const R* m, T& v0, T& v1) {
    T o0, o1;
    o0.x = m[0] * v0.x - m[1] * v0.y + m[2] * v1.x - m[3] * v1.y;
    o0.y = m[0] * v0.y + m[1] * v0.x + m[2] * v1.y + m[3] * v1.x;
    o1.x = m[4] * v0.x - m[5] * v0.y + m[6] * v1.x - m[7] * v1.y;
    o1.y = m[4] * v0.y + m[5] * v0.x + m[6] * v1.y + m[7] * v1.x;
    v0 = o0;
    v1 = o1;
}

// One gate on target slot S of the registers (pairs j0, j0 | 2^S).  Returns
// the thread's gradient term (reverse sweep, trainable gate) before the
// update.
template <typename R, int NA, int S, bool REV, typename T>
__device__ __forceinline__ double adj_slot(T (&a)[NA], T (&l)[NA], const R* m, int cj, bool cok, int gen) {
    double g = 0;
#pragma unroll
    for (int j0 = 0; j0 < NA; ++j0) {
        if (j0 & (1 << S)) continue;
        constexpr int step = 1 << S;
        const int j1 = j0 | step;
        if (!(cok && (j0 & cj) == cj)) continue;
        if (REV) {
            if (gen) g += gen_term(gen, a[j0], a[j1], l[j0], l[j1]);
            mul2<R>(m, l[j0], l[j1]);
        }
        mul2<R>(m, a[j0], a[j1]);
    }
    return g;
}

template <typename R, int r, bool REV>
__global__ __launch_bounds__(kAdjThreads) void k_adj_group(typename AC2<R>::T* __restrict__ psi,
                                                           typename AC2<R>::T* __restrict__ lam,
                                                           uint64_t state_len, uint64_t items,
                                                           AdjGroupArgs A,
                                                           const AdjOpDev* __restrict__ ops,
                                                           const double* __restrict__ mats, int batch,
                                                           double* __restrict__ part) {
    using T = typename AC2<R>::T;
    constexpr int NA = 1 << r;
    __shared__ double acc[kAdjMaxTrain * (kAdjThreads / 64)];
    const int b = blockIdx.y;
    T* P = psi + (size_t)b * state_len;
    T* Lm = lam + (size_t)b * state_len;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (REV) {
        for (int i = threadIdx.x; i < A.n_train * (kAdjThreads / 64); i += kAdjThreads) acc[i] = 0;
        __syncthreads();
    }
    uint64_t off[NA];
#pragma unroll
    for (int j = 0; j < NA; ++j) {
        uint64_t o = 0;
#pragma unroll
        for (int s = 0; s < r; ++s)
            if (j & (1 << s)) o |= A.tbit[s];
        off[j] = o;
    }
    const uint64_t stride = (uint64_t)gridDim.x * kAdjThreads;
    // the loop bound is uniform over the wave, so every lane takes part in
    // the wave reductions; lanes past the end hold zeros and store nothing
    for (uint64_t w0 = (uint64_t)blockIdx.x * kAdjThreads + wave * 64; w0 < items; w0 += stride) {
        const uint64_t w = w0 + lane;
        const bool act = w < items;
        const uint64_t base = act ? adep(w, A.tmask) : 0;
        T a[NA], l[NA];
#pragma unroll
        for (int j = 0; j < NA; ++j) {
            a[j] = act ? P[base | off[j]] : T{0, 0};
            if (REV) l[j] = act ? Lm[base | off[j]] : T{0, 0};
        }
        for (int oi = 0; oi < A.count; ++oi) {
            const AdjOpDev op = ops[A.first + (REV ? A.count - 1 - oi : oi)];
            const double* md = mats + ((size_t)op.gate * batch + b) * 8;
            R m[8];
#pragma unroll
            for (int i = 0; i < 8; ++i) m[i] = (R)md[i];
            const bool cok = act && (base & op.cout) == op.cout;
            const int gen = REV ? op.gen : 0;
            double g = 0;
            switch (op.slot) {
                case 0: g = adj_slot<R, NA, 0, REV>(a, l, m, op.cj, cok, gen); break;
                case 1: if constexpr (r > 1) g = adj_slot<R, NA, (r > 1 ? 1 : 0), REV>(a, l, m, op.cj, cok, gen); break;
                case 2: if constexpr (r > 2) g = adj_slot<R, NA, (r > 2 ? 2 : 0), REV>(a, l, m, op.cj, cok, gen); break;
                default: if constexpr (r > 3) g = adj_slot<R, NA, (r > 3 ? 3 : 0), REV>(a, l, m, op.cj, cok, gen); break;
            }
            if (REV && gen) {
                for (int o = 32; o > 0; o >>= 1) g += __shfl_down(g, o, 64);
                if (lane == 0) acc[op.tix * (kAdjThreads / 64) + wave] += g;
            }
        }
        if (act) {
#pragma unroll
            for (int j = 0; j < NA; ++j) {
                P[base | off[j]] = a[j];
                if (REV) Lm[base | off[j]] = l[j];
            }
        }
    }
    if (REV) {
        __syncthreads();
        for (int t = threadIdx.x; t < A.n_train; t += kAdjThreads) {
            const double* v = acc + t * (kAdjThreads / 64);
            part[((size_t)(A.row0 + t) * batch + b) * kAdjBlocks + blockIdx.x] = (v[0] + v[1]) + (v[2] + v[3]);
        }
    }
}

// |0..0> in every batch element.
template <typename R>
__global__ __launch_bounds__(256) void k_bzero(typename AC2<R>::T* __restrict__ psi, uint64_t total,
                                               uint64_t state_len) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += stride) {
        typename AC2<R>::T v;
        v.x = (i % state_len) == 0 ? (R)1 : (R)0;
        v.y = 0;
        psi[i] = v;
    }
}

struct PauliTerms {
    int nt;
    uint64_t x[48], z[48];
    double c[48];
};

// lam = sum_t c_t P_t psi, with (P psi)_i = i^{|x&z|} (-1)^{|z&(i^x)|} psi_{i^x}.
template <typename R>
__global__ __launch_bounds__(256) void k_bpauli(const typename AC2<R>::T* __restrict__ psi,
                                                typename AC2<R>::T* __restrict__ lam,
                                                uint64_t state_len, PauliTerms T, int accumulate) {
    const int b = blockIdx.y;
    const auto* P = psi + (size_t)b * state_len;
    auto* Lm = lam + (size_t)b * state_len;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < state_len; i += stride) {
        R sr = 0, si = 0;
        if (accumulate) {
            sr = Lm[i].x;
            si = Lm[i].y;
        }
        for (int t = 0; t < T.nt; ++t) {
            const uint64_t j = i ^ T.x[t];
            const auto v = P[j];
            R vr = v.x, vi = v.y;
            if (__popcll(T.z[t] & j) & 1) { vr = -vr; vi = -vi; }
            R wr = vr, wi = vi;
            switch (__popcll(T.x[t] & T.z[t]) & 3) {
                case 1: wr = -vi; wi = vr; break;
                case 2: wr = -vr; wi = -vi; break;
                case 3: wr = vi; wi = -vr; break;
                default: break;
            }
            sr += (R)T.c[t] * wr;
            si += (R)T.c[t] * wi;
        }
        typename AC2<R>::T o;
        o.x = sr;
        o.y = si;
        Lm[i] = o;
    }
}

// part[b][blk] = partial Re <psi|lam> of batch element b.
template <typename R>
__global__ __launch_bounds__(256) void k_bdot(const typename AC2<R>::T* __restrict__ psi,
                                              const typename AC2<R>::T* __restrict__ lam,
                                              uint64_t state_len, double* __restrict__ part) {
    __shared__ double sh[4];
    const int b = blockIdx.y;
    const auto* P = psi + (size_t)b * state_len;
    const auto* Lm = lam + (size_t)b * state_len;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    double s = 0;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < state_len; i += stride)
        s += (double)P[i].x * (double)Lm[i].x + (double)P[i].y * (double)Lm[i].y;
    const double r = adj_block_sum(s, sh);
    if (threadIdx.x == 0) part[(size_t)b * kAdjBlocks + blockIdx.x] = r;
}

// out[r] = sum over kAdjBlocks partials of row r, in order.
__global__ __launch_bounds__(256) void k_rows(const double* __restrict__ part, uint64_t rows,
                                              double* __restrict__ out) {
    const uint64_t r = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= rows) return;
    double s = 0;
    for (int k = 0; k < kAdjBlocks; ++k) s += part[r * kAdjBlocks + k];
    out[r] = s;
}

namespace {

struct AdjGate {
    int target;
    uint64_t cmask;
    int pidx;          // -1: fixed
    int gen;           // 1/2/3 for trainable X/Y/Z rotations
    std::vector<cd> u; // fixed gates: 2x2
};

struct AdjLayout {
    size_t mats_off, mats_bytes;     // per-(gate, batch) 2x2 matrices, forward then dagger
    size_t ops_off, ops_bytes;       // group op table
    size_t part_off, part_bytes;     // gradient partials [row][batch][blocks]
    size_t res_off, res_bytes;       // reduced rows
    size_t total;
};

AdjLayout adj_layout(int batch, size_t n_gates, size_t n_occ) {
    auto al = [](size_t v) { return (v + 255) & ~size_t(255); };
    AdjLayout L{};
    size_t off = 0;
    L.mats_off = off;
    L.mats_bytes = al(2 * n_gates * (size_t)batch * 8 * sizeof(double));
    off += L.mats_bytes;
    L.ops_off = off;
    L.ops_bytes = al((n_gates + 1) * sizeof(AdjOpDev));
    off += L.ops_bytes;
    L.part_off = off;
    L.part_bytes = al((n_occ + 1) * (size_t)batch * kAdjBlocks * sizeof(double));
    off += L.part_bytes;
    L.res_off = off;
    L.res_bytes = al((n_occ + 1) * (size_t)batch * sizeof(double));
    off += L.res_bytes;
    L.total = off;
    return L;
}

qvm_status adj_fail(qvm_status st, const std::string& m) { return fail(st, "adjoint: " + m); }

struct HostGroup {
    AdjGroupArgs args;
    std::vector<int> gates;          // in program order
};

// Split the gate sequence into groups of at most r target qubits.  Each
// group scans the gates not yet placed, in program order, and takes a gate
// when none of its qubits is held by a gate the scan has passed over (so
// the order of gates that share a qubit is kept: gates that share no qubit
// commute) and its target is a slot or a slot is free.  Slots left free are
// filled with the highest unused qubits, so that the item index runs over
// the low bits and a wave's loads stay contiguous.
std::vector<HostGroup> adj_groups(const std::vector<AdjGate>& G, int n, int r) {
    std::vector<HostGroup> out;
    std::vector<char> done(G.size(), 0);
    size_t left = G.size(), first = 0;
    while (left) {
        HostGroup h{};
        int nb = 0, ntrain = 0;
        int bits[4] = {0, 0, 0, 0};
        uint64_t blocked = 0, tset = 0;
        for (size_t i = first; i < G.size(); ++i) {
            if (done[i]) continue;
            const uint64_t tb = 1ull << G[i].target;
            const uint64_t q = tb | G[i].cmask;
            bool ok = !(q & blocked);
            if (ok && !(tset & tb) && nb == r) ok = false;
            if (ok && G[i].pidx >= 0 && ntrain == kAdjMaxTrain) ok = false;
            if (ok && (int)h.gates.size() == kAdjMaxOps) ok = false;
            if (!ok) {
                blocked |= q;
                continue;
            }
            if (!(tset & tb)) {
                tset |= tb;
                bits[nb++] = G[i].target;
            }
            h.gates.push_back((int)i);
            done[i] = 1;
            --left;
            if (G[i].pidx >= 0) ++ntrain;
        }
        while (first < G.size() && done[first]) ++first;
        for (int q = n - 1; nb < r && q >= 0; --q)
            if (!(tset >> q & 1)) {
                tset |= 1ull << q;
                bits[nb++] = q;
            }
        for (int s = 0; s < 4; ++s) h.args.tbit[s] = s < r ? 1ull << bits[s] : 0;
        h.args.tmask = tset;
        h.args.n_train = ntrain;
        out.push_back(std::move(h));
    }
    return out;
}

// Slots (target qubits) per gate group: complex64 holds 2 x 16 amplitudes
// per thread (160 VGPRs), complex128 2 x 8 (four slots would take all 256
// and leave one wave per SIMD).
int adj_slots(int n, qvm_dtype dt) { return std::min(dt == QVM_C64 ? 4 : 3, n); }

}  // namespace

template <typename R>
static qvm_status adjoint_t(int n, int batch, const std::vector<AdjGate>& G, int n_params,
                            const double* params, const PauliTerms* terms, int n_term_chunks,
                            void* psi_dev, void* lam_dev, char* work, const AdjLayout& L,
                            hipStream_t stream, bool want_grad, double* f_out, double* grad_out) {
    using T = typename AC2<R>::T;
    T* psi = (T*)psi_dev;
    T* lam = (T*)lam_dev;
    const uint64_t N = 1ull << n;
    qvm_sv dummy{};
    qvm_sv* sv = &dummy;      // for the error macros only
    // matrices: forward M and dagger M^H for every (gate, batch element)
    const size_t ng = G.size();
    std::vector<double> mats(2 * ng * (size_t)batch * 8);
    for (size_t g = 0; g < ng; ++g) {
        for (int b = 0; b < batch; ++b) {
            cd u[4];
            if (G[g].pidx < 0) {
                for (int i = 0; i < 4; ++i) u[i] = G[g].u[i];
            } else {
                const double th = params[(size_t)b * n_params + G[g].pidx];
                const double c = std::cos(th / 2), s = std::sin(th / 2);
                if (G[g].gen == 1) { u[0] = c; u[1] = cd(0, -s); u[2] = cd(0, -s); u[3] = c; }
                else if (G[g].gen == 2) { u[0] = c; u[1] = -s; u[2] = s; u[3] = c; }
                else { u[0] = std::polar(1.0, -th / 2); u[1] = 0; u[2] = 0; u[3] = std::polar(1.0, th / 2); }
            }
            double* f = &mats[((g * batch) + b) * 8];
            double* d = &mats[(((ng + g) * batch) + b) * 8];
            for (int i = 0; i < 4; ++i) {
                f[2 * i] = u[i].real();
                f[2 * i + 1] = u[i].imag();
            }
            const cd h[4] = {std::conj(u[0]), std::conj(u[2]), std::conj(u[1]), std::conj(u[3])};
            for (int i = 0; i < 4; ++i) {
                d[2 * i] = h[i].real();
                d[2 * i + 1] = h[i].imag();
            }
        }
    }
    double* dm = (double*)(work + L.mats_off);
    double* part = (double*)(work + L.part_off);
    double* res = (double*)(work + L.res_off);
    AdjOpDev* dops = (AdjOpDev*)(work + L.ops_off);
    // gate groups and their op table; gradient rows follow the group order
    const int r = adj_slots(n, sizeof(R) == 4 ? QVM_C64 : QVM_C128);
    std::vector<HostGroup> groups = adj_groups(G, n, r);
    std::vector<AdjOpDev> optab;
    std::vector<int> row_gate;        // gradient row (from 1) -> gate
    row_gate.push_back(-1);
    for (HostGroup& h : groups) {
        h.args.first = (int)optab.size();
        h.args.count = (int)h.gates.size();
        h.args.row0 = (int)row_gate.size();
        int tix = 0;
        for (int gi : h.gates) {
            AdjOpDev o{};
            o.gate = gi;
            o.slot = -1;
            o.cout = G[gi].cmask;
            for (int s = 0; s < r; ++s) {
                if (h.args.tbit[s] == (1ull << G[gi].target)) o.slot = s;
                if (G[gi].cmask & h.args.tbit[s]) {
                    o.cj |= 1 << s;
                    o.cout &= ~h.args.tbit[s];
                }
            }
            o.gen = G[gi].pidx >= 0 ? G[gi].gen : 0;
            o.tix = G[gi].pidx >= 0 ? tix++ : -1;
            if (G[gi].pidx >= 0) row_gate.push_back(gi);
            optab.push_back(o);
        }
    }
    QVM_HIP(sv, hipMemcpyAsync(dm, mats.data(), mats.size() * sizeof(double), hipMemcpyHostToDevice, stream));
    if (!optab.empty())
        QVM_HIP(sv, hipMemcpyAsync(dops, optab.data(), optab.size() * sizeof(AdjOpDev),
                                   hipMemcpyHostToDevice, stream));
    const dim3 blk(256);
    const uint64_t items = 1ull << (n - r);
    auto launch_group = [&](const HostGroup& h, bool rev) -> qvm_status {
        const dim3 grid(kAdjBlocks, batch);
        const double* mt = dm + (rev ? ng : 0) * (size_t)batch * 8;
#define QVM_ADJ_LAUNCH(RR)                                                                           \
    if (rev)                                                                                         \
        hipLaunchKernelGGL((k_adj_group<R, RR, true>), grid, blk, 0, stream, psi, lam, N, items,     \
                           h.args, dops, mt, batch, part);                                           \
    else                                                                                             \
        hipLaunchKernelGGL((k_adj_group<R, RR, false>), grid, blk, 0, stream, psi, lam, N, items,    \
                           h.args, dops, mt, batch, part);
        switch (r) {
            case 1: QVM_ADJ_LAUNCH(1) break;
            case 2: QVM_ADJ_LAUNCH(2) break;
            case 3: QVM_ADJ_LAUNCH(3) break;
            default: QVM_ADJ_LAUNCH(4) break;
        }
#undef QVM_ADJ_LAUNCH
        QVM_LAUNCH_CHECK(sv);
        return QVM_OK;
    };
    // forward
    hipLaunchKernelGGL((k_bzero<R>), dim3(1024), blk, 0, stream, psi, N * (uint64_t)batch, N);
    QVM_LAUNCH_CHECK(sv);
    for (const HostGroup& h : groups) {
        qvm_status st = launch_group(h, false);
        if (st) return st;
    }
    // lambda = H psi, f = Re <psi|lambda>
    for (int ch = 0; ch < n_term_chunks; ++ch) {
        hipLaunchKernelGGL((k_bpauli<R>), dim3((unsigned)std::min<uint64_t>((N + 255) / 256, 4096), batch),
                           blk, 0, stream, psi, lam, N, terms[ch], ch > 0 ? 1 : 0);
        QVM_LAUNCH_CHECK(sv);
    }
    double* fpart = part;   // row 0 of the partials holds f
    hipLaunchKernelGGL((k_bdot<R>), dim3(kAdjBlocks, batch), blk, 0, stream, psi, lam, N, fpart);
    QVM_LAUNCH_CHECK(sv);
    hipLaunchKernelGGL(k_rows, dim3((batch + 255) / 256), blk, 0, stream, fpart, (uint64_t)batch, res);
    QVM_LAUNCH_CHECK(sv);
    QVM_HIP(sv, hipMemcpyAsync(f_out, res, batch * sizeof(double), hipMemcpyDeviceToHost, stream));
    QVM_HIP(sv, hipStreamSynchronize(stream));
    if (!want_grad) return QVM_OK;
    // reverse sweep: groups in reverse order, gates in reverse inside each
    for (size_t gi = groups.size(); gi-- > 0;) {
        qvm_status st = launch_group(groups[gi], true);
        if (st) return st;
    }
    const uint64_t rows = (uint64_t)row_gate.size() * batch;
    if (row_gate.size() > 1) {
        hipLaunchKernelGGL(k_rows, dim3((unsigned)((rows + 255) / 256)), blk, 0, stream, part, rows, res);
        QVM_LAUNCH_CHECK(sv);
    }
    std::vector<double> rv(rows);
    QVM_HIP(sv, hipMemcpyAsync(rv.data(), res, rows * sizeof(double), hipMemcpyDeviceToHost, stream));
    QVM_HIP(sv, hipStreamSynchronize(stream));
    std::fill(grad_out, grad_out + (size_t)batch * n_params, 0.0);
    for (size_t row = 1; row < row_gate.size(); ++row)
        for (int b = 0; b < batch; ++b)
            grad_out[(size_t)b * n_params + G[row_gate[row]].pidx] += rv[row * batch + b];
    return QVM_OK;
}

static qvm_status adj_prepare(int n, int batch, const qvm_gate* gates, size_t n_gates,
                              const int32_t* param_index, int n_params, size_t n_terms,
                              const uint64_t* x, const uint64_t* z, const double* c,
                              std::vector<AdjGate>& G, std::vector<PauliTerms>& terms) {
    if (n < 1 || n > QVM_MAX_QUBITS) return adj_fail(QVM_EARG, "n_qubits outside 1..34");
    if (batch < 1 || batch > 65535) return adj_fail(QVM_EARG, "batch outside 1..65535");
    if (n_gates && (!gates || !param_index)) return adj_fail(QVM_EARG, "NULL gate list");
    if (n_params < 0) return adj_fail(QVM_EARG, "negative n_params");
    if (n_terms < 1 || !x || !z || !c) return adj_fail(QVM_EARG, "empty or NULL observable");
    const uint64_t lim = (n >= 64) ? ~0ull : ((1ull << n) - 1);
    for (size_t t = 0; t < n_terms; ++t)
        if ((x[t] & ~lim) || (z[t] & ~lim)) return adj_fail(QVM_ERANGE, "Pauli mask names a qubit >= n");
    G.clear();
    for (size_t i = 0; i < n_gates; ++i) {
        qvm_status st = validate_gate(gates[i], n, true);
        if (st) return fail(st, "adjoint gate " + std::to_string(i) + ": " + qvm_last_error());
        if (gates[i].k != 1) return adj_fail(QVM_EUNSUPPORTED, "gate " + std::to_string(i) + " has k != 1");
        AdjGate a{};
        a.target = gates[i].targets[0];
        a.cmask = gates[i].ctrl_mask;
        a.pidx = param_index[i];
        if (a.pidx >= n_params) return adj_fail(QVM_ERANGE, "parameter index >= n_params");
        if (a.pidx >= 0) {
            switch (gates[i].kind) {
                case QVM_G_RX: a.gen = 1; break;
                case QVM_G_RY: a.gen = 2; break;
                case QVM_G_RZ: a.gen = 3; break;
                default: return adj_fail(QVM_EARG, "trainable gate " + std::to_string(i) + " is not RX/RY/RZ");
            }
        } else {
            a.pidx = -1;
            st = gate_matrix(gates[i], a.u);
            if (st) return st;
        }
        G.push_back(std::move(a));
    }
    terms.clear();
    for (size_t t0 = 0; t0 < n_terms; t0 += 48) {
        PauliTerms T{};
        T.nt = (int)std::min<size_t>(48, n_terms - t0);
        for (int t = 0; t < T.nt; ++t) {
            T.x[t] = x[t0 + t];
            T.z[t] = z[t0 + t];
            T.c[t] = c[t0 + t];
        }
        terms.push_back(T);
    }
    return QVM_OK;
}

// Trainable gates: the gradient rows the sweep fills (plus row 0, f).
size_t adj_trainable(const std::vector<AdjGate>& G) {
    size_t t = 0;
    for (const AdjGate& g : G) t += g.pidx >= 0;
    return t;
}

qvm_status adj_dispatch(int n, qvm_dtype dt, int batch, const std::vector<AdjGate>& G, int n_params,
                        const double* params_host, const std::vector<PauliTerms>& terms, void* psi_dev,
                        void* lam_dev, char* work, const AdjLayout& L, void* hip_stream, double* f_out,
                        double* grad_out);

// Workspace of qvm_adjoint_expect_grad_static: one array per device, held
// until the process ends.  Host code never passes the array's name to a
// kernel or a copy (on the host it is only a stand-in for the symbol): its
// device address is looked up once per device, with that device current,
// and kept below.  Every entry a call reads is written earlier in the same
// call (matrices and op table copied in, each reduction partial stored by
// its block), so nothing needs clearing between calls.
static __device__ __align__(256) char scratch[QVM_ADJ_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
static char* g_scratch_dev[kMaxDevices] = {};
static std::mutex g_scratch_mu;

qvm_status adj_scratch(char** out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail(QVM_EDEVICE, std::string("adjoint: hipGetDevice: ") + hipGetErrorString(e));
    if (dev < 0 || dev >= kMaxDevices) return adj_fail(QVM_EUNSUPPORTED, "device index above 63");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(QVM_EDEVICE, std::string("adjoint: hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        g_scratch_dev[dev] = (char*)p;
    }
    *out = g_scratch_dev[dev];
    return QVM_OK;
}

}  // namespace qvm

using namespace qvm;

extern "C" {

qvm_status qvm_adjoint_group_count(int n, qvm_dtype dt, const qvm_gate* gates, size_t n_gates,
                                   const int32_t* param_index, int n_params, int32_t* n_groups) {
    if (dt != QVM_C64 && dt != QVM_C128) return adj_fail(QVM_EARG, "unknown dtype");
    if (!n_groups) return adj_fail(QVM_EARG, "NULL output");
    std::vector<AdjGate> G;
    std::vector<PauliTerms> terms;
    const uint64_t z = 0;
    const double c = 0;
    qvm_status st = adj_prepare(n, 1, gates, n_gates, param_index, n_params, 1, &z, &z, &c, G, terms);
    if (st) return st;
    *n_groups = (int32_t)adj_groups(G, n, adj_slots(n, dt)).size();
    return QVM_OK;
}

size_t qvm_adjoint_workspace_bytes(int n_qubits, int batch, size_t n_gates) {
    (void)n_qubits;
    return adj_layout(batch, n_gates, n_gates).total;
}

qvm_status qvm_adjoint_expect_grad(int n, qvm_dtype dt, int batch, const qvm_gate* gates,
                                   size_t n_gates, const int32_t* param_index, int n_params,
                                   const double* params_host, size_t n_terms, const uint64_t* x_mask,
                                   const uint64_t* z_mask, const double* coeff, void* psi_dev,
                                   void* lam_dev, void* work_dev, size_t work_bytes, void* hip_stream,
                                   double* f_out, double* grad_out) {
    if (dt != QVM_C64 && dt != QVM_C128) return adj_fail(QVM_EARG, "unknown dtype");
    if (!psi_dev || !lam_dev || !work_dev || !f_out) return adj_fail(QVM_EARG, "NULL buffer");
    if (n_params > 0 && !params_host) return adj_fail(QVM_EARG, "NULL parameters");
    if (psi_dev == lam_dev) return adj_fail(QVM_EARG, "psi and lambda must not alias");
    std::vector<AdjGate> G;
    std::vector<PauliTerms> terms;
    qvm_status st = adj_prepare(n, batch, gates, n_gates, param_index, n_params, n_terms, x_mask,
                                z_mask, coeff, G, terms);
    if (st) return st;
    const AdjLayout L = adj_layout(batch, G.size(), adj_trainable(G));
    if (work_bytes < L.total) return adj_fail(QVM_ENOMEM, "workspace too small");
    return adj_dispatch(n, dt, batch, G, n_params, params_host, terms, psi_dev, lam_dev, (char*)work_dev, L,
                        hip_stream, f_out, grad_out);
}

qvm_status qvm_adjoint_expect_grad_static(int n, qvm_dtype dt, int batch, const qvm_gate* gates,
                                          size_t n_gates, const int32_t* param_index, int n_params,
                                          const double* params_host, size_t n_terms,
                                          const uint64_t* x_mask, const uint64_t* z_mask,
                                          const double* coeff, void* psi_dev, void* lam_dev,
                                          void* hip_stream, double* f_out, double* grad_out) {
    if (dt != QVM_C64 && dt != QVM_C128) return adj_fail(QVM_EARG, "unknown dtype");
    if (!psi_dev || !lam_dev || !f_out) return adj_fail(QVM_EARG, "NULL buffer");
    if (n_params > 0 && !params_host) return adj_fail(QVM_EARG, "NULL parameters");
    if (psi_dev == lam_dev) return adj_fail(QVM_EARG, "psi and lambda must not alias");
    std::vector<AdjGate> G;
    std::vector<PauliTerms> terms;
    qvm_status st = adj_prepare(n, batch, gates, n_gates, param_index, n_params, n_terms, x_mask,
                                z_mask, coeff, G, terms);
    if (st) return st;
    const AdjLayout L = adj_layout(batch, G.size(), adj_trainable(G));
    if (L.total > QVM_ADJ_SCRATCH_BYTES)
        return adj_fail(QVM_ENOMEM, "needs " + std::to_string(L.total) + " bytes of workspace, the static "
                        "scratch holds " + std::to_string((size_t)QVM_ADJ_SCRATCH_BYTES));
    char* work = nullptr;
    st = adj_scratch(&work);
    if (st) return st;
    return adj_dispatch(n, dt, batch, G, n_params, params_host, terms, psi_dev, lam_dev, work, L, hip_stream,
                        f_out, grad_out);
}

}  // extern "C"

namespace qvm {

qvm_status adj_dispatch(int n, qvm_dtype dt, int batch, const std::vector<AdjGate>& G, int n_params,
                        const double* params_host, const std::vector<PauliTerms>& terms, void* psi_dev,
                        void* lam_dev, char* work, const AdjLayout& L, void* hip_stream, double* f_out,
                        double* grad_out) {
    const bool want = grad_out != nullptr;
    if (dt == QVM_C64)
        return adjoint_t<float>(n, batch, G, n_params, params_host, terms.data(), (int)terms.size(),
                                psi_dev, lam_dev, work, L, (hipStream_t)hip_stream, want, f_out, grad_out);
    return adjoint_t<double>(n, batch, G, n_params, params_host, terms.data(), (int)terms.size(),
                             psi_dev, lam_dev, work, L, (hipStream_t)hip_stream, want, f_out, grad_out);
}

}  // namespace qvm
