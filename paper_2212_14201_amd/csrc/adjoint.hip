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
// All batch elements advance together: one launch per gate covers the whole
// batch (blockIdx.y = batch element).  In the reverse sweep a launch reads
// each amplitude pair of psi and lambda once, accumulates the gradient term
// in double precision and writes back U^dagger applied to both.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "internal.hpp"

namespace qvm {

template <typename R> struct AC2;
template <> struct AC2<float> { using T = float2; };
template <> struct AC2<double> { using T = double2; };

constexpr int kAdjBlocks = 256;       // blocks per batch element (and reduction partials)

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

// One gate on every batch element.  m points at 8 doubles (2x2 complex,
// row-major) per batch element when per_batch, else at one matrix.
// mode 0: psi <- M psi.  mode 1: gradient term (gen 1/2/3 = X/Y/Z, 0 = none)
// from (psi, lam), then psi <- M psi, lam <- M lam (M = U^dagger).
template <typename R>
__global__ __launch_bounds__(256) void k_badj(typename AC2<R>::T* __restrict__ psi,
                                              typename AC2<R>::T* __restrict__ lam,
                                              uint64_t state_len, uint64_t items, uint64_t tbit,
                                              uint64_t cmask, const double* __restrict__ m,
                                              int per_batch, int mode, int gen,
                                              double* __restrict__ part) {
    __shared__ double sh[4];
    const int b = blockIdx.y;
    auto* P = psi + (size_t)b * state_len;
    auto* Lm = lam + (size_t)b * state_len;
    const double* mb = m + (per_batch ? 8 * b : 0);
    const R m00r = (R)mb[0], m00i = (R)mb[1], m01r = (R)mb[2], m01i = (R)mb[3];
    const R m10r = (R)mb[4], m10i = (R)mb[5], m11r = (R)mb[6], m11i = (R)mb[7];
    const uint64_t fixed = tbit | cmask;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    double g = 0;
    for (uint64_t w = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; w < items; w += stride) {
        const uint64_t i0 = adep(w, fixed) | cmask, i1 = i0 | tbit;
        auto a0 = P[i0], a1 = P[i1];
        if (mode == 1) {
            auto l0 = Lm[i0], l1 = Lm[i1];
            // Im( conj(l0) (G psi)_0 + conj(l1) (G psi)_1 ) in double
            const double p0r = a0.x, p0i = a0.y, p1r = a1.x, p1i = a1.y;
            const double q0r = l0.x, q0i = l0.y, q1r = l1.x, q1i = l1.y;
            if (gen == 1) {          // X: (G psi)_0 = psi_1, (G psi)_1 = psi_0
                g += (q0r * p1i - q0i * p1r) + (q1r * p0i - q1i * p0r);
            } else if (gen == 2) {   // Y: (G psi)_0 = -i psi_1, (G psi)_1 = i psi_0
                g += -(q0r * p1r + q0i * p1i) + (q1r * p0r + q1i * p0i);
            } else if (gen == 3) {   // Z: (G psi)_0 = psi_0, (G psi)_1 = -psi_1
                g += (q0r * p0i - q0i * p0r) - (q1r * p1i - q1i * p1r);
            }
            typename AC2<R>::T o0, o1;
            o0.x = m00r * l0.x - m00i * l0.y + m01r * l1.x - m01i * l1.y;
            o0.y = m00r * l0.y + m00i * l0.x + m01r * l1.y + m01i * l1.x;
            o1.x = m10r * l0.x - m10i * l0.y + m11r * l1.x - m11i * l1.y;
            o1.y = m10r * l0.y + m10i * l0.x + m11r * l1.y + m11i * l1.x;
            Lm[i0] = o0;
            Lm[i1] = o1;
        }
        typename AC2<R>::T o0, o1;
        o0.x = m00r * a0.x - m00i * a0.y + m01r * a1.x - m01i * a1.y;
        o0.y = m00r * a0.y + m00i * a0.x + m01r * a1.y + m01i * a1.x;
        o1.x = m10r * a0.x - m10i * a0.y + m11r * a1.x - m11i * a1.y;
        o1.y = m10r * a0.y + m10i * a0.x + m11r * a1.y + m11i * a1.x;
        P[i0] = o0;
        P[i1] = o1;
    }
    if (mode == 1 && gen) {
        const double r = adj_block_sum(g, sh);
        if (threadIdx.x == 0) part[(size_t)b * kAdjBlocks + blockIdx.x] = r;
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
    size_t part_off, part_bytes;     // gradient partials [occ][batch][blocks]
    size_t res_off, res_bytes;       // reduced rows
    size_t fpart_off, total;
};

AdjLayout adj_layout(int batch, size_t n_gates, size_t n_occ) {
    auto al = [](size_t v) { return (v + 255) & ~size_t(255); };
    AdjLayout L{};
    size_t off = 0;
    L.mats_off = off;
    L.mats_bytes = al(2 * n_gates * (size_t)batch * 8 * sizeof(double));
    off += L.mats_bytes;
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
    QVM_HIP(sv, hipMemcpyAsync(dm, mats.data(), mats.size() * sizeof(double), hipMemcpyHostToDevice, stream));
    const dim3 blk(256);
    // every launch uses exactly kAdjBlocks blocks per batch element, so each
    // gradient row gets all its partials written (idle threads add zero)
    auto grid_items = [&](uint64_t) { return (unsigned)kAdjBlocks; };
    // forward
    hipLaunchKernelGGL((k_bzero<R>), dim3(1024), blk, 0, stream, psi, N * (uint64_t)batch, N);
    QVM_LAUNCH_CHECK(sv);
    for (size_t g = 0; g < ng; ++g) {
        const uint64_t tb = 1ull << G[g].target;
        const uint64_t items = 1ull << (n - 1 - __builtin_popcountll(G[g].cmask));
        hipLaunchKernelGGL((k_badj<R>), dim3(grid_items(items), batch), blk, 0, stream, psi, psi, N,
                           items, tb, G[g].cmask, dm + g * batch * 8, 1, 0, 0, part);
        QVM_LAUNCH_CHECK(sv);
    }
    // lambda = H psi, f = Re <psi|lambda>
    for (int ch = 0; ch < n_term_chunks; ++ch) {
        hipLaunchKernelGGL((k_bpauli<R>), dim3((unsigned)std::min<uint64_t>((N + 255) / 256, 4096), batch),
                           blk, 0, stream, psi, lam, N, terms[ch], ch > 0 ? 1 : 0);
        QVM_LAUNCH_CHECK(sv);
    }
    double* fpart = part;   // row block 0 of the partials holds f
    hipLaunchKernelGGL((k_bdot<R>), dim3(kAdjBlocks, batch), blk, 0, stream, psi, lam, N, fpart);
    QVM_LAUNCH_CHECK(sv);
    hipLaunchKernelGGL(k_rows, dim3((batch + 255) / 256), blk, 0, stream, fpart, (uint64_t)batch, res);
    QVM_LAUNCH_CHECK(sv);
    QVM_HIP(sv, hipMemcpyAsync(f_out, res, batch * sizeof(double), hipMemcpyDeviceToHost, stream));
    QVM_HIP(sv, hipStreamSynchronize(stream));
    if (!want_grad) return QVM_OK;
    // reverse sweep: occurrence row o >= 1 for every trainable gate
    std::vector<int> occ_of(ng, -1);
    int n_occ = 0;
    for (size_t g = 0; g < ng; ++g)
        if (G[g].pidx >= 0) occ_of[g] = ++n_occ;
    for (size_t gi = ng; gi-- > 0;) {
        const uint64_t tb = 1ull << G[gi].target;
        const uint64_t items = 1ull << (n - 1 - __builtin_popcountll(G[gi].cmask));
        const int gen = G[gi].pidx >= 0 ? G[gi].gen : 0;
        double* prow = part + (size_t)(occ_of[gi] > 0 ? occ_of[gi] : 0) * batch * kAdjBlocks;
        const unsigned gx = grid_items(items);
        hipLaunchKernelGGL((k_badj<R>), dim3(gx, batch), blk, 0, stream, psi, lam, N, items, tb,
                           G[gi].cmask, dm + (ng + gi) * batch * 8, 1, 1, gen, prow);
        QVM_LAUNCH_CHECK(sv);
    }
    const uint64_t rows = (uint64_t)(n_occ + 1) * batch;
    hipLaunchKernelGGL(k_rows, dim3((unsigned)((rows + 255) / 256)), blk, 0, stream, part, rows, res);
    QVM_LAUNCH_CHECK(sv);
    std::vector<double> r(rows);
    QVM_HIP(sv, hipMemcpyAsync(r.data(), res, rows * sizeof(double), hipMemcpyDeviceToHost, stream));
    QVM_HIP(sv, hipStreamSynchronize(stream));
    std::fill(grad_out, grad_out + (size_t)batch * n_params, 0.0);
    for (size_t g = 0; g < ng; ++g)
        if (occ_of[g] > 0)
            for (int b = 0; b < batch; ++b)
                grad_out[(size_t)b * n_params + G[g].pidx] += r[(size_t)occ_of[g] * batch + b];
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

}  // namespace qvm

using namespace qvm;

extern "C" {

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
    AdjLayout L = adj_layout(batch, G.size(), G.size());
    if (work_bytes < L.total) return adj_fail(QVM_ENOMEM, "workspace too small");
    const bool want = grad_out != nullptr;
    if (dt == QVM_C64)
        return adjoint_t<float>(n, batch, G, n_params, params_host, terms.data(), (int)terms.size(),
                                psi_dev, lam_dev, (char*)work_dev, L, (hipStream_t)hip_stream, want,
                                f_out, grad_out);
    return adjoint_t<double>(n, batch, G, n_params, params_host, terms.data(), (int)terms.size(),
                             psi_dev, lam_dev, (char*)work_dev, L, (hipStream_t)hip_stream, want,
                             f_out, grad_out);
}

}  // extern "C"
