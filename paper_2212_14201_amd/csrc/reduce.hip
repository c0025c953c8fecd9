// Readout kernels: norm, probabilities and marginals, <Z_q> for every qubit,
// Pauli-string expectations, sampling, amplitude copies.
//
// All sums are accumulated in double precision (single-precision amplitudes
// are widened before squaring) over a fixed grid and reduced in a fixed
// order, so every readout is bitwise reproducible run to run.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>

#include "internal.hpp"

namespace qvm {

template <typename R> struct C2r;
template <> struct C2r<float> { using T = float2; };
template <> struct C2r<double> { using T = double2; };

struct Perm {
    int n;
    int identity;
    int p[QVM_MAX_QUBITS];            // logical -> physical bit
};

static Perm make_perm(const qvm_sv* sv) {
    Perm P{};
    P.n = sv->n;
    P.identity = 1;
    for (int q = 0; q < sv->n; ++q) {
        P.p[q] = sv->perm[q];
        if (sv->perm[q] != q) P.identity = 0;
    }
    return P;
}

__device__ __forceinline__ uint64_t to_phys(uint64_t l, const Perm& P) {
    if (P.identity) return l;
    uint64_t r = 0;
    for (int q = 0; q < P.n; ++q) r |= ((l >> q) & 1ull) << P.p[q];
    return r;
}

__device__ __forceinline__ uint64_t deposit_r(uint64_t w, uint64_t fixed) {
    while (fixed) {
        uint64_t low = fixed & (~fixed + 1);
        uint64_t lo = w & (low - 1);
        w = ((w - lo) << 1) | lo;
        fixed ^= low;
    }
    return w;
}

template <typename T>
__device__ __forceinline__ double prob(const T& v) {
    double x = (double)v.x, y = (double)v.y;
    return x * x + y * y;
}

// Sum over a 256-thread block; the result is valid in thread 0.
__device__ double block_sum256(double v, double* sh) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) sh[wid] = v;
    __syncthreads();
    return (sh[0] + sh[1]) + (sh[2] + sh[3]);
}

// ------------------------------------------------------------ norm / scale
template <typename R>
__global__ __launch_bounds__(256) void k_norm_partial(const typename C2r<R>::T* __restrict__ psi,
                                                      uint64_t N, double* __restrict__ part) {
    __shared__ double sh[4];
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    double s = 0;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += stride)
        s += prob(psi[i]);
    double r = block_sum256(s, sh);
    if (threadIdx.x == 0) part[(size_t)blockIdx.x * kRedSlots] = r;
}

// Reduce `nv` values over kRedBlocks partial rows into res[0..nv).
__global__ __launch_bounds__(256) void k_final(const double* __restrict__ part, int nv,
                                               double* __restrict__ res) {
    __shared__ double sh[4];
    for (int v = 0; v < nv; ++v) {
        double s = 0;
        for (int b = threadIdx.x; b < kRedBlocks; b += 256) s += part[(size_t)b * kRedSlots + v];
        double r = block_sum256(s, sh);
        if (threadIdx.x == 0) res[v] = r;
        __syncthreads();
    }
}

template <typename R>
__global__ __launch_bounds__(256) void k_scale(typename C2r<R>::T* __restrict__ psi, uint64_t N,
                                               R f) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += stride) {
        auto v = psi[i];
        v.x *= f;
        v.y *= f;
        psi[i] = v;
    }
}

// ----------------------------------------------------- <Z_q> for every q
// part row: [0] = total, [1 + q] = sum of p_i over i with physical bit q set.
template <typename R>
__global__ __launch_bounds__(256) void k_zall_partial(const typename C2r<R>::T* __restrict__ psi,
                                                      int n, double* __restrict__ part) {
    __shared__ double sh[4];
    const uint64_t N = 1ull << n;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;   // 2^19
    const uint64_t gt = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int lowb = n < 19 ? n : 19;   // bits below log2(stride) are fixed per thread
    double total = 0;
    double acc[QVM_MAX_QUBITS];
#pragma unroll
    for (int q = 0; q < QVM_MAX_QUBITS; ++q) acc[q] = 0;
    for (uint64_t i = gt; i < N; i += stride) {
        double p = prob(psi[i]);
        total += p;
#pragma unroll
        for (int q = 19; q < QVM_MAX_QUBITS; ++q)
            if (q < n && ((i >> q) & 1)) acc[q] += p;
    }
#pragma unroll
    for (int q = 0; q < 19; ++q)
        if (q < lowb) acc[q] = ((gt >> q) & 1) ? total : 0.0;
    double r = block_sum256(total, sh);
    if (threadIdx.x == 0) part[(size_t)blockIdx.x * kRedSlots] = r;
#pragma unroll
    for (int q = 0; q < QVM_MAX_QUBITS; ++q) {
        if (q < n) {
            double rq = block_sum256(acc[q], sh);
            if (threadIdx.x == 0) part[(size_t)blockIdx.x * kRedSlots + 1 + q] = rq;
        }
    }
}

// ----------------------------------------------------- Pauli expectations
struct PauliArgs {
    uint64_t x, hbit;
    int nt;
    uint64_t z[32];
};

// For x = 0:   acc_t = sum_i p_i (-1)^{|z_t & i|}.
// For x != 0:  over pairs (i, i^x) with i's hbit = 0, a = conj(psi_{i^x}) psi_i,
//              acc_t = sum (-1)^{|z_t & i|} * (Re a if |x&z_t| even else Im a);
//              the host applies the factor +-2 given by |x & z_t| mod 4.
template <typename R>
__global__ __launch_bounds__(256) void k_pauli_partial(const typename C2r<R>::T* __restrict__ psi,
                                                       uint64_t N, PauliArgs a,
                                                       double* __restrict__ part) {
    __shared__ double sh[4];
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    double acc[32];
#pragma unroll
    for (int t = 0; t < 32; ++t) acc[t] = 0;
    if (a.x == 0) {
        for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += stride) {
            double p = prob(psi[i]);
#pragma unroll
            for (int t = 0; t < 32; ++t)
                if (t < a.nt) acc[t] += (__popcll(a.z[t] & i) & 1) ? -p : p;
        }
    } else {
        const uint64_t items = N >> 1;
        for (uint64_t w = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; w < items; w += stride) {
            uint64_t i = deposit_r(w, a.hbit);
            auto vi = psi[i];
            auto vj = psi[i ^ a.x];
            double ir = vi.x, ii = vi.y, jr = vj.x, ji = vj.y;
            double ar = jr * ir + ji * ii;        // Re conj(psi_j) psi_i
            double ai = jr * ii - ji * ir;        // Im conj(psi_j) psi_i
#pragma unroll
            for (int t = 0; t < 32; ++t) {
                if (t < a.nt) {
                    double v = (__popcll(a.x & a.z[t]) & 1) ? ai : ar;
                    acc[t] += (__popcll(a.z[t] & i) & 1) ? -v : v;
                }
            }
        }
    }
#pragma unroll
    for (int t = 0; t < 32; ++t) {
        if (t < a.nt) {
            double r = block_sum256(acc[t], sh);
            if (threadIdx.x == 0) part[(size_t)blockIdx.x * kRedSlots + t] = r;
        }
    }
}

// --------------------------------------------------------- probabilities
template <typename R>
__global__ __launch_bounds__(256) void k_probs(const typename C2r<R>::T* __restrict__ psi,
                                               uint64_t first, uint64_t cnt, Perm P,
                                               double* __restrict__ out) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t j = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; j < cnt; j += stride)
        out[j] = prob(psi[to_phys(first + j, P)]);
}

// One block per (bucket j, segment s): sums p over the bucket's indices
// i = deposit(o, qmask) | scatter(j), o in the segment.
struct MargArgs {
    uint64_t qmask;
    int m;
    int q[20];
    uint64_t per_bucket;              // 2^(n-m)
    uint64_t seg_len;
    uint32_t segs;
};

template <typename R>
__global__ __launch_bounds__(256) void k_marg_partial(const typename C2r<R>::T* __restrict__ psi,
                                                      MargArgs a, double* __restrict__ part) {
    __shared__ double sh[4];
    const uint64_t blk = blockIdx.x;
    const uint64_t j = blk / a.segs;
    const uint64_t s = blk % a.segs;
    uint64_t jb = 0;
    for (int r = 0; r < a.m; ++r) jb |= ((j >> r) & 1ull) << a.q[r];
    const uint64_t o0 = s * a.seg_len;
    const uint64_t o1 = min(o0 + a.seg_len, a.per_bucket);
    double acc = 0;
    for (uint64_t o = o0 + threadIdx.x; o < o1; o += 256)
        acc += prob(psi[deposit_r(o, a.qmask) | jb]);
    double r = block_sum256(acc, sh);
    if (threadIdx.x == 0) part[blk] = r;
}

__global__ __launch_bounds__(256) void k_marg_final(const double* __restrict__ part,
                                                    uint64_t nb, uint32_t segs,
                                                    double* __restrict__ out) {
    const uint64_t j = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= nb) return;
    double s = 0;
    for (uint32_t k = 0; k < segs; ++k) s += part[j * segs + k];
    out[j] = s;
}

// -------------------------------------------------------------- sampling
template <typename R>
__global__ __launch_bounds__(256) void k_chunk_sums(const typename C2r<R>::T* __restrict__ psi,
                                                    int clog, Perm P, double* __restrict__ csum) {
    __shared__ double sh[4];
    const uint64_t C = 1ull << clog;
    const uint64_t base = (uint64_t)blockIdx.x << clog;
    // the layout map is a bit permutation, so phys(base + j + t) =
    // phys(base) | phys(j) | phys(t) for the block's base, the uniform step j
    // (a multiple of 256) and the thread's t < 256: one OR per element
    const uint64_t pbt = to_phys(base, P) | to_phys(threadIdx.x, P);
    double s = 0;
    for (uint64_t j = 0; j < C; j += 256)
        if (j + threadIdx.x < C) s += prob(psi[pbt | to_phys(j, P)]);
    double r = block_sum256(s, sh);
    if (threadIdx.x == 0) csum[blockIdx.x] = r;
}

// Exclusive prefix over nchunks chunk sums (one block of 1024 threads);
// prefix[nchunks] = total.
__global__ __launch_bounds__(1024) void k_scan_chunks(const double* __restrict__ csum,
                                                      uint64_t nchunks,
                                                      double* __restrict__ prefix) {
    __shared__ double sh[1024];
    const uint64_t per = (nchunks + 1023) / 1024;
    const uint64_t c0 = min((uint64_t)threadIdx.x * per, nchunks);
    const uint64_t c1 = min(c0 + per, nchunks);
    double loc = 0;
    for (uint64_t c = c0; c < c1; ++c) loc += csum[c];
    sh[threadIdx.x] = loc;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        double v = threadIdx.x >= (unsigned)off ? sh[threadIdx.x - off] : 0.0;
        __syncthreads();
        sh[threadIdx.x] += v;
        __syncthreads();
    }
    double run = threadIdx.x ? sh[threadIdx.x - 1] : 0.0;   // exclusive
    for (uint64_t c = c0; c < c1; ++c) {
        prefix[c] = run;
        run += csum[c];
    }
    if (threadIdx.x == 1023) prefix[nchunks] = sh[1023];
}

// One block per sample: locate the chunk by binary search on the prefix,
// then scan the chunk in order.
template <typename R>
__global__ __launch_bounds__(256) void k_find(const typename C2r<R>::T* __restrict__ psi,
                                              int n, int clog, Perm P,
                                              const double* __restrict__ prefix,
                                              uint64_t nchunks, const double* __restrict__ uni,
                                              uint64_t* __restrict__ out) {
    __shared__ double sh[256];
    __shared__ unsigned long long best;
    const uint64_t N = 1ull << n;
    const uint64_t C = 1ull << clog;
    const double total = prefix[nchunks];
    const double target = uni[blockIdx.x] * total;
    // largest c with prefix[c] <= target
    uint64_t lo = 0, hi = nchunks - 1;
    while (lo < hi) {
        uint64_t mid = (lo + hi + 1) >> 1;
        if (prefix[mid] <= target) lo = mid;
        else hi = mid - 1;
    }
    const uint64_t c = lo;
    const uint64_t E = C >= 256 ? C / 256 : 1;
    const uint64_t e0 = min((uint64_t)threadIdx.x * E, C);
    const uint64_t e1 = min(e0 + E, C);
    const uint64_t base = c << clog;
    // e0 is a multiple of E, so phys(base + e0 + k) = phys(base + e0) | phys(k), k < E
    const uint64_t pb0 = to_phys(base + e0, P);
    double loc = 0;
    for (uint64_t e = e0; e < e1; ++e) loc += prob(psi[pb0 | to_phys(e - e0, P)]);
    if (threadIdx.x == 0) best = ~0ull;
    sh[threadIdx.x] = loc;
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {
        double v = threadIdx.x >= (unsigned)off ? sh[threadIdx.x - off] : 0.0;
        __syncthreads();
        sh[threadIdx.x] += v;
        __syncthreads();
    }
    double run = prefix[c] + (threadIdx.x ? sh[threadIdx.x - 1] : 0.0);
    uint64_t cand = ~0ull;
    for (uint64_t e = e0; e < e1; ++e) {
        run += prob(psi[pb0 | to_phys(e - e0, P)]);
        if (run > target) {
            cand = base + e;
            break;
        }
    }
    if (cand != ~0ull) atomicMin(&best, (unsigned long long)cand);
    __syncthreads();
    if (threadIdx.x == 0) {
        uint64_t r = best;
        if (r == ~0ull) r = min(base + C, N - 1);
        out[blockIdx.x] = r;
    }
}

// ------------------------------------------------------------ amplitudes
template <typename R>
__global__ __launch_bounds__(256) void k_copy(const typename C2r<R>::T* __restrict__ psi,
                                              uint64_t first, uint64_t cnt, Perm P,
                                              double2* __restrict__ out) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t j = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; j < cnt; j += stride) {
        auto v = psi[to_phys(first + j, P)];
        out[j] = make_double2((double)v.x, (double)v.y);
    }
}

template <typename R>
__global__ __launch_bounds__(256) void k_gather(const typename C2r<R>::T* __restrict__ psi,
                                                const uint64_t* __restrict__ idx, uint64_t cnt,
                                                Perm P, double2* __restrict__ out) {
    const uint64_t j = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= cnt) return;
    auto v = psi[to_phys(idx[j], P)];
    out[j] = make_double2((double)v.x, (double)v.y);
}

// ------------------------------------------ one qubit's reduced density matrix
// Over the pairs (i, j = i | 2^b) with physical bit b of i clear:
// part row [0] = sum |psi_i|^2, [1] = sum |psi_j|^2, [2] + i [3] = sum psi_i conj(psi_j).
template <typename R>
__global__ __launch_bounds__(256) void k_rdm1_partial(const typename C2r<R>::T* __restrict__ psi,
                                                      uint64_t half, int b, double* __restrict__ part) {
    __shared__ double sh[4];
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    const uint64_t low = (1ull << b) - 1;
    double r00 = 0, r11 = 0, re = 0, im = 0;
    for (uint64_t w = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; w < half; w += stride) {
        const uint64_t i = ((w & ~low) << 1) | (w & low);
        const auto x = psi[i], y = psi[i | (low + 1)];
        const double xr = x.x, xi = x.y, yr = y.x, yi = y.y;
        r00 += xr * xr + xi * xi;
        r11 += yr * yr + yi * yi;
        re += xr * yr + xi * yi;
        im += xi * yr - xr * yi;
    }
    const double v[4] = {r00, r11, re, im};
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        const double t = block_sum256(v[s], sh);
        if (threadIdx.x == 0) part[(size_t)blockIdx.x * kRedSlots + s] = t;
    }
}

// ============================================================ host side
static unsigned grid_of(uint64_t items) {
    uint64_t g = (items + 255) / 256;
    return (unsigned)std::max<uint64_t>(1, std::min<uint64_t>(g, 1u << 20));
}

static double* red_part(qvm_sv* sv) { return (double*)(sv->work + sv->lay.red_off); }
static double* red_res(qvm_sv* sv) { return red_part(sv) + (size_t)kRedBlocks * kRedSlots; }
static char* io(qvm_sv* sv) { return sv->work + sv->lay.io_off; }

static qvm_status fetch(qvm_sv* sv, void* host, const void* dev, size_t bytes) {
    QVM_HIP(sv, hipMemcpyAsync(host, dev, bytes, hipMemcpyDeviceToHost, sv->stream));
    QVM_HIP(sv, hipStreamSynchronize(sv->stream));
    return QVM_OK;
}

template <typename R>
static qvm_status norm_t(qvm_sv* sv, double* out) {
    using T = typename C2r<R>::T;
    uint64_t N = 1ull << sv->n;
    hipLaunchKernelGGL((k_norm_partial<R>), dim3(kRedBlocks), dim3(256), 0, sv->stream,
                       (const T*)sv->amps, N, red_part(sv));
    QVM_LAUNCH_CHECK(sv);
    hipLaunchKernelGGL(k_final, dim3(1), dim3(256), 0, sv->stream, red_part(sv), 1, red_res(sv));
    QVM_LAUNCH_CHECK(sv);
    return fetch(sv, out, red_res(sv), sizeof(double));
}

qvm_status rd_norm(qvm_sv* sv, double* out) {
    return sv->dt == QVM_C64 ? norm_t<float>(sv, out) : norm_t<double>(sv, out);
}

qvm_status rd_scale(qvm_sv* sv, double f) {
    uint64_t N = 1ull << sv->n;
    if (sv->dt == QVM_C64)
        hipLaunchKernelGGL((k_scale<float>), dim3(grid_of(N)), dim3(256), 0, sv->stream,
                           (float2*)sv->amps, N, (float)f);
    else
        hipLaunchKernelGGL((k_scale<double>), dim3(grid_of(N)), dim3(256), 0, sv->stream,
                           (double2*)sv->amps, N, f);
    QVM_LAUNCH_CHECK(sv);
    return QVM_OK;
}

template <typename R>
static qvm_status zall_t(qvm_sv* sv, double* total, double* bit) {
    using T = typename C2r<R>::T;
    hipLaunchKernelGGL((k_zall_partial<R>), dim3(kRedBlocks), dim3(256), 0, sv->stream,
                       (const T*)sv->amps, sv->n, red_part(sv));
    QVM_LAUNCH_CHECK(sv);
    hipLaunchKernelGGL(k_final, dim3(1), dim3(256), 0, sv->stream, red_part(sv), sv->n + 1,
                       red_res(sv));
    QVM_LAUNCH_CHECK(sv);
    double res[QVM_MAX_QUBITS + 1];
    qvm_status st = fetch(sv, res, red_res(sv), sizeof(double) * (sv->n + 1));
    if (st) return st;
    *total = res[0];
    for (int q = 0; q < sv->n; ++q) bit[q] = res[1 + q];
    return QVM_OK;
}

template <typename R>
static qvm_status rdm1_t(qvm_sv* sv, int pbit, double* out) {
    using T = typename C2r<R>::T;
    const int tok = prof_begin(sv);
    hipLaunchKernelGGL((k_rdm1_partial<R>), dim3(kRedBlocks), dim3(256), 0, sv->stream,
                       (const T*)sv->amps, 1ull << (sv->n - 1), pbit, red_part(sv));
    prof_end(sv, tok, PK_RDM1, (double)(1ull << sv->n) * sizeof(T), 8.0 * (double)(1ull << sv->n));
    QVM_LAUNCH_CHECK(sv);
    hipLaunchKernelGGL(k_final, dim3(1), dim3(256), 0, sv->stream, red_part(sv), 4, red_res(sv));
    QVM_LAUNCH_CHECK(sv);
    return fetch(sv, out, red_res(sv), 4 * sizeof(double));
}

qvm_status rd_rdm1(qvm_sv* sv, int pbit, double* out) {
    return sv->dt == QVM_C64 ? rdm1_t<float>(sv, pbit, out) : rdm1_t<double>(sv, pbit, out);
}

qvm_status rd_z_all(qvm_sv* sv, double* total, double* bit) {
    return sv->dt == QVM_C64 ? zall_t<float>(sv, total, bit) : zall_t<double>(sv, total, bit);
}

template <typename R>
static qvm_status pauli_t(qvm_sv* sv, uint64_t x, int nt, const uint64_t* z, double* out) {
    using T = typename C2r<R>::T;
    PauliArgs a{};
    a.x = x;
    a.hbit = x & (~x + 1);
    a.nt = nt;
    for (int t = 0; t < nt; ++t) a.z[t] = z[t];
    hipLaunchKernelGGL((k_pauli_partial<R>), dim3(kRedBlocks), dim3(256), 0, sv->stream,
                       (const T*)sv->amps, 1ull << sv->n, a, red_part(sv));
    QVM_LAUNCH_CHECK(sv);
    hipLaunchKernelGGL(k_final, dim3(1), dim3(256), 0, sv->stream, red_part(sv), nt, red_res(sv));
    QVM_LAUNCH_CHECK(sv);
    double res[32];
    qvm_status st = fetch(sv, res, red_res(sv), sizeof(double) * nt);
    if (st) return st;
    for (int t = 0; t < nt; ++t) {
        if (x == 0) {
            out[t] = res[t];
        } else {
            int c = __builtin_popcountll(x & z[t]) & 3;
            double f = (c == 0 || c == 3) ? 2.0 : -2.0;
            out[t] = f * res[t];
        }
    }
    return QVM_OK;
}

qvm_status rd_pauli_group(qvm_sv* sv, uint64_t x, int nt, const uint64_t* z, double* out) {
    return sv->dt == QVM_C64 ? pauli_t<float>(sv, x, nt, z, out) : pauli_t<double>(sv, x, nt, z, out);
}

template <typename R>
static qvm_status probs_t(qvm_sv* sv, double* out) {
    using T = typename C2r<R>::T;
    const uint64_t N = 1ull << sv->n;
    const uint64_t cap = sv->lay.io_bytes / sizeof(double);
    Perm P = make_perm(sv);
    for (uint64_t f = 0; f < N; f += cap) {
        uint64_t cnt = std::min(cap, N - f);
        hipLaunchKernelGGL((k_probs<R>), dim3(grid_of(cnt)), dim3(256), 0, sv->stream,
                           (const T*)sv->amps, f, cnt, P, (double*)io(sv));
        QVM_LAUNCH_CHECK(sv);
        qvm_status st = fetch(sv, out + f, io(sv), cnt * sizeof(double));
        if (st) return st;
    }
    return QVM_OK;
}

qvm_status rd_probs_full(qvm_sv* sv, double* out) {
    return sv->dt == QVM_C64 ? probs_t<float>(sv, out) : probs_t<double>(sv, out);
}

template <typename R>
static qvm_status marg_t(qvm_sv* sv, int m, const int* pq, double* out) {
    using T = typename C2r<R>::T;
    MargArgs a{};
    a.m = m;
    a.qmask = 0;
    for (int r = 0; r < m; ++r) {
        a.q[r] = pq[r];
        a.qmask |= 1ull << pq[r];
    }
    const int nO = sv->n - m;
    a.per_bucket = 1ull << nO;
    a.segs = nO > 14 ? (1u << (nO - 14)) : 1u;
    a.seg_len = (a.per_bucket + a.segs - 1) / a.segs;
    const uint64_t nb = 1ull << m;
    const uint64_t nblk = nb * a.segs;
    double* part = (double*)io(sv);
    double* res = part + nblk;
    if ((nblk + nb) * sizeof(double) > sv->lay.io_bytes)
        return fail(QVM_ENOMEM, "marginal partials exceed the staging area");
    hipLaunchKernelGGL((k_marg_partial<R>), dim3((unsigned)nblk), dim3(256), 0, sv->stream,
                       (const T*)sv->amps, a, part);
    QVM_LAUNCH_CHECK(sv);
    hipLaunchKernelGGL(k_marg_final, dim3((unsigned)((nb + 255) / 256)), dim3(256), 0, sv->stream,
                       part, nb, a.segs, res);
    QVM_LAUNCH_CHECK(sv);
    return fetch(sv, out, res, nb * sizeof(double));
}

qvm_status rd_marginal(qvm_sv* sv, int m, const int* pq, double* out) {
    return sv->dt == QVM_C64 ? marg_t<float>(sv, m, pq, out) : marg_t<double>(sv, m, pq, out);
}

template <typename R>
static qvm_status sample_t(qvm_sv* sv, size_t ns, const double* u, uint64_t* out) {
    using T = typename C2r<R>::T;
    const int clog = sv->lay.chunk_log;
    const uint64_t nchunks = 1ull << (sv->n - clog);
    double* csum = (double*)(sv->work + sv->lay.chunk_off);
    double* prefix = csum + nchunks;
    Perm P = make_perm(sv);
    hipLaunchKernelGGL((k_chunk_sums<R>), dim3((unsigned)nchunks), dim3(256), 0, sv->stream,
                       (const T*)sv->amps, clog, P, csum);
    QVM_LAUNCH_CHECK(sv);
    hipLaunchKernelGGL(k_scan_chunks, dim3(1), dim3(1024), 0, sv->stream, csum, nchunks, prefix);
    QVM_LAUNCH_CHECK(sv);
    const size_t cap = sv->lay.io_bytes / 16;
    double* du = (double*)io(sv);
    uint64_t* dout = (uint64_t*)(io(sv) + cap * sizeof(double));
    for (size_t s0 = 0; s0 < ns; s0 += cap) {
        size_t cnt = std::min(cap, ns - s0);
        QVM_HIP(sv, hipMemcpyAsync(du, u + s0, cnt * sizeof(double), hipMemcpyHostToDevice,
                                   sv->stream));
        hipLaunchKernelGGL((k_find<R>), dim3((unsigned)cnt), dim3(256), 0, sv->stream,
                           (const T*)sv->amps, sv->n, clog, P, prefix, nchunks, du, dout);
        QVM_LAUNCH_CHECK(sv);
        qvm_status st = fetch(sv, out + s0, dout, cnt * sizeof(uint64_t));
        if (st) return st;
    }
    return QVM_OK;
}

qvm_status rd_sample(qvm_sv* sv, size_t ns, const double* u, uint64_t* out) {
    if (ns == 0) return QVM_OK;
    return sv->dt == QVM_C64 ? sample_t<float>(sv, ns, u, out) : sample_t<double>(sv, ns, u, out);
}

template <typename R>
static qvm_status copy_t(qvm_sv* sv, uint64_t first, uint64_t count, double* out) {
    using T = typename C2r<R>::T;
    const uint64_t cap = sv->lay.io_bytes / 16;
    Perm P = make_perm(sv);
    for (uint64_t f = 0; f < count; f += cap) {
        uint64_t cnt = std::min(cap, count - f);
        hipLaunchKernelGGL((k_copy<R>), dim3(grid_of(cnt)), dim3(256), 0, sv->stream,
                           (const T*)sv->amps, first + f, cnt, P, (double2*)io(sv));
        QVM_LAUNCH_CHECK(sv);
        qvm_status st = fetch(sv, out + 2 * f, io(sv), cnt * 16);
        if (st) return st;
    }
    return QVM_OK;
}

qvm_status rd_copy(qvm_sv* sv, uint64_t first, uint64_t count, double* out) {
    if (!count) return QVM_OK;
    return sv->dt == QVM_C64 ? copy_t<float>(sv, first, count, out)
                             : copy_t<double>(sv, first, count, out);
}

template <typename R>
static qvm_status gather_t(qvm_sv* sv, size_t count, const uint64_t* idx, double* out) {
    using T = typename C2r<R>::T;
    const size_t cap = sv->lay.io_bytes / 24;
    Perm P = make_perm(sv);
    uint64_t* di = (uint64_t*)io(sv);
    double2* dv = (double2*)(io(sv) + ((cap * 8 + 255) & ~size_t(255)));
    for (size_t f = 0; f < count; f += cap) {
        size_t cnt = std::min(cap, count - f);
        QVM_HIP(sv, hipMemcpyAsync(di, idx + f, cnt * 8, hipMemcpyHostToDevice, sv->stream));
        hipLaunchKernelGGL((k_gather<R>), dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0,
                           sv->stream, (const T*)sv->amps, di, cnt, P, dv);
        QVM_LAUNCH_CHECK(sv);
        qvm_status st = fetch(sv, out + 2 * f, dv, cnt * 16);
        if (st) return st;
    }
    return QVM_OK;
}

qvm_status rd_gather(qvm_sv* sv, size_t count, const uint64_t* idx, double* out) {
    if (!count) return QVM_OK;
    return sv->dt == QVM_C64 ? gather_t<float>(sv, count, idx, out)
                             : gather_t<double>(sv, count, idx, out);
}

}  // namespace qvm
