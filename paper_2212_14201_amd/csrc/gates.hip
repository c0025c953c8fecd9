// Plain per-gate kernels: one pass over the amplitudes per gate.
//
// Every kernel enumerates exactly the amplitudes a gate changes: a work
// index w is spread over the free bits of the amplitude index ("deposit"),
// and the fixed bits (targets at 0, controls at 1, or a phase/move
// condition) are OR-ed in.  Lanes take consecutive w, so accesses stay
// coalesced whenever the lowest physical bits are free bits.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "internal.hpp"

namespace qvm {

template <typename R> struct C2;
template <> struct C2<float> { using T = float2; };
template <> struct C2<double> { using T = double2; };

// Spread the bits of w over the zero bits of `fixed` (ascending order).
__device__ __forceinline__ uint64_t deposit(uint64_t w, uint64_t fixed) {
    while (fixed) {
        uint64_t low = fixed & (~fixed + 1);
        uint64_t lo = w & (low - 1);
        w = ((w - lo) << 1) | lo;
        fixed ^= low;
    }
    return w;
}

template <typename R, int K> struct DenseArgs {
    uint64_t items, fixed, cmask;
    uint64_t off[1 << K];
    R m[2 << (2 * K)];               // 2^K x 2^K complex, row-major (re, im)
};

// Access kind.  Measured on MI355X, an in-place read-modify-write of a
// large buffer streams fastest with one 16-byte item per thread and
// nontemporal loads and stores (6.6 TB/s, against 5.3-5.7 TB/s with 2-8
// items per thread or with ordinary accesses); the state is touched once per
// gate, so caching it gains nothing.
constexpr int kTPB = 256;                    // threads per block of the plain kernels

typedef float nt_f2 __attribute__((ext_vector_type(2)));
typedef double nt_d2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ float2 ld_stream(const float2* p) {
    const nt_f2 v = __builtin_nontemporal_load((const nt_f2*)p);
    return make_float2(v.x, v.y);
}
__device__ __forceinline__ double2 ld_stream(const double2* p) {
    const nt_d2 v = __builtin_nontemporal_load((const nt_d2*)p);
    return make_double2(v.x, v.y);
}
__device__ __forceinline__ void st_stream(float2* p, float2 v) {
    __builtin_nontemporal_store(nt_f2{v.x, v.y}, (nt_f2*)p);
}
__device__ __forceinline__ void st_stream(double2* p, double2 v) {
    __builtin_nontemporal_store(nt_d2{v.x, v.y}, (nt_d2*)p);
}

template <typename R, int K>
__global__ __launch_bounds__(kTPB) void k_dense(typename C2<R>::T* __restrict__ psi,
                                                DenseArgs<R, K> a) {
    using T = typename C2<R>::T;
    constexpr int D = 1 << K;
    const uint64_t stride = (uint64_t)gridDim.x * kTPB;
    for (uint64_t w = (uint64_t)blockIdx.x * kTPB + threadIdx.x; w < a.items; w += stride) {
        const uint64_t b = deposit(w, a.fixed) | a.cmask;
        T v[D];
#pragma unroll
        for (int j = 0; j < D; ++j) v[j] = ld_stream(psi + b + a.off[j]);
#pragma unroll
        for (int i = 0; i < D; ++i) {
            R re = 0, im = 0;
#pragma unroll
            for (int j = 0; j < D; ++j) {
                R mr = a.m[2 * (i * D + j)], mi = a.m[2 * (i * D + j) + 1];
                re += mr * v[j].x - mi * v[j].y;
                im += mr * v[j].y + mi * v[j].x;
            }
            T o;
            o.x = re;
            o.y = im;
            st_stream(psi + b + a.off[i], o);
        }
    }
}

// A one-qubit complex128 gate with one amplitude (one 16-byte piece) per
// lane, the streaming shape above: lanes 0-31 of a wave load the first
// amplitude of 32 consecutive pairs, lanes 32-63 the second; partners trade
// their values across the wave's halves (lane ^ 32) and each lane writes its
// own row of the 2 x 2 product.  The loop runs per wave, so every lane of a
// wave takes part in the exchange; lanes past the end store nothing.
__global__ __launch_bounds__(kTPB) void k_dense1_lanes(double2* __restrict__ psi, DenseArgs<double, 1> a) {
    const int lane = threadIdx.x & 63, h = lane >> 5;
    const uint64_t waves = (a.items + 31) / 32;
    const uint64_t wstride = (uint64_t)gridDim.x * (kTPB / 64);
    const double r0 = a.m[4 * h], i0 = a.m[4 * h + 1], r1 = a.m[4 * h + 2], i1 = a.m[4 * h + 3];
    for (uint64_t wv = (uint64_t)blockIdx.x * (kTPB / 64) + (threadIdx.x >> 6); wv < waves; wv += wstride) {
        const uint64_t w = wv * 32 + (lane & 31);
        const bool act = w < a.items;
        const uint64_t idx = (deposit(act ? w : 0, a.fixed) | a.cmask) + a.off[h];
        const double2 v = act ? ld_stream(psi + idx) : make_double2(0.0, 0.0);
        const double2 u = make_double2(__shfl_xor(v.x, 32, 64), __shfl_xor(v.y, 32, 64));
        const double2 v0 = h ? u : v, v1 = h ? v : u;
        double2 o;
        o.x = r0 * v0.x - i0 * v0.y + r1 * v1.x - i1 * v1.y;
        o.y = r0 * v0.y + i0 * v0.x + r1 * v1.y + i1 * v1.x;
        if (act) st_stream(psi + idx, o);
    }
}

template <typename R> struct DiagArgs {
    uint64_t items, cmask;
    int k;
    int t[3];
    R d[16];                          // up to 2^3 complex entries
};

template <typename R>
__global__ __launch_bounds__(kTPB) void k_diag(typename C2<R>::T* __restrict__ psi, DiagArgs<R> a) {
    using T = typename C2<R>::T;
    const uint64_t stride = (uint64_t)gridDim.x * kTPB;
    for (uint64_t w = (uint64_t)blockIdx.x * kTPB + threadIdx.x; w < a.items; w += stride) {
        const uint64_t idx = deposit(w, a.cmask) | a.cmask;
        const T v = ld_stream(psi + idx);
        int j = 0;
        for (int r = 0; r < a.k; ++r) j |= (int)((idx >> a.t[r]) & 1) << r;
        const R dr = a.d[2 * j], di = a.d[2 * j + 1];
        T o;
        o.x = dr * v.x - di * v.y;
        o.y = dr * v.y + di * v.x;
        st_stream(psi + idx, o);
    }
}

template <typename R>
__global__ __launch_bounds__(kTPB) void k_phase(typename C2<R>::T* __restrict__ psi, uint64_t items,
                                                uint64_t cmask, uint64_t cval, R pr, R pi) {
    using T = typename C2<R>::T;
    const uint64_t stride = (uint64_t)gridDim.x * kTPB;
    for (uint64_t w = (uint64_t)blockIdx.x * kTPB + threadIdx.x; w < items; w += stride) {
        const uint64_t idx = deposit(w, cmask) | cval;
        const T v = ld_stream(psi + idx);
        T o;
        o.x = pr * v.x - pi * v.y;
        o.y = pr * v.y + pi * v.x;
        st_stream(psi + idx, o);
    }
}

// A phase whose condition includes index bits inside a 128-byte line (bits
// 0..2 of complex128, 0..3 of complex64).  Enumerating only the matching
// amplitudes spreads a wave's 64 accesses over 2 to 16 times as many lines,
// each fetched whole, and stores runs shorter than 64 bytes (measured: a CZ
// on qubits 0, 1 of a 30-qubit complex128 state runs 6.6x slower than one
// on qubits 28, 29, at 24 GiB of HBM traffic for 8 GiB of algorithmic
// bytes); instead the kernel walks the lines whose bits above the line
// match, one 16-byte piece per thread (a wave reads whole lines), and stores
// either the pieces that hold a matching amplitude (all = 0: the matching
// runs are 64 bytes or longer) or every piece, unchanged ones included
// (all = 1: a full-line write streams faster than short runs).
template <typename R>
__global__ __launch_bounds__(kTPB) void k_phase_lines(typename C2<R>::T* __restrict__ psi, uint64_t items,
                                                      uint64_t hmask, uint64_t hval, uint32_t lmask,
                                                      uint32_t lval, R pr, R pi, int all) {
    using T = typename C2<R>::T;
    constexpr int LB = sizeof(R) == 8 ? 3 : 4;          // amplitude-index bits inside a line
    constexpr int PB = sizeof(R) == 8 ? 0 : 1;          // amplitude-index bits inside a piece
    constexpr uint64_t PM = (1u << (LB - PB)) - 1;       // piece within the line
    const uint64_t stride = (uint64_t)gridDim.x * kTPB;
    for (uint64_t w = (uint64_t)blockIdx.x * kTPB + threadIdx.x; w < items; w += stride) {
        const uint64_t line = deposit(w >> (LB - PB), hmask) | hval;     // hmask, hval: bits above the line
        const uint64_t idx = (line << LB) | ((w & PM) << PB);
        if constexpr (PB == 0) {
            const bool m = ((uint32_t)idx & lmask) == lval;
            if (!m && !all) continue;
            const T v = ld_stream(psi + idx);
            T o = v;
            if (m) {
                o.x = pr * v.x - pi * v.y;
                o.y = pr * v.y + pi * v.x;
            }
            st_stream(psi + idx, o);
        } else {
            const bool m0 = ((uint32_t)idx & lmask) == lval, m1 = ((uint32_t)(idx | 1) & lmask) == lval;
            if (!m0 && !m1 && !all) continue;
            typedef float f4 __attribute__((ext_vector_type(4)));
            const f4 v = __builtin_nontemporal_load((const f4*)(psi + idx));   // amplitudes idx, idx + 1
            f4 o = v;
            if (m0) {
                o.x = pr * v.x - pi * v.y;
                o.y = pr * v.y + pi * v.x;
            }
            if (m1) {
                o.z = pr * v.z - pi * v.w;
                o.w = pr * v.w + pi * v.z;
            }
            __builtin_nontemporal_store(o, (f4*)(psi + idx));
        }
    }
}

template <typename R>
__global__ __launch_bounds__(kTPB) void k_swappair(typename C2<R>::T* __restrict__ psi, uint64_t items,
                                                   uint64_t fixed, uint64_t cval, uint64_t xmask) {
    using T = typename C2<R>::T;
    const uint64_t stride = (uint64_t)gridDim.x * kTPB;
    for (uint64_t w = (uint64_t)blockIdx.x * kTPB + threadIdx.x; w < items; w += stride) {
        const uint64_t idx = deposit(w, fixed) | cval;
        const T a = ld_stream(psi + idx), b = ld_stream(psi + (idx ^ xmask));
        st_stream(psi + idx, b);
        st_stream(psi + (idx ^ xmask), a);
    }
}

// The complex128 form with one amplitude per lane: lanes 0-31 of a wave
// take 32 consecutive pairs' first amplitudes, lanes 32-63 their partners,
// and each lane stores its amplitude at its partner's index.  The wave's
// load completes for every lane before its store is issued (the store
// waits for the loaded value), so no lane overwrites an amplitude another
// lane has still to read; different waves touch different pairs.
__global__ __launch_bounds__(kTPB) void k_swappair_lanes(double2* __restrict__ psi, uint64_t items,
                                                         uint64_t fixed, uint64_t cval, uint64_t xmask) {
    const int lane = threadIdx.x & 63, h = lane >> 5;
    const uint64_t waves = (items + 31) / 32;
    const uint64_t wstride = (uint64_t)gridDim.x * (kTPB / 64);
    for (uint64_t wv = (uint64_t)blockIdx.x * (kTPB / 64) + (threadIdx.x >> 6); wv < waves; wv += wstride) {
        const uint64_t w = wv * 32 + (lane & 31);
        if (w >= items) continue;
        const uint64_t idx = deposit(w, fixed) | cval;
        const uint64_t mine = h ? idx ^ xmask : idx;
        st_stream(psi + (mine ^ xmask), ld_stream(psi + mine));
    }
}

template <typename R>
__global__ __launch_bounds__(256) void k_basis(typename C2<R>::T* __restrict__ psi, uint64_t N,
                                               uint64_t idx) {
    using T = typename C2<R>::T;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += stride) {
        T v;
        v.x = i == idx ? (R)1 : (R)0;
        v.y = 0;
        st_stream(psi + i, v);
    }
}

// Blocks for `items` work items, one per thread, capped at 2^23 blocks: a
// dispatch holds its size in work items as a 32-bit value, so at most 2^31
// threads are launched and the kernels loop over the rest (a 34-qubit state
// has up to 2^34 items; below 32 qubits every thread takes one item).
constexpr uint64_t kMaxBlocks = 1ull << 23;
static unsigned grid_for(uint64_t items) {
    const uint64_t g = (items + kTPB - 1) / kTPB;
    return (unsigned)std::max<uint64_t>(1, std::min<uint64_t>(g, kMaxBlocks));
}

static inline int popc(uint64_t v) { return __builtin_popcountll(v); }

template <typename R, int K>
static qvm_status launch_dense_k(qvm_sv* sv, const LOp& op) {
    using T = typename C2<R>::T;
    DenseArgs<R, K> a{};
    uint64_t tmask = 0;
    for (int r = 0; r < K; ++r) tmask |= 1ull << op.t[r];
    a.fixed = tmask | op.cmask;
    a.cmask = op.cmask;
    a.items = 1ull << (sv->n - popc(a.fixed));
    for (int j = 0; j < (1 << K); ++j) {
        uint64_t o = 0;
        for (int r = 0; r < K; ++r)
            if ((j >> r) & 1) o |= 1ull << op.t[r];
        a.off[j] = o;
    }
    for (int i = 0; i < (1 << (2 * K)); ++i) {
        a.m[2 * i] = (R)op.m[i].real();
        a.m[2 * i + 1] = (R)op.m[i].imag();
    }
    const double touched = (double)a.items * (1 << K);
    const int tok = prof_begin(sv);
    if constexpr (K == 1 && sizeof(R) == 8)
        hipLaunchKernelGGL(k_dense1_lanes, dim3(grid_for(2 * a.items)), dim3(kTPB), 0, sv->stream,
                           (T*)sv->amps, a);
    else
        hipLaunchKernelGGL((k_dense<R, K>), dim3(grid_for(a.items)), dim3(kTPB), 0, sv->stream,
                           (T*)sv->amps, a);
    QVM_LAUNCH_CHECK(sv);
    prof_end(sv, tok, PK_DENSE1 + K - 1, 2.0 * touched * sizeof(T), touched * 8.0 * (1 << K));
    return QVM_OK;
}

template <typename R>
static qvm_status launch_op_t(qvm_sv* sv, const LOp& op) {
    using T = typename C2<R>::T;
    switch (op.cls) {
        case OP_PHASE: {
            if (op.phase == cd(1.0, 0.0)) return QVM_OK;   // identity
            uint64_t items = 1ull << (sv->n - popc(op.cond_mask));
            const int tok = prof_begin(sv);
            constexpr int LB = sizeof(R) == 8 ? 3 : 4, PB = sizeof(R) == 8 ? 0 : 1;
            const uint64_t lowm = (1ull << LB) - 1;
            if ((op.cond_mask & lowm) && sv->n >= LB) {
                // condition bits inside the lines: whole lines, pieces that match
                const uint64_t hmask = op.cond_mask >> LB;
                const uint64_t pieces = 1ull << (sv->n - LB - popc(hmask) + (LB - PB));
                // matching runs span 2^(lowest condition bit) amplitudes
                const int low = __builtin_ctzll(op.cond_mask);
                const int all = ((size_t)sizeof(T) << low) < 64 ? 1 : 0;
                hipLaunchKernelGGL((k_phase_lines<R>), dim3(grid_for(pieces)), dim3(kTPB), 0, sv->stream,
                                   (T*)sv->amps, pieces, hmask, op.cond_val >> LB, (uint32_t)(op.cond_mask & lowm),
                                   (uint32_t)(op.cond_val & lowm), (R)op.phase.real(), (R)op.phase.imag(), all);
            } else {
                hipLaunchKernelGGL((k_phase<R>), dim3(grid_for(items)), dim3(kTPB), 0, sv->stream,
                                   (T*)sv->amps, items, op.cond_mask, op.cond_val,
                                   (R)op.phase.real(), (R)op.phase.imag());
            }
            QVM_LAUNCH_CHECK(sv);
            prof_end(sv, tok, PK_PHASE, 2.0 * items * sizeof(T), 6.0 * items);
            return QVM_OK;
        }
        case OP_DIAG: {
            if (op.k > 3) return fail(QVM_EUNSUPPORTED, "diagonal gate with k > 3 on the plain path");
            DiagArgs<R> a{};
            a.cmask = op.cmask;
            a.items = 1ull << (sv->n - popc(op.cmask));
            a.k = op.k;
            for (int r = 0; r < op.k; ++r) a.t[r] = op.t[r];
            for (int j = 0; j < (1 << op.k); ++j) {
                a.d[2 * j] = (R)op.m[j].real();
                a.d[2 * j + 1] = (R)op.m[j].imag();
            }
            const int tok = prof_begin(sv);
            hipLaunchKernelGGL((k_diag<R>), dim3(grid_for(a.items)), dim3(kTPB), 0, sv->stream,
                               (T*)sv->amps, a);
            QVM_LAUNCH_CHECK(sv);
            prof_end(sv, tok, PK_DIAG, 2.0 * a.items * sizeof(T), 6.0 * a.items);
            return QVM_OK;
        }
        case OP_SWAPPAIR: {
            uint64_t fixed = op.cond_mask | op.hbit;
            uint64_t items = 1ull << (sv->n - popc(fixed));
            const int tok = prof_begin(sv);
            if constexpr (sizeof(R) == 8)
                hipLaunchKernelGGL(k_swappair_lanes, dim3(grid_for(2 * items)), dim3(kTPB), 0, sv->stream,
                                   (T*)sv->amps, items, fixed, op.cond_val, op.xmask);
            else
                hipLaunchKernelGGL((k_swappair<R>), dim3(grid_for(items)), dim3(kTPB), 0, sv->stream,
                                   (T*)sv->amps, items, fixed, op.cond_val, op.xmask);
            QVM_LAUNCH_CHECK(sv);
            prof_end(sv, tok, PK_SWAP, 4.0 * items * sizeof(T), 0.0);
            return QVM_OK;
        }
        case OP_DENSE:
            switch (op.k) {
                case 1: return launch_dense_k<R, 1>(sv, op);
                case 2: return launch_dense_k<R, 2>(sv, op);
                case 3: return launch_dense_k<R, 3>(sv, op);
                default: return fail(QVM_EUNSUPPORTED, "dense gate with k > 3 on the plain path");
            }
    }
    return fail(QVM_EARG, "bad op class");
}

qvm_status launch_op(qvm_sv* sv, const LOp& op) {
    return sv->dt == QVM_C64 ? launch_op_t<float>(sv, op) : launch_op_t<double>(sv, op);
}

qvm_status launch_init_basis(qvm_sv* sv, uint64_t idx) {
    uint64_t N = 1ull << sv->n;
    const int tok = prof_begin(sv);
    if (sv->dt == QVM_C64)
        hipLaunchKernelGGL((k_basis<float>), dim3(std::min<unsigned>(grid_for(N), 1u << 20)), dim3(kTPB), 0, sv->stream,
                           (float2*)sv->amps, N, idx);
    else
        hipLaunchKernelGGL((k_basis<double>), dim3(std::min<unsigned>(grid_for(N), 1u << 20)), dim3(kTPB), 0, sv->stream,
                           (double2*)sv->amps, N, idx);
    QVM_LAUNCH_CHECK(sv);
    prof_end(sv, tok, PK_BASIS, (double)N * (sv->dt == QVM_C64 ? 8 : 16), 0.0);
    return QVM_OK;
}

qvm_status launch_swap_bits(qvm_sv* sv, int a, int b) {
    if (a == b) return QVM_OK;
    LOp op{};
    op.cls = OP_SWAPPAIR;
    op.xmask = (1ull << a) | (1ull << b);
    // representative i: bit a = 0, bit b = 1; partner has them exchanged
    op.hbit = 1ull << a;
    op.cond_mask = 1ull << b;
    op.cond_val = 1ull << b;
    return launch_op(sv, op);
}

}  // namespace qvm
