// Tile kernel: one pass of a fused plan.
//
// Each workgroup owns one tile: the 2^L amplitudes that share the values of
// all non-tile physical bits.  The tile always contains the lowest c
// physical bits, so it is read and written as runs of 2^c contiguous
// amplitudes (128 bytes).  The tile is staged in LDS, the pass's ops run on
// it in order, and it is written back, optionally with its tile bits
// permuted (qubit-index remapping at no extra traffic).
//
// Ops:
//   TOP_BLOCK  a fused k-qubit block (k = 3..6): Y = M X over the tile's
//              2^(L-k) columns, as a real GEMM on MFMA 16x16x4 (FP32 for
//              complex64, FP64 for complex128).  The complex matrix M is
//              expanded to the real 2^(k+1) x 2^(k+1) matrix
//              [[Re, -Im], [Im, Re]] per entry, so interleaved (re, im)
//              amplitudes are used as they are stored.
//   TOP_DIAGRUN  a run of diagonal gates (CZ, CR, S, T, RZ, RZZ, controlled
//              phases), each as phase terms on bit patterns over tile bits
//              and the tile's fixed outer bits, applied with the tile
//              elements held in registers.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "internal.hpp"
#include "tile.hpp"

namespace qvm {

constexpr int NT = kTileThreads;      // threads per tile workgroup (8 waves)

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));

template <typename R> struct TT;
// Output layout of the 16x16x4 MFMA: register r of lane l holds column
// l % 16 and a row that differs between the FP32 and FP64 instructions
// (checked on gfx950): FP32 rows 4 (l / 16) + r, FP64 rows l / 16 + 4 r.
typedef float f32v4 __attribute__((ext_vector_type(4)));
typedef double f64v2 __attribute__((ext_vector_type(2)));
typedef float f32v2 __attribute__((ext_vector_type(2)));
template <> struct TT<float> {
    using V4 = f32x4;
    using V2 = f32v2;                 // one complex64 as (re, im)
    using V16 = f32v4;                // one 16-byte access: two complex64
    static constexpr int EP = 2;      // elements per 16-byte access
    static constexpr int C = 4;       // low bits per tile: 16 x 8 B = 128-byte runs
    static __host__ __device__ constexpr int out_row(int g, int r) { return 4 * g + r; }
};
template <> struct TT<double> {
    using V4 = f64x4;
    using V2 = f64v2;                 // one complex128 as (re, im)
    using V16 = f64v2;                // one 16-byte access: one complex128
    static constexpr int EP = 1;
    static constexpr int C = 3;       // low bits per tile: 8 x 16 B = 128-byte runs
    static __host__ __device__ constexpr int out_row(int g, int r) { return g + 4 * r; }
};

__device__ __forceinline__ f32x4 mfma16(float a, float b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f64x4 mfma16(double a, double b, f64x4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ uint32_t sw(uint32_t e) { return tile_swizzle(e); }

// Slot of element a + b for a < 2^m and b a multiple of 2^m (m >= 4): the
// swizzle only changes bits 0..3, so sw(a + b) = (sw(a) ^ low) + b with low
// = sw(b) ^ b below 16.  For a constant b the XOR takes an inline constant
// and the add folds into the LDS instruction's offset (no register holds
// the constant).
__device__ __forceinline__ uint32_t sw_add(uint32_t swa, uint32_t b) { return (swa ^ (sw(b) ^ b)) + b; }

// A 16-byte piece of two complex64 elements (2m, 2m + 1) as it sits in LDS:
// at the slot pair of sw(2m), swapped when that slot is odd (the swizzle
// keeps the pair adjacent but may reverse it).  Its own inverse.
template <int EP, typename V>
__device__ __forceinline__ V pair_order(V v, uint32_t s) {
    if constexpr (EP == 2) {
        const bool odd = (s & 1u) != 0;
        return odd ? V{v[2], v[3], v[0], v[1]} : v;
    } else {
        return v;
    }
}

// w with a zero inserted at every set bit of `fixed` (the tile bits), one
// run of consecutive set bits at a time: the tile's base index from its
// workgroup index.
__device__ __forceinline__ uint64_t dep64(uint64_t w, uint64_t fixed) {
    while (fixed) {
        const uint64_t low = fixed & (~fixed + 1);
        const uint64_t run = ((fixed + low) & ~fixed) - low;     // the lowest run of ones
        const uint64_t lo = w & (low - 1);
        w = ((w - lo) << __builtin_popcountll(run)) | lo;
        fixed &= ~run;
    }
    return w;
}

// ------------------------------------------------------------ phase angles
// Long runs: every term adds its angle (a fixed-point fraction of a turn,
// so sums wrap exactly modulo a full turn) to the elements it matches; each
// element then takes one factor exp(2 pi i acc / 2^bits), or, when every
// term is a factor of -1, one sign flip.  complex64 keeps 32-bit turns (each
// term's angle rounded to 2^-32 turns by the planner), complex128 64-bit.
template <typename R> struct Turn;
template <> struct Turn<float> { using T = uint32_t; };
template <> struct Turn<double> { using T = uint64_t; };

// (cos, sin) of 2 pi t / 2^32: the quadrant from the top two bits, the angle
// inside it folded to [0, pi/4] (sin and cos exchanged past pi/4), then the
// Taylor series of sin and cos at 0 (truncation below 2e-10 on [0, pi/4]).
__device__ __forceinline__ void cis_turns(uint32_t t, float& c, float& s) {
    const uint32_t q = t >> 30;
    uint32_t f = t & 0x3FFFFFFFu;
    const bool fold = f > 0x20000000u;
    f = fold ? 0x40000000u - f : f;
    const float x = (float)f * 1.4629180792671596e-9f;          // 2 pi / 2^32
    const float x2 = x * x;
    const float sn = x * (1.f + x2 * (-1.f / 6 + x2 * (1.f / 120 + x2 * (-1.f / 5040 + x2 * (1.f / 362880)))));
    const float cs = 1.f + x2 * (-0.5f + x2 * (1.f / 24 + x2 * (-1.f / 720 + x2 * (1.f / 40320 +
                                                                                  x2 * (-1.f / 3628800)))));
    const float a = fold ? sn : cs, b = fold ? cs : sn;
    c = q == 0 ? a : q == 1 ? -b : q == 2 ? -a : b;
    s = q == 0 ? b : q == 1 ? a : q == 2 ? -b : -a;
}

// The same for 2 pi t / 2^64 in double precision (truncation below 2e-19).
__device__ __forceinline__ void cis_turns(uint64_t t, double& c, double& s) {
    const uint32_t q = (uint32_t)(t >> 62);
    uint64_t f = t & ((1ull << 62) - 1);
    const bool fold = f > (1ull << 61);
    f = fold ? (1ull << 62) - f : f;
    const double x = (double)f * 3.4061215800865545e-19;         // 2 pi / 2^64
    const double x2 = x * x;
    const double sn =
        x * (1.0 + x2 * (-1.0 / 6 + x2 * (1.0 / 120 + x2 * (-1.0 / 5040 + x2 * (1.0 / 362880 +
        x2 * (-1.0 / 39916800 + x2 * (1.0 / 6227020800.0 + x2 * (-1.0 / 1307674368000.0 +
        x2 * (1.0 / 355687428096000.0)))))))));
    const double cs =
        1.0 + x2 * (-0.5 + x2 * (1.0 / 24 + x2 * (-1.0 / 720 + x2 * (1.0 / 40320 + x2 * (-1.0 / 3628800 +
        x2 * (1.0 / 479001600 + x2 * (-1.0 / 87178291200.0 + x2 * (1.0 / 20922789888000.0 +
        x2 * (-1.0 / 6402373705728000.0)))))))));
    const double a = fold ? sn : cs, b = fold ? cs : sn;
    c = q == 0 ? a : q == 1 ? -b : q == 2 ? -a : b;
    s = q == 0 ? b : q == 1 ? a : q == 2 ? -b : -a;
}

// x negated when the top bit of the accumulated angle a is set (a half
// turn): a sign-bit flip, the same result as a multiplication by -1.
__device__ __forceinline__ float flip_if(float x, uint32_t a) {
    return __uint_as_float(__float_as_uint(x) ^ (a & 0x80000000u));
}
__device__ __forceinline__ double flip_if(double x, uint64_t a) {
    return __longlong_as_double((long long)((unsigned long long)__double_as_longlong(x) ^ (a & 0x8000000000000000ull)));
}

// Each thread's total angle per element code: one sum per group of terms
// (per set of element bits they require), then subset sums over the element
// bits, so element code i collects every group S contained in i.
template <typename TU, int NHB>
__device__ __forceinline__ void run_angles(TU (&acc)[1 << NHB], const DTerm* __restrict__ terms,
                                           const uint32_t* __restrict__ grp, uint64_t base, uint32_t t) {
    constexpr int NE = 1 << NHB;
#pragma unroll
    for (int g = 0; g < NE; ++g) {
        TU a = 0;
        const uint32_t q1 = grp[g + 1];
#pragma unroll 1
        for (uint32_t q = grp[g]; q < q1; ++q) {
            // branch-free (every field always used), so the whole record
            // is fetched by one scalar load
            const DTerm& d = terms[q];
            const TU on = (TU)(((base & d.omask) == d.oval) & ((t & d.lmask) == d.lval));
            a += (TU)d.turns & ((TU)0 - on);
        }
        acc[g] = a;
    }
#pragma unroll
    for (int b = 0; b < NHB; ++b)
#pragma unroll
        for (int i = 0; i < NE; ++i)
            if ((i >> b) & 1) acc[i] += acc[i ^ (1 << b)];
}

// The tile kernel declares no static LDS, so its dynamic LDS (the tile
// first) starts at LDS address 0 and a tile byte offset is an LDS address:
// accesses through these take no base add.
template <typename T>
__device__ __forceinline__ T lds_ld(uint32_t off) {
    return *(const __attribute__((address_space(3))) T*)(size_t)off;
}
template <typename T>
__device__ __forceinline__ void lds_st(uint32_t off, T v) {
    *(__attribute__((address_space(3))) T*)(size_t)off = v;
}

// exp(2 pi i a / 2^32) from the LDS cis table (at byte address tab): the
// entry of the top kCisBits bits times cos + i sin of the rest, an angle
// d below 2 pi / kCisEntries (cos d = 1 - d^2 / 2 and sin d = d - d^3 / 6
// leave errors below d^4 / 24 < 6e-11).
__device__ __forceinline__ void cis_lds(uint32_t a, uint32_t tab, float& c, float& s) {
    typedef float f2 __attribute__((ext_vector_type(2)));
    const f2 t = lds_ld<f2>(tab + 8u * (a >> (32 - kCisBits)));
    const float d = (float)(a & ((1u << (32 - kCisBits)) - 1u)) * 1.4629180792671596e-9f;   // 2 pi / 2^32
    const float d2 = d * d;
    const float cd = 1.f - 0.5f * d2;
    const float sd = d - d * d2 * (1.f / 6);
    c = t.x * cd - t.y * sd;
    s = t.y * cd + t.x * sd;
}

// N uniform table words in one scalar load (dword alignment only).
template <int N>
__device__ __forceinline__ void sload(uint32_t (&dst)[N], const uint32_t* __restrict__ p) {
    if constexpr (N == 1) {
        dst[0] = p[0];
    } else {
        typedef uint32_t V __attribute__((ext_vector_type(N), aligned(4)));
        const V v = *(const V*)p;
#pragma unroll
        for (int i = 0; i < N; ++i) dst[i] = v[i];
    }
}

// Sign runs applied in a block's epilogue (ETerm records, complex64): whether a
// record matches thread t of tile w, as a vector test (tile-index test and
// thread test in one compare, no scalar compares); two records per scalar
// load (groups are padded to even counts).
__device__ __forceinline__ bool eterm_on(const uint32_t* r, uint32_t w, uint32_t t) {
    return (((w & r[0]) ^ r[1]) | ((t ^ r[3]) & r[2])) == 0;
}

// A sign run: bit i of the result is the parity of the thread's matching
// terms whose group is contained in element code i (each record holds the
// codes its group is contained in), i.e. whether element i changes sign.
__device__ __forceinline__ uint32_t erun_signs(const ETerm* __restrict__ terms, const uint32_t* __restrict__ grp,
                                               uint32_t w, uint32_t t) {
    const uint32_t n = grp[16];
    uint32_t m = 0;
#pragma unroll 1
    for (uint32_t q = 0; q < n; q += 2) {
        uint32_t r[16];
        sload<16>(r, (const uint32_t*)(terms + q));
        m ^= eterm_on(r, w, t) ? r[4] : 0u;
        m ^= eterm_on(r + 8, w, t) ? r[12] : 0u;
    }
    return m;
}

// A phase run from the pass's phase sums (layout in tile.hpp): per group,
// the sum of each combo (formed by the workgroup before its first op, in
// LDS at psum) where the thread meets the combo's thread condition (its
// wave's lane mask), four combos per step; then subset sums over the four
// element-code bits.
__device__ __forceinline__ void erun_psums(uint32_t (&acc)[16], const char* __restrict__ tab,
                                           const uint32_t* __restrict__ grp, int wave, uint32_t psum) {
    typedef uint32_t U4 __attribute__((ext_vector_type(4)));
    uint32_t hd[4];
    sload<4>(hd, (const uint32_t*)tab);
    const uint32_t* __restrict__ mk = (const uint32_t*)(tab + hd[3]) + 2 * (size_t)wave * hd[0];
    uint32_t go[17];                   // the group offsets in two scalar loads, one wait
    {
        uint32_t g16[16], g1[1];
        sload<16>(g16, grp);
        sload<1>(g1, grp + 16);
#pragma unroll
        for (int g = 0; g < 16; ++g) go[g] = g16[g];
        go[16] = g1[0];
    }
#pragma unroll
    for (int g = 0; g < 16; ++g) {
        uint32_t a = 0;
        const uint32_t c1 = go[g + 1];
#pragma unroll 1
        for (uint32_t c = go[g]; c < c1; c += 4) {
            uint32_t m[8];
            sload<8>(m, mk + 2 * c);
            const U4 v = lds_ld<U4>(psum + 4 * c);
#pragma unroll
            for (int j = 0; j < 4; ++j)
                a += __builtin_amdgcn_inverse_ballot_w64(m[2 * j] | (uint64_t)m[2 * j + 1] << 32) ? v[j] : 0u;
        }
        acc[g] = a;
    }
#pragma unroll
    for (int b = 0; b < 4; ++b)
#pragma unroll
        for (int i = 0; i < 16; ++i)
            if ((i >> b) & 1) acc[i] += acc[i ^ (1 << b)];
}

// ---------------------------------------------------------------- blocks
// The block's real fragments are already in LDS (after the tile; the
// kernel stages them while the previous op runs); every k-step reads one A
// value per row block from there.  The
// contraction index is ordered so that k-steps 2t and 2t+1 take the real
// and imaginary parts of complex input row 4t + l / 16: lane l reads that
// amplitude of its column (l % 16) once, as a (re, im) pair, and feeds the
// two halves to the two k-steps.  The 16x16 result leaves rows
// out_row(l / 16, r) of column l % 16 in register r of lane l.  Each wave
// owns whole columns, so the in-place update needs no barrier between its
// reads and writes.
//
// Addressing: the LDS swizzle is linear over GF(2) and the column bits,
// the lane's row bits and the k-step's row bits are disjoint, so every
// address is a per-column constant XOR a per-lane constant XOR a
// wave-uniform term.
constexpr int AREG_MAX = 32;       // widest real block (K = 2^(k+1)) whose fragments stay in registers

//
// With RUN (complex64, 13-qubit tiles, 3- and 4-qubit blocks: one column
// iteration per wave) the diagonal run that follows the block is applied to
// the outputs before they are stored: RUN = 1 a run of phases (one factor
// per element from its angle sum, from the pass's phase sums), RUN = 2 a
// run of sign flips (one parity bit per element).  The run's terms are
// encoded over the
// epilogue's layout: thread code threadIdx.x (lane l holds column bits 0..3
// as l % 16 and block bits 1, 2 as l / 16; the wave holds the top column
// bits) and element code hh | ct << 1 | rb << (1 + log2 CT) (block bit 0,
// the column tile, block bit 3).
//
// With GA (blocks of up to 4 qubits in passes without wider blocks) the A
// fragments come from the caller's registers (fetched from the plan one
// block ahead) instead of the LDS fragment area.
template <typename R, int K, int LT, int RUN = 0, bool GA = false, int NF = 1, bool PRE = false>
__device__ __forceinline__ void tile_block(R* __restrict__ lds, const R* __restrict__ ldsA, const R (&fa)[NF],
                                           uint64_t tab_off, const char* __restrict__ blob, int L_,
                                           const TOp* __restrict__ run = nullptr, int wave_ = -1,
                                           uint32_t cis_tab = 0, const uint32_t* pre = nullptr) {
    static_assert(RUN == 0 || (sizeof(R) == 4 && LT == 13 && (K == 16 || K == 32)),
                  "epilogue runs: complex64, 13-qubit tiles, k = 3, 4");
    constexpr int L = LT;                      // the kernel's tile width
    (void)L_;
    using V4 = typename TT<R>::V4;
    constexpr int RB = K / 16;                 // 16-row blocks of the real matrix
    constexpr int KS = K / 4;                  // k-steps of 4 real rows
    constexpr int k = K == 16 ? 3 : K == 32 ? 4 : K == 64 ? 5 : 6;
    // column tiles per wave iteration.  complex64: all of a wave's share of
    // a 13-qubit tile for 3-qubit blocks (one iteration, so no column tile's
    // loads wait behind another's stores), 4 for 4-qubit blocks; complex128
    // (twice the accumulator registers): 4 / RB; 1 for wider blocks
    // (at most the wave's share of the tile's column tiles, so that narrower
    // tiles keep every wave busy)
    constexpr int NW = NT / 64;
    constexpr int CT = block_ct(k, LT, sizeof(R) == 8);
    static_assert(!GA || RB * KS <= NF, "register fragments: the block's share fits the registers");
    // the wave index as a scalar, so the column table reads below are scalar loads
    const int lane = threadIdx.x & 63;
    const int wave = wave_ >= 0 ? wave_ : __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    constexpr int ncol = L >= k ? 1 << (L - k) : 1;
    constexpr int ntile = (ncol + 15) >> 4;
    // every wave takes whole column tiles of full columns: no bounds tests
    constexpr bool FULL = ncol >= 16 && ntile % (NW * CT) == 0;
    const int g = lane >> 4;
    // The slots are linear in the bits they are built from, so each address
    // is a per-lane part computed once here XOR a wave-uniform part from the
    // block's table (scalar loads, combined on the scalar unit: the
    // readfirstlane below only tells the compiler the value is uniform), as
    // byte offsets from the tile's start (LDS address 0): one XOR per access.
    constexpr uint32_t ES = 2 * sizeof(R);     // bytes per amplitude
    (void)lds;
    const BlockTabLayout lay(L, k);
    const uint32_t* __restrict__ tab = (const uint32_t*)(blob + tab_off);
    // one column iteration per wave: its column tiles' words are loaded with
    // the others, so the block waits for its table once
    constexpr bool ONE = FULL && ntile == NW * CT;
    static_assert(!PRE || ONE, "preloaded words: one column iteration per wave");
    constexpr int NBW = KS / 2, NEW = 4 * RB;
    uint32_t cw1[CT];
    uint32_t lanew[4], rbit[4], bw[NBW], ew[NEW];
    if constexpr (PRE) {
        // loaded by the caller with the op's record: the wave's column
        // words, then the k-step, output-row, lane and row-bit words
#pragma unroll
        for (int i = 0; i < CT; ++i) cw1[i] = pre[i];
#pragma unroll
        for (int i = 0; i < NBW; ++i) bw[i] = pre[CT + i];
#pragma unroll
        for (int i = 0; i < NEW; ++i) ew[i] = pre[CT + NBW + i];
#pragma unroll
        for (int i = 0; i < 4; ++i) lanew[i] = pre[CT + NBW + NEW + i];
#pragma unroll
        for (int i = 0; i < 4; ++i) rbit[i] = pre[CT + NBW + NEW + 4 + i];
    } else {
        if constexpr (ONE) sload<CT>(cw1, tab + lay.col() + wave * CT);
        // the block's uniform words that do not depend on the column tile,
        // each group in one scalar load
        sload<4>(lanew, tab + lay.lane());
        sload<4>(rbit, tab + lay.rbit());
        sload<NBW>(bw, tab + lay.brow());
        sload<NEW>(ew, tab + lay.erow());
    }
    // lane-bit masks (all ones where bit i of the lane index is set): each
    // conditional slot below is one AND-XOR of a mask and a table word
    auto lmask = [&](int i) { return 0u - (((uint32_t)lane >> i) & 1u); };
    // the lane's column inside a column tile: its four lane bits' slots
    uint32_t swl = 0;
#pragma unroll
    for (int i = 0; i < 4; ++i) swl ^= lanew[i] & lmask(i);
    // B operand: complex input row 4 t + g (g = lane bits 4, 5 on block
    // bits 0, 1); the lane's share is rows(g)
    uint32_t pin = swl ^ (rbit[0] & lmask(4)) ^ (rbit[1] & lmask(5));
    // epilogue: the lane's share of the output row index, rows(jlane):
    // complex64 jlane = 2 g (block bits 1, 2), complex128 jlane = g >> 1
    // (block bit 0; g & 1 picks the real or imaginary part)
    constexpr bool F32 = TT<R>::EP == 2;
    static_assert((TT<R>::out_row(1, 0) >> 1) == (F32 ? 2 : 0) && (TT<R>::out_row(2, 0) >> 1) == (F32 ? 4 : 1),
                  "output row layout");
    const int plane = TT<R>::out_row(g, 0) & 1;
    uint32_t pout = F32 ? swl ^ (rbit[1] & lmask(4)) ^ (rbit[2] & lmask(5)) : swl ^ (rbit[0] & lmask(5));
    // opaque copies: each access then takes one XOR of these with a scalar
    // (the compiler would otherwise re-split them into their parts)
    asm volatile("" : "+v"(pin));
    asm volatile("" : "+v"(pout));
    const R* __restrict__ Arow = ldsA + lane;
    // small blocks keep their A fragments in registers for the whole block
    // (the epilogue's LDS writes would otherwise force a re-read per column
    // tile: the compiler cannot tell the tile from the fragment area)
    constexpr int NA = K <= AREG_MAX ? RB * KS : 1;
    R afr[NA];
    if constexpr (K <= AREG_MAX) {
#pragma unroll
        for (int i = 0; i < NA; ++i) afr[i] = GA ? fa[i] : Arow[i * 64];
    }
    // one wave iteration over CT column tiles from t0 (no loop where there
    // is one iteration, so the table loads above are issued together)
    auto columns = [&](const int t0) {
        uint32_t cw[CT];                       // column tiles' slots (uniform)
        bool ok[CT];
#pragma unroll
        for (int ct = 0; ct < CT; ++ct) {
            const int c = (t0 + ct) * 16 + (lane & 15);
            if constexpr (FULL) {
                ok[ct] = true;
            } else {
                ok[ct] = (t0 + ct) < ntile && c < ncol;
                cw[ct] = tab[lay.col() + min(t0 + ct, ntile - 1)];
            }
        }
        if constexpr (ONE) {
#pragma unroll
            for (int ct = 0; ct < CT; ++ct) cw[ct] = cw1[ct];
        } else if constexpr (FULL) {
            sload<CT>(cw, tab + lay.col() + t0);
        }
        V4 acc[CT][RB];
#pragma unroll
        for (int ct = 0; ct < CT; ++ct)
#pragma unroll
            for (int rb = 0; rb < RB; ++rb) acc[ct][rb] = V4{0, 0, 0, 0};
        using V2 = typename TT<R>::V2;
#pragma unroll (K <= AREG_MAX ? KS / 2 : 2)
        for (int t = 0; t < KS / 2; ++t) {
            const uint32_t st = bw[t];
            V2 b[CT];
#pragma unroll
            for (int ct = 0; ct < CT; ++ct)
                b[ct] = ok[ct] ? lds_ld<V2>(pin ^ __builtin_amdgcn_readfirstlane(cw[ct] ^ st)) : V2{0, 0};
#pragma unroll
            for (int h = 0; h < 2; ++h) {
#pragma unroll
                for (int rb = 0; rb < RB; ++rb) {
                    const R av = K <= AREG_MAX ? afr[(rb * KS + 2 * t + h) % NA]
                                               : Arow[(rb * KS + 2 * t + h) * 64];
#pragma unroll
                    for (int ct = 0; ct < CT; ++ct) acc[ct][rb] = mfma16(av, b[ct][h], acc[ct][rb]);
                }
            }
        }
        using TU = typename Turn<R>::T;
        constexpr int NEC = RUN == 1 ? 16 : 1;
        constexpr int LCT = CT == 8 ? 3 : CT == 4 ? 2 : CT == 2 ? 1 : 0;
        TU ang[NEC];
        static_assert(RUN == 0 || 2 * CT * RB == 16, "epilogue element code");
        // the tile index: a vector operand where registers allow (the run's
        // tile-index tests then take no scalar instructions)
        uint32_t wv = blockIdx.x;
        if constexpr (RUN == 2 && GA && NF == 4) asm volatile("" : "+v"(wv));
        if constexpr (RUN == 1)
            erun_psums(ang, blob + run->data, (const uint32_t*)(blob + run->tab), wave,
                       cis_tab + 8u * kCisEntries);
        // a sign run: the thread's flips, one bit per element code
        uint32_t smask = 0;
        if constexpr (RUN == 2)
            smask = erun_signs((const ETerm*)(blob + run->data), (const uint32_t*)(blob + run->tab), wv, threadIdx.x);
#pragma unroll
        for (int ct = 0; ct < CT; ++ct) {
            if (!ok[ct]) continue;
#pragma unroll
            for (int rb = 0; rb < RB; ++rb) {
                if constexpr (TT<R>::EP == 2) {
                    // FP32: registers (0, 1) and (2, 3) are the (re, im) of
                    // complex rows 8 rb + 2 g and 8 rb + 2 g + 1
#pragma unroll
                    for (int hh = 0; hh < 2; ++hh) {
                        const uint32_t sl = pout ^ __builtin_amdgcn_readfirstlane(cw[ct] ^ ew[4 * rb + hh]);
                        R yr = acc[ct][rb][2 * hh], yi = acc[ct][rb][2 * hh + 1];
                        const int ec = hh | ct << 1 | rb << (1 + LCT);   // element code
                        if constexpr (RUN == 2) {
                            const uint32_t f = (smask << (31 - ec)) & 0x80000000u;
                            yr = __uint_as_float(__float_as_uint(yr) ^ f);
                            yi = __uint_as_float(__float_as_uint(yi) ^ f);
                        } else if constexpr (RUN == 1) {
                            R fr, fi;
                            cis_lds(ang[ec % NEC], cis_tab, fr, fi);
                            const R xr = yr;
                            yr = fr * xr - fi * yi;
                            yi = fr * yi + fi * xr;
                        }
                        lds_st<typename TT<R>::V2>(sl, typename TT<R>::V2{yr, yi});
                    }
                } else {
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const uint32_t sl = pout ^ __builtin_amdgcn_readfirstlane(cw[ct] ^ ew[4 * rb + r]);
                        lds_st<R>(sl | (uint32_t)plane * sizeof(R), acc[ct][rb][r]);
                    }
                }
            }
        }
    };
    if constexpr (ONE) {
        columns(wave * CT);
    } else {
        for (int t0 = wave * CT; t0 < ntile; t0 += NW * CT) columns(t0);
    }
}

// ----------------------------------------------------------- diagonal runs
// A run of consecutive diagonal gates, each lowered to phase terms "multiply
// by p where (index & mask) == val".  Thread t holds the tile elements
// t + NT i in registers.  The pattern test on the bits below log2(NT)
// depends only on t and becomes a per-lane factor chosen once per term; the
// test on the bits above depends only on i, so it is uniform across the
// wave and skips whole elements without divergence.
template <typename R, int L>
__device__ __forceinline__ void tile_diagrun(R* __restrict__ lds, const DSub* __restrict__ subs,
                                             int nsub, uint64_t base) {
    constexpr uint32_t nE = 1u << L;
    constexpr int NROW = nE >= NT ? (int)(nE / NT) : 1;   // elements per thread
    constexpr int NPT = NROW < 8 ? NROW : 8;               // elements per sweep
    constexpr uint32_t LOWM = NT - 1;
    const uint32_t t = threadIdx.x;
    const bool live = t < nE;
    const uint32_t swt = sw(t);          // slots are linear: sw(t + NT i) = sw(t) ^ sw(NT i)
#pragma unroll 1
    for (int i0 = 0; i0 < NROW; i0 += NPT) {
        R xr[NPT], xi[NPT];
        if (live) {
#pragma unroll
            for (int i = 0; i < NPT; ++i) {
                const uint32_t s = 2 * sw_add(swt, NT * (uint32_t)(i0 + i));
                xr[i] = lds[s];
                xi[i] = lds[s + 1];
            }
        }
#pragma unroll 1
        for (int q = 0; q < nsub; ++q) {
            const DSub& d = subs[q];
            if ((base & d.omask) != d.oval) continue;
            const bool hlo = (t & d.lmask & LOWM) == (d.lval & LOWM);
            const uint32_t rows = d.rows >> i0;     // bit i: element i of this sweep matches
            if (d.neg) {
                // factor -1 where the low bits match: a sign flip
                const R sg = hlo ? (R)-1 : (R)1;
#pragma unroll
                for (int i = 0; i < NPT; ++i) {
                    if ((rows >> i) & 1) {
                        xr[i] *= sg;
                        xi[i] *= sg;
                    }
                }
                continue;
            }
            // per-lane factor: the term's phase where the low bits match, else 1
            const R fr = hlo ? (R)d.pr : (R)1;
            const R fi = hlo ? (R)d.pi : (R)0;
#pragma unroll
            for (int i = 0; i < NPT; ++i) {
                if ((rows >> i) & 1) {
                    const R a = xr[i], b = xi[i];
                    xr[i] = fr * a - fi * b;
                    xi[i] = fr * b + fi * a;
                }
            }
        }
        if (live) {
#pragma unroll
            for (int i = 0; i < NPT; ++i) {
                const uint32_t s = 2 * sw_add(swt, NT * (uint32_t)(i0 + i));
                lds[s] = xr[i];
                lds[s + 1] = xi[i];
            }
        }
    }
}

template <typename R, int L>
__device__ __forceinline__ void tile_diagrun_turns(R* __restrict__ lds, const DTerm* __restrict__ terms,
                                                   const uint32_t* __restrict__ grp, uint64_t base,
                                                   bool signs) {
    using TU = typename Turn<R>::T;
    constexpr uint32_t nE = 1u << L;
    constexpr int NHB = L > kLogTileThreads ? L - kLogTileThreads : 0;   // element bits
    constexpr int NE = 1 << NHB;                                          // elements per thread
    const uint32_t t = threadIdx.x;
    TU acc[NE];
    run_angles<TU, NHB>(acc, terms, grp, base, t);
    if (t >= nE) return;
    const uint32_t swt = sw(t);
#pragma unroll
    for (int i = 0; i < NE; ++i) {
        const uint32_t e = 2 * sw_add(swt, NT * (uint32_t)i);
        const R xr = lds[e], xi = lds[e + 1];
        if (signs) {
            // the accumulated angle is 0 or a half turn
            lds[e] = flip_if(xr, acc[i]);
            lds[e + 1] = flip_if(xi, acc[i]);
        } else {
            R fr, fi;
            cis_turns(acc[i], fr, fi);
            lds[e] = fr * xr - fi * xi;
            lds[e + 1] = fr * xi + fi * xr;
        }
    }
}

// Orders a wave's LDS accesses before and after it: a wave's LDS operations
// execute in issue order, so it is enough that the compiler moves no memory
// access across (no wait for the writes before it is needed); used between
// two blocks in which every wave touches the same tile elements.
__device__ __forceinline__ void wave_lds_order() {
    asm volatile("" ::: "memory");
    __builtin_amdgcn_wave_barrier();
}

// A block's real A fragments for GA blocks: lane l's share, fragment (rb, s)
// at index rb KS + s, read from the plan.  Every block of a pass is fetched
// with the same count NF (4 when all its blocks have 3 qubits, else 16: the
// planner pads 3-qubit fragments of such passes to 16), so the loads in
// flight are known at every point and waiting for one block's fragments
// never waits for the next block's.
template <typename R, int NF>
__device__ __forceinline__ void fetch_frag(R (&dst)[NF], uint64_t data, const char* __restrict__ blob) {
    const R* __restrict__ f = (const R*)(blob + data) + (threadIdx.x & 63);
#pragma unroll
    for (int i = 0; i < NF; ++i) dst[i] = f[64 * i];
}

// The ops of a pass whose blocks all have 3 or 4 qubits: fragments in
// registers (fetched one block ahead), a workgroup barrier between ops
// except before blocks marked BLK_NOSYNC.
template <typename R, int L, int NF>
__device__ __forceinline__ void tile_ops_regfrag(R* __restrict__ lds, const TOp* __restrict__ ops, const PassDesc& pd,
                                                 const char* __restrict__ blob, uint64_t base, R (&fa)[NF],
                                                 uint32_t cis_tab) {
    R fb[NF];
    bool first = true;           // the barrier after the load phase covers the first op
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    // 3-qubit block layout: column tiles, per-wave share (one iteration)
    constexpr int CT3 = block_ct(3, L, sizeof(R) == 8);
    constexpr int NTILE3 = L > 3 ? ((1 << (L - 3)) + 15) >> 4 : 1;
    constexpr bool PRE3 = NF == 4 && L > 7 && NTILE3 == (NT / 64) * CT3 && (1 << (L - 3)) % 16 == 0;
    static_assert(!PRE3 || 2 + 4 + 8 == 14, "3-qubit table words after the column words");
    for (int oi = 0; oi < pd.nops; ++oi) {
        // the whole op record in one scalar load (one wait per op); in
        // passes of 3-qubit blocks with one column iteration per wave, the
        // op's table words too (they sit at a fixed stride by op index)
        uint32_t r[16];
        sload<16>(r, (const uint32_t*)(ops + oi));
        uint32_t pw[PRE3 ? CT3 + 14 : 1];
        if constexpr (PRE3) {
            const uint32_t* __restrict__ tp = (const uint32_t*)(blob + pd.tabs) + oi * kTabWords;
            uint32_t pc[CT3], ps[14];
            sload<CT3>(pc, tp + wave * CT3);
            sload<14>(ps, tp + NTILE3);
#pragma unroll
            for (int i = 0; i < CT3; ++i) pw[i] = pc[i];
#pragma unroll
            for (int i = 0; i < 14; ++i) pw[CT3 + i] = ps[i];
        }
        const int32_t type = (int32_t)r[0], k = (int32_t)r[1], flags = (int32_t)r[11];
        const uint64_t data = r[8] | (uint64_t)r[9] << 32, tab = r[12] | (uint64_t)r[13] << 32;
        const uint64_t next_data = r[14] | (uint64_t)r[15] << 32;
        const bool has_next = (int32_t)r[10] >= 0;
        if (type != TOP_BLOCK && (flags & DRUN_EPILOGUE)) continue;   // applied by the block before it
        if (!first) {
            if (type == TOP_BLOCK && (flags & BLK_NOSYNC)) wave_lds_order();
            else __syncthreads();
        }
        first = false;
        if (type == TOP_BLOCK) {
            if (has_next) fetch_frag<R, NF>(fb, next_data, blob);
            // a diagonal run right after the block may ride in its epilogue
            constexpr bool RUNOK = sizeof(R) == 4 && L == 13;
            constexpr int RP = RUNOK ? 1 : 0, RS = RUNOK ? 2 : 0;
            const int erun = !RUNOK || !(flags & BLK_RUN) ? 0 : (flags & BLK_RUN_SIGNS) ? 2 : 1;
            const TOp* run = &ops[oi + 1];
            if (NF == 4 || k == 3) {
                if (erun == 2) tile_block<R, 16, L, RS, true, NF, PRE3>(lds, lds, fa, tab, blob, L, run, wave, 0, pw);
                else if (erun == 1)
                    tile_block<R, 16, L, RP, true, NF, PRE3>(lds, lds, fa, tab, blob, L, run, wave, cis_tab, pw);
                else tile_block<R, 16, L, 0, true, NF, PRE3>(lds, lds, fa, tab, blob, L, nullptr, wave, 0, pw);
            } else if constexpr (NF >= 16) {
                if (erun == 2) tile_block<R, 32, L, RS, true>(lds, lds, fa, tab, blob, L, run, wave);
                else if (erun == 1) tile_block<R, 32, L, RP, true>(lds, lds, fa, tab, blob, L, run, wave, cis_tab);
                else tile_block<R, 32, L, 0, true>(lds, lds, fa, tab, blob, L, nullptr, wave);
            }
            if (has_next) {
#pragma unroll
                for (int i = 0; i < NF; ++i) fa[i] = fb[i];
            }
        } else if (flags & DRUN_TURNS) {
            tile_diagrun_turns<R, L>(lds, (const DTerm*)(blob + data), (const uint32_t*)(blob + tab), base,
                                     (flags & DRUN_SIGNS) != 0);
        } else {
            tile_diagrun<R, L>(lds, (const DSub*)(blob + data), k, base);
        }
    }
    __syncthreads();
}

// ---------------------------------------------------------------- kernel
// The tile is read and written once per pass with nontemporal accesses (the
// state streams through; caching it in L2 gains nothing).
//
// Stream phases: thread t moves the 16-byte pieces t + NT i (i < NIT) of the
// tile, tile element e = EP (t + NT i).  Its chunk of 2^C elements is
// e >> C = (EP t >> C) + (EP NT >> C) i and its offset in the chunk EP t mod
// 2^C (EP NT is a multiple of 2^C); the chunk-offset and remap tables are
// linear over disjoint bits (deposits and bit permutations), so a piece's
// entry is the thread's entry OR the uniform entry of i: one per-thread
// table load per phase, the rest scalar loads.
//
// Passes whose blocks are all of 3 or 4 qubits keep every block's A
// fragments in registers (the first block's fetched before the load phase,
// each later block's one block ahead) and need no LDS fragment area; a
// workgroup barrier separates consecutive ops except blocks marked
// BLK_NOSYNC, whose waves touch the same elements as in the block before.
// Passes with wider blocks stage each block's fragments in LDS, with a
// barrier after every op.
template <typename R, int L, int MODE>   // MODE: 4 or 16 fragment registers, 0 LDS fragments
__device__ __forceinline__ void tile_pass(R* __restrict__ psi, const PassDesc& pd, const char* __restrict__ blob) {
    extern __shared__ __align__(16) char smem[];
    // LDS: the tile first (at address 0, so tile addresses need no base),
    // in passes with wider blocks the widest block's fragments after it
    R* lds = (R*)smem;
    R* ldsA = lds + (2u << L);
    constexpr int EP = TT<R>::EP;
    constexpr int C = TT<R>::C < L ? TT<R>::C : L;          // low bits in every tile
    constexpr uint32_t NP = (1u << L) / EP;                  // 16-byte pieces per tile
    constexpr int NIT = NP >= NT ? (int)(NP / NT) : 1;       // pieces per thread
    constexpr int BATCH = NIT < 4 ? NIT : 4;
    constexpr uint32_t CM = (1u << C) - 1;
    constexpr uint32_t HI = (uint32_t)EP * NT >> C;          // chunk step of piece i
    static_assert(((uint32_t)EP * NT & CM) == 0, "pieces i > 0 start on chunk boundaries");
    using V16 = typename TT<R>::V16;
    const uint64_t* __restrict__ ldoff = (const uint64_t*)(blob + pd.ldoff);
    const uint32_t* __restrict__ rmhi = (const uint32_t*)(blob + pd.rmhi);
    const uint32_t* __restrict__ rmlo = (const uint32_t*)(blob + pd.rmlo);
    const TOp* __restrict__ ops = (const TOp*)(blob + pd.ops);
    const bool live = threadIdx.x < NP;
    const bool remap = pd.remap != 0;
    const uint32_t e0 = EP * threadIdx.x;
    // the thread's table entries first (the tile loads wait for them only):
    // its chunk offset and, in complex64 passes with few fragment registers,
    // its remap entries for the store phase
    constexpr bool PRE_RM = MODE == 4 && EP == 2;
    uint64_t tofs = 0;
    uint32_t rh0 = 0, rl0 = 0, rl1 = 0;
    if (live) {
        tofs = ldoff[e0 >> C] + (e0 & CM);
        if (PRE_RM && remap) {
            rh0 = rmhi[e0 >> C];
            rl0 = rmlo[e0 & CM];
            rl1 = EP == 2 ? rmlo[(e0 + 1) & CM] : 0u;
        }
    }
    R fa[MODE > 0 ? MODE : 1];
    if constexpr (MODE > 0)
        if (pd.first_block >= 0) fetch_frag<R, MODE>(fa, ops[pd.first_block].data, blob);
    const uint64_t base = dep64((uint64_t)blockIdx.x, pd.qmask);
    // the thread's piece offsets: its table entry plus the uniform one of i
    tofs += base;

    // the cis table of phase runs in block epilogues, in LDS after the
    // tile (and after the fragment area of passes with wider blocks)
    const uint32_t cis_tab = (uint32_t)((2u << L) * sizeof(R)) +
                             (MODE == 0 && pd.kmax >= 5 ? (uint32_t)((2u << pd.kmax) * (2u << pd.kmax) * sizeof(R)) : 0u);
    if constexpr (sizeof(R) == 4 && L == 13) {
        if (pd.cistab) {
            typedef float f4 __attribute__((ext_vector_type(4)));
            static_assert(kCisEntries == 2 * NT, "one 16-byte piece of the table per thread");
            const f4 v = *(const f4*)(blob + pd.cistab + 16 * threadIdx.x);
            lds_st<f4>(cis_tab + 16 * threadIdx.x, v);
        }
    }
    // the phase sums of the pass's epilogue phase runs (after the cis
    // table): the combos split over the waves, each summed on the scalar
    // unit while the first batch of the tile's loads is in flight; the
    // barrier after the load phase publishes them
    auto phase_sums = [&]() {
        if constexpr (sizeof(R) == 4 && L == 13) {
            if (pd.psum) {
                const uint32_t* __restrict__ tp = (const uint32_t*)(blob + pd.psum);
                uint32_t hd[4];
                sload<4>(hd, tp);
                const uint32_t* __restrict__ rec = tp + hd[2] / 4;
                const uint32_t w = blockIdx.x;
                const uint32_t psum = cis_tab + 8u * kCisEntries;
#pragma unroll 1
                for (uint32_t c = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6); c < hd[0]; c += NT / 64) {
                    uint32_t cr[2];
                    sload<2>(cr, tp + 4 + c);
                    uint32_t sum = 0;
#pragma unroll 1
                    for (uint32_t r = cr[0]; r < cr[1]; ++r) {
                        uint32_t q[4];
                        sload<4>(q, rec + 4 * r);
                        sum += (w & q[0]) == q[1] ? q[2] : 0u;
                    }
                    if ((threadIdx.x & 63) == 0) lds_st<uint32_t>(psum + 4 * c, sum);
                }
            }
        }
    };
    // load: per batch, all loads in flight, then LDS.  The slot of piece i
    // is the thread's slot XOR a constant (the swizzle is linear and the
    // thread's bits and i's are disjoint).
    const uint32_t se0 = sw(e0);
    if (live) {
#pragma unroll
        for (int b0 = 0; b0 < NIT; b0 += BATCH) {
            V16 v[BATCH];
#pragma unroll
            for (int it = 0; it < BATCH; ++it)
                v[it] = __builtin_nontemporal_load((const V16*)(psi + 2 * (tofs + ldoff[HI * (b0 + it)])));
            if (b0 == 0) phase_sums();
#pragma unroll
            for (int it = 0; it < BATCH; ++it) {
                const uint32_t s = sw_add(se0, (uint32_t)EP * NT * (uint32_t)(b0 + it));
                *(V16*)(lds + 2 * (s & ~(uint32_t)(EP - 1))) = pair_order<EP>(v[it], s);
            }
        }
    }
    __syncthreads();

    if constexpr (MODE > 0) {
        tile_ops_regfrag<R, L, MODE>(lds, ops, pd, blob, base, fa, cis_tab);
    } else {
    // fragments: the first block's are copied to LDS with the tile (the
    // barrier below covers them); each later block's are read into
    // registers while the block before it runs and stored to LDS after it.
    if (pd.first_block >= 0) {
        const TOp& fb = ops[pd.first_block];
        const R* __restrict__ frag = (const R*)(blob + fb.data);
        const int kk = 4 << (2 * fb.k);                       // (2^(k+1))^2 reals
        for (int i = threadIdx.x; i < kk; i += NT) ldsA[i] = frag[i];
    }
    __syncthreads();
    for (int oi = 0; oi < pd.nops; ++oi) {
        const TOp& op = ops[oi];
        if (op.type == TOP_BLOCK) {
            constexpr int PF = 8;                             // prefetch registers per thread
            R pre[PF];
            const int nb = op.next_block;
            const R* __restrict__ nfrag = nullptr;
            int nkk = 0;
            if (nb >= 0) {
                nfrag = (const R*)(blob + ops[nb].data);
                nkk = 4 << (2 * ops[nb].k);
                if (nkk <= PF * NT) {
#pragma unroll
                    for (int j = 0; j < PF; ++j) {
                        const int i = threadIdx.x + j * NT;
                        if (i < nkk) pre[j] = nfrag[i];
                    }
                }
            }
            // (the planner puts no run in the epilogue of a block in these passes)
            switch (op.k) {
                case 3: tile_block<R, 16, L>(lds, ldsA, fa, op.tab, blob, L); break;
                case 4: tile_block<R, 32, L>(lds, ldsA, fa, op.tab, blob, L); break;
                case 5: tile_block<R, 64, L>(lds, ldsA, fa, op.tab, blob, L); break;
                case 6: tile_block<R, 128, L>(lds, ldsA, fa, op.tab, blob, L); break;
                default: break;
            }
            __syncthreads();
            if (nb >= 0) {
                if (nkk <= PF * NT) {
#pragma unroll
                    for (int j = 0; j < PF; ++j) {
                        const int i = threadIdx.x + j * NT;
                        if (i < nkk) ldsA[i] = pre[j];
                    }
                } else {
                    for (int i = threadIdx.x; i < nkk; i += NT) ldsA[i] = nfrag[i];
                }
                __syncthreads();
            }
        } else {
            if (op.flags & DRUN_EPILOGUE) continue;          // applied by the block before it
            if (op.flags & DRUN_TURNS)
                tile_diagrun_turns<R, L>(lds, (const DTerm*)(blob + op.data),
                                         (const uint32_t*)(blob + op.tab), base,
                                         (op.flags & DRUN_SIGNS) != 0);
            else
                tile_diagrun<R, L>(lds, (const DSub*)(blob + op.data), op.k, base);
            __syncthreads();
        }
    }
    }

    // store: per batch, LDS reads first (optionally through the tile-bit
    // remap), then the global stores.  Passes with more fragment registers
    // read the thread's chunk offset again rather than keep it through the
    // ops (the opaque copy of the thread index stops the reuse).
    if constexpr (MODE != 4) {
        uint32_t tid = threadIdx.x;
        asm volatile("" : "+v"(tid));
        if (live) tofs = base + ldoff[(EP * tid) >> C] + ((EP * tid) & CM);
    }
    // the thread's first slot, formed again (not kept through the ops)
    uint32_t e0s = e0;
    asm volatile("" : "+v"(e0s));
    const uint32_t ss0 = sw(e0s);
    if (live) {
        if (!PRE_RM && remap) {                 // the thread's remap entries
            rh0 = rmhi[e0 >> C];
            rl0 = rmlo[e0 & CM];
            rl1 = EP == 2 ? rmlo[(e0 + 1) & CM] : 0u;
        }
#pragma unroll
        for (int b0 = 0; b0 < NIT; b0 += BATCH) {
            V16 v[BATCH];
            if (!remap) {
#pragma unroll
                for (int it = 0; it < BATCH; ++it) {
                    const uint32_t s = sw_add(ss0, (uint32_t)EP * NT * (uint32_t)(b0 + it));
                    v[it] = pair_order<EP>(*(const V16*)(lds + 2 * (s & ~(uint32_t)(EP - 1))), s);
                }
            } else {
#pragma unroll
                for (int it = 0; it < BATCH; ++it) {
                    // the tables hold slots: disjoint bits, so their XOR is the slot
                    const uint32_t hi = rh0 ^ rmhi[HI * (b0 + it)];
                    const uint32_t s0 = 2 * (hi ^ rl0);
                    if constexpr (EP == 2) {
                        const uint32_t s1 = 2 * (hi ^ rl1);
                        v[it] = V16{lds[s0], lds[s0 + 1], lds[s1], lds[s1 + 1]};
                    } else {
                        v[it] = V16{lds[s0], lds[s0 + 1]};
                    }
                }
            }
#pragma unroll
            for (int it = 0; it < BATCH; ++it)
                __builtin_nontemporal_store(v[it], (V16*)(psi + 2 * (tofs + ldoff[HI * (b0 + it)])));
        }
    }
}

// One kernel per fragment mode, so that each gets its own register budget:
// four waves per SIMD (two workgroups per CU) where the tile leaves room
// for two workgroups in LDS and the registers allow it.
template <typename R, int L, int MODE>
__global__ __launch_bounds__(NT, (sizeof(R) == 4 || (MODE == 4 && L <= 12)) ? 4 : 2) void k_tile(R* __restrict__ psi, PassDesc pd,
                                                 const char* __restrict__ blob) {
    tile_pass<R, L, MODE>(psi, pd, blob);
}

size_t tile_lds_bytes(qvm_dtype dt, int L, int kmax_block, bool cis, int npsum) {
    const size_t es = dt == QVM_C64 ? 4 : 8;          // bytes per real
    // blocks of up to 4 qubits keep their fragments in registers
    const size_t K = kmax_block >= 5 ? (size_t)2 << kmax_block : 0;
    return ((size_t)2 << L) * es + K * K * es +
           (cis ? (size_t)kCisEntries * 2 * sizeof(float) + (size_t)4 * npsum : 0);
}

template <typename R>
static qvm_status launch_tile_t(qvm_sv* sv, const PassDesc& pd, const char* blob_dev, size_t lds,
                                double flops) {
    static bool attr_set[64][16][3] = {};    // per device, tile size and fragment mode
    int dev = 0;
    QVM_HIP(sv, hipGetDevice(&dev));
    if (dev < 0 || dev >= 64) return fail(QVM_EUNSUPPORTED, "device index above 63");
    const unsigned grid = 1u << (sv->n - pd.L);
    const int mode = pd.kmax <= 3 ? 0 : pd.kmax == 4 ? 1 : 2;
    const void* fn = nullptr;
    switch (pd.L) {
#define QVM_TILE_CASE(LL)                                                          \
        case LL:                                                                   \
            fn = mode == 0 ? (const void*)k_tile<R, LL, 4>                         \
               : mode == 1 ? (const void*)k_tile<R, LL, 16> : (const void*)k_tile<R, LL, 0>; \
            break;
        QVM_TILE_CASE(3) QVM_TILE_CASE(4) QVM_TILE_CASE(5) QVM_TILE_CASE(6) QVM_TILE_CASE(7)
        QVM_TILE_CASE(8) QVM_TILE_CASE(9) QVM_TILE_CASE(10) QVM_TILE_CASE(11) QVM_TILE_CASE(12)
        QVM_TILE_CASE(13)
#undef QVM_TILE_CASE
        default: return fail(QVM_EUNSUPPORTED, "tile size outside 3..13");
    }
    if (pd.c != (TT<R>::C < pd.L ? TT<R>::C : pd.L)) return fail(QVM_EARG, "internal: pass low-bit count");
    if (!attr_set[dev][pd.L][mode]) {
        QVM_HIP(sv, hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)kTileLdsMax));
        attr_set[dev][pd.L][mode] = true;
    }
    R* amps = (R*)sv->amps;
    void* args[] = {(void*)&amps, (void*)&pd, (void*)&blob_dev};
    const int tok = prof_begin(sv);
    QVM_HIP(sv, hipLaunchKernel(fn, dim3(grid), dim3(NT), args, lds, sv->stream));
    prof_end(sv, tok, PK_TILE, 2.0 * (double)(1ull << sv->n) * 2 * sizeof(R), flops);
    return QVM_OK;
}

qvm_status launch_tile_pass(qvm_sv* sv, const PassDesc& pd, const char* blob_dev, double flops) {
    if (pd.cistab && (sv->dt != QVM_C64 || pd.L != 13)) return fail(QVM_EARG, "internal: cis table outside complex64 13-qubit passes");
    if ((pd.psum != 0) != (pd.npsum > 0) || pd.npsum % 4 || pd.npsum > kPSumMax || (pd.psum && !pd.cistab))
        return fail(QVM_EARG, "internal: phase sums of a pass");
    const size_t lds = tile_lds_bytes(sv->dt, pd.L, pd.kmax, pd.cistab != 0, pd.npsum);
    if (lds > kTileLdsMax) return fail(QVM_EUNSUPPORTED, "pass needs more LDS than a workgroup has");
    return sv->dt == QVM_C64 ? launch_tile_t<float>(sv, pd, blob_dev, lds, flops)
                             : launch_tile_t<double>(sv, pd, blob_dev, lds, flops);
}

}  // namespace qvm
