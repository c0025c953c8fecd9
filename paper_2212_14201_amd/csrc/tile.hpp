// Device-visible plan records shared by the planner (host) and the tile
// kernel.  A plan is a list of passes; a pass streams every tile of 2^L
// amplitudes through LDS once and applies a list of ops to it.
#pragma once

#include <cstdint>

#include <hip/hip_runtime.h>

namespace qvm {

constexpr int kTileThreads = 512;    // threads per tile workgroup (8 waves)
constexpr int kLogTileThreads = 9;
static_assert(1 << kLogTileThreads == kTileThreads, "kLogTileThreads");

enum TileOpType : int32_t { TOP_BLOCK = 1, TOP_DIAGRUN = 2 };

constexpr size_t kTileLdsMax = 160 * 1024;   // LDS per workgroup on gfx950

// Diagonal-run flags (TOp::flags).
enum : int32_t {
    DRUN_TURNS = 1,         // accumulate each element's phase in turns, one factor per element
    DRUN_SIGNS = 2,         // every term is a factor of -1 (with DRUN_TURNS: a sign flip per element)
    DRUN_EPILOGUE = 4       // applied by the preceding block's epilogue (its element layout)
};
// Block flags (TOp::flags of a TOP_BLOCK).
enum : int32_t {
    BLK_RUN = 1,            // the next op is a DRUN_EPILOGUE run this block applies to its outputs
    BLK_NOSYNC = 2,         // each wave touches exactly the tile elements it touched in the
                            // block before (same wave bits): no workgroup barrier between them
    BLK_RUN_SIGNS = 4       // with BLK_RUN: the run is a sign run (DRUN_SIGNS)
};

struct TOp {
    int32_t type;
    int32_t k;              // block: matrix width in qubits; diagonal run: number of terms
    int32_t lb[6];          // block: local tile bit of block bit r
    uint64_t data;          // byte offset into the plan blob: fragments or DSub[k]
    int32_t next_block;     // index of the pass's next TOP_BLOCK op, -1 if none
    int32_t flags;          // diagonal run: DRUN_* bits
    uint64_t tab;           // block: byte offset of its address table (BlockTab layout);
                            // angle-path diagonal run: byte offset of its group offsets
    uint64_t next_data;     // data of the pass's next TOP_BLOCK op (its fragments), 0 if none
};
static_assert(sizeof(TOp) == 64, "TOp is read as one 64-byte scalar load");

// LDS slot of tile element e: the four low bits are XOR-ed with a fixed
// image of every bit above them (bits 4..12 contribute 3, 5, 6, 9, 10, 12,
// 7, 11, 13: distinct vectors of weight two or three), so that for every
// block the planner can choose four column bits whose slots differ in the
// low bits that select the LDS bank (a 16-lane column walk then hits
// distinct banks).  The map is linear over GF(2) (slot(a ^ b) = slot(a) ^
// slot(b)) and an involution (the bits above 3 are unchanged); elements 2m
// and 2m + 1 keep adjacent slots, in either order (slot bit 0).
__host__ __device__ constexpr uint32_t tile_swizzle(uint32_t e) {
    constexpr uint32_t img[9] = {3, 5, 6, 9, 10, 12, 7, 11, 13};
    uint32_t x = 0;
    for (int j = 0; j < 9; ++j) x ^= ((e >> (4 + j)) & 1u) ? img[j] : 0u;
    return e ^ x;
}

// Address table of a block op (uint32 words, byte offsets into the tile:
// LDS slot times the bytes of one complex amplitude; the tile sits at the
// start of LDS): the wave-uniform parts of the block's LDS addresses, so
// that the kernel forms each address with one XOR per access (byte offsets
// of slots are linear over GF(2) as well).  The block's columns are the
// tile bits outside the block; the planner assigns them roles: four lane
// bits (a lane's column l % 16), then the bits of the column-tile index ti.
//   col[ti], ti < ntile = ceil(2^(L-k) / 16): slot of the column tile's
//            base (its ti bits placed on their tile bits)
//   brow[t], t < K/8:  slot(rows(4 t)), the input rows of k-step pair t
//   erow[4 rb + r], rb < K/16, r < 4: slot of the output rows a lane's
//            register r of row block rb holds, without the lane's own share
//   lane[i], i < 4: slot of lane bit i's tile bit (0 where the block has
//            fewer than four column bits)
//   rbit[r], r < 4: slot of block bit r's tile bit (0 for r >= k)
// rows(j) places block row index j on the block's tile bits lb[].  Wave w
// takes the column tiles ti = ct + CT (w + 8 j) (ct < CT, j = 0, 1, ...),
// so the three ti bits above the CT bits are the wave's: when two blocks
// put the same tile bits there, each wave touches the same elements in both.
struct BlockTabLayout {
    int ntile, nb, ne;
    __host__ __device__ BlockTabLayout(int L, int k) {
        const int ncol = 1 << (L - k);
        ntile = (ncol + 15) >> 4;
        nb = (2 << k) / 8;
        ne = 4 * ((2 << k) / 16);
    }
    __host__ __device__ int col() const { return 0; }
    __host__ __device__ int brow() const { return ntile; }
    __host__ __device__ int erow() const { return ntile + nb; }
    __host__ __device__ int lane() const { return ntile + nb + ne; }
    __host__ __device__ int rbit() const { return ntile + nb + ne + 4; }
    __host__ __device__ int words() const { return ntile + nb + ne + 8; }
};

// The address tables of a pass's block ops sit at a fixed stride by op
// index (a table has at most 80 words: 13-qubit tiles, 3-qubit blocks), so
// the kernel can load an op's table together with its record.
constexpr int kTabWords = 80;
constexpr size_t kTabStride = kTabWords * sizeof(uint32_t);

// Column tiles a wave takes per iteration in the block kernel (K = 2^(k+1)
// real rows): complex64 8 for k = 3, 4 for k = 4; complex128 4 / (K / 16);
// 1 for k >= 5; at most the wave's share of the tile's column tiles.
__host__ __device__ constexpr int block_ct(int k, int L, bool c128) {
    const int K = 2 << k, RB = K / 16;
    const int ct0 = RB >= 4 ? 1 : c128 ? 4 / RB : (K == 16 ? 8 : 4);
    const int lk = L > k ? L - k : 0;
    const int ntile = ((1 << lk) + 15) >> 4;
    const int share = ntile / (kTileThreads / 64);
    return ct0 < share ? ct0 : share >= 1 ? share : 1;
}

// One phase term of a diagonal run: amplitudes whose local tile bits match
// (lmask, lval) and whose tile's outer bits match (omask, oval) are
// multiplied by the unit-modulus factor (pr + i pi) = exp(2 pi i turns / 2^64);
// neg marks a factor of exactly -1.  Thread t of the tile workgroup holds
// elements t + kTileThreads i; bit i of rows is set when the bits of
// kTileThreads i match the term's condition on the local bits above the
// thread bits (the part of the test that is uniform across the workgroup).
struct DSub {
    uint32_t lmask, lval;
    int32_t neg;
    uint32_t rows;
    uint64_t omask, oval;
    double pr, pi;
    uint64_t turns;         // the factor's angle as a 64-bit fraction of a full turn
    uint64_t pad2_;         // 64 bytes: read as four 16-byte words
};
static_assert(sizeof(DSub) == 64, "DSub is read as four 16-byte words");

// One term of a diagonal run on the angle path (DRUN_TURNS).  Thread t holds
// elements t + kTileThreads i, i < 2^h (h = L - kLogTileThreads element
// bits).  A term adds `turns` (the kernel's fixed-point width: the low 32
// bits for complex64, all 64 for complex128) to element (t, i) when the
// tile's outer bits match (omask, oval), t matches (lmask, lval) on the
// thread bits, and i has every element bit of the term's group set.  The
// run's terms are stored grouped by that element-bit set S, with group
// offsets (2^h + 1 words, TOp::tab); each thread sums its groups and a
// subset-sum over the element bits gives element i the total of every group
// S contained in i.  A condition h_j = 0 on an element bit is rewritten as
// 1 - h_j on the host, so every term's element condition is a set of ones.
// A DRUN_EPILOGUE run uses ETerm records over the layout of the block
// before it instead (thread code threadIdx.x, four element-code bits; the
// block kernel documents which tile bits those are).
struct DTerm {
    uint64_t omask, oval;
    uint64_t turns;
    uint32_t lmask, lval;   // thread bits only
};
static_assert(sizeof(DTerm) == 32, "DTerm layout");

// One term of a sign run (every term a factor of -1) applied in a block's
// epilogue (DRUN_EPILOGUE, complex64): the DTerm condition with the tile's
// outer-bit test taken over the workgroup index (the tile index, whose bits
// are the non-tile physical bits in ascending order), so that every field
// is 32 bits.  A term matches thread t of tile w when (w & om) == ov and
// (t & lm) == lv, and element code i when i contains its group's element
// bits; w holds the element codes it flips: the codes that contain its
// group.  The records are stored by group with offsets (17 words,
// TOp::tab); each group is padded to an even count with a record that
// never matches (om = 0, ov = 1), as the kernel reads two records per
// scalar load.  (Phase runs in epilogues use the phase sums below.)
struct ETerm {
    uint32_t om, ov;
    uint32_t lm, lv;
    uint32_t w;
    uint32_t pad_[3];       // 32 bytes: two records per 64-byte scalar load
};
static_assert(sizeof(ETerm) == 32, "ETerm layout");

// Phase runs in block epilogues (complex64) are encoded per pass as phase
// sums instead of ETerm records.  A run's terms are merged into combos: the
// terms of one group (element-code bits) with one thread condition
// (t & lm) == lv.  A combo's sum S(w) = sum of its records' turns whose
// tile-index test (w & om) == ov holds depends on the tile only, so each
// workgroup forms every combo's S once, on the scalar unit, while its tile
// loads are in flight (combos split over the waves), and keeps them in LDS
// after the cis table.  In the epilogue a thread adds S of each combo of
// a group whose thread condition it meets; that condition is stored as one
// 64-bit lane mask per wave (thread t = 64 wave + lane), so a combo costs a
// masked select and an add.
//
// The pass's table (PassDesc::psum): a PSumHead, then uint32 cb[ncombo + 1]
// (combo c's records are [cb[c], cb[c + 1])), the records (PRec, at
// rec_off) and the lane masks (uint64 mask[8][ncombo], at mask_off; byte
// offsets from the table).  A run op's tab holds 17 words: its groups'
// combo ranges (pass combo indices, each group's range a multiple of 4,
// padded with combos without records); its data is the pass's table.
struct PSumHead {
    uint32_t ncombo;        // multiple of 4
    uint32_t nrec;
    uint32_t rec_off;       // 16-byte aligned
    uint32_t mask_off;      // 16-byte aligned
};
struct PRec {
    uint32_t om, ov;        // tile-index test
    uint32_t w;             // turns of 2^-32
    uint32_t pad_;
};
static_assert(sizeof(PSumHead) == 16 && sizeof(PRec) == 16, "phase-sum layout");
constexpr int kPSumMax = 1024;     // combos per pass (4 KiB of LDS)

struct PassDesc {
    int32_t L;              // tile qubits
    int32_t c;              // low physical bits that are always tile bits (coalescing)
    int32_t nops;
    int32_t remap;          // nonzero: store through the remap table
    int32_t kmax;           // widest block in the pass (sizes the LDS fragment area)
    int32_t first_block;    // index of the pass's first TOP_BLOCK op, -1 if none
    uint64_t qmask;         // physical bits that are tile bits
    uint64_t ops;           // byte offset of TOp[nops]
    uint64_t ldoff;         // byte offset of uint64 off[2^(L-c)]: chunk -> physical offset
    uint64_t rmhi;          // byte offset of uint32 tab[2^(L-c)]: LDS slot of the remapped high local bits
    uint64_t rmlo;          // byte offset of uint32 tab[2^c]: LDS slot of the remapped low local bits
    uint64_t tabs;          // byte offset of the ops' address tables: op i's at tabs + i kTabStride
    uint64_t cistab;        // complex64 passes with a phase run in a block epilogue: byte offset
                            // of the cis table (kCisEntries float pairs), else 0
    uint64_t psum;          // such passes: byte offset of the phase-sum table, else 0
    int32_t npsum;          // its combo count (LDS words after the cis table)
    int32_t pad_;
};

// The cis table of complex64 phase runs in block epilogues: entry j is
// (cos, sin) of 2 pi j / kCisEntries, rounded to float; the kernel keeps it
// in LDS after the tile and multiplies an entry by the short Taylor factor
// of the remaining angle (below 2 pi / kCisEntries).
constexpr int kCisBits = 10;
constexpr int kCisEntries = 1 << kCisBits;

}  // namespace qvm
