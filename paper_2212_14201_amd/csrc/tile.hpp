// Device-visible plan records shared by the planner (host) and the tile
// kernel.  A plan is a list of passes; a pass streams every tile of 2^L
// amplitudes through LDS once and applies a list of ops to it.
#pragma once

#include <cstdint>

namespace qvm {

enum TileOpType : int32_t { TOP_BLOCK = 1, TOP_DIAGRUN = 2 };

constexpr size_t kTileLdsMax = 160 * 1024;   // LDS per workgroup on gfx950

// Diagonal-run flags (TOp::flags).
enum : int32_t {
    DRUN_TURNS = 1,         // accumulate each element's phase in turns, one factor per element
    DRUN_SIGNS = 2          // every term is a factor of -1 (with DRUN_TURNS: a sign flip per element)
};

struct TOp {
    int32_t type;
    int32_t k;              // block: matrix width in qubits; diagonal run: number of terms
    int32_t lb[6];          // block: local tile bit of block bit r
    uint64_t data;          // byte offset into the plan blob: fragments or DSub[k]
    int32_t next_block;     // index of the pass's next TOP_BLOCK op, -1 if none
    int32_t flags;          // diagonal run: DRUN_* bits
};

// One phase term of a diagonal run: amplitudes whose local tile bits match
// (lmask, lval) and whose tile's outer bits match (omask, oval) are
// multiplied by the unit-modulus factor (pr + i pi) = exp(2 pi i turns / 2^64);
// neg marks a factor of exactly -1.
struct DSub {
    uint32_t lmask, lval;
    int32_t neg;
    int32_t pad_;
    uint64_t omask, oval;
    double pr, pi;
    uint64_t turns;         // the factor's angle as a 64-bit fraction of a full turn
};

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
    uint64_t rmhi;          // byte offset of uint32 tab[2^(L-c)]: remap of the high local bits
    uint64_t rmlo;          // byte offset of uint32 tab[2^c]: remap of the low local bits
};

}  // namespace qvm
