// Fusion planner and plan execution (paper, "Quantum circuit fusion": the
// Fusion / aggregate_operations step that rewrites a program into unitary
// blocks before simulation; the paper does not specify its algorithm).
//
// A plan is built in three steps, all on the host in double precision:
//  1. Wires.  Uncontrolled SWAPs become relabelings of the wires (no data
//     movement); every later gate is rewritten onto wires.
//  2. Passes.  Gates are scheduled over their dependency order into passes.
//     A pass owns a tile of L physical bits that always includes the c
//     lowest ones; a gate whose matrix is not diagonal can run in a pass
//     only if all its qubits are tile bits, a diagonal gate can run in any
//     pass.  In "block" mode (L = 0 requested) every fused block gets a pass
//     of its own, i.e. one HBM round trip per block.
//  3. Blocks.  Inside a pass, gates are fused greedily over the dependency
//     frontier into blocks of at most k_max qubits; controls of a fused gate
//     are folded into the block matrix.  Diagonal gates whose qubits lie
//     outside the open block become phase/diagonal ops of their own.
// At the end of each pass the tile bits are permuted so that the qubits
// needed soonest sit on the low physical bits (qubit-index remapping).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <atomic>
#include <cmath>
#include <cstring>
#include <map>
#include <numeric>
#include <string>
#include <vector>

#include "internal.hpp"
#include "tile.hpp"

namespace qvm {

qvm_status launch_tile_pass(qvm_sv* sv, const PassDesc& pd, const char* blob_dev, double flops);

namespace {

struct PGate {
    int k;
    int t[QVM_MAX_K];            // wires
    uint64_t cmask;              // wires
    std::vector<cd> u;           // 2^k x 2^k
    bool diag;
    uint64_t qmask;              // targets | controls
    int src;                     // index in the caller's list
};

struct Unit {                    // a fused block or a standalone diagonal gate
    bool block;
    std::vector<int> gates;      // indices into the PGate list, in order
    std::vector<int> qubits;     // block qubits (wires), bit r <-> qubits[r]
};

struct PassPlan {
    std::vector<Unit> units;
};

std::atomic<uint64_t> g_plan_ids{1};

}  // namespace
}  // namespace qvm

struct qvm_plan {
    int n;
    qvm_dtype dt;
    int k_max;
    int tile_qubits;
    std::vector<char> blob;                 // device image
    std::vector<qvm::PassDesc> passes;
    std::vector<double> pass_flops;         // MFMA flops of each pass over the whole state
    std::vector<float> pass_features;       // QVM_PASS_FEATURES per pass
    std::vector<int> final_perm;            // logical qubit -> physical bit after the plan
    std::vector<uint32_t> block_of_gate;    // pass-ordered block id per input gate (-1: diag op)
    std::vector<int32_t> exec_pos;          // rank of each input gate in execution order (-1: relabel)
    std::vector<int32_t> unit_of;           // unit (block or diagonal op) of each input gate
    struct Block {
        std::vector<int> qubits;            // wires (logical qubits when no SWAP precedes), padded to >= 3
        int k_true;                         // qubits spanned by the block's gates
        std::vector<int> gates;             // input gate indices
        std::vector<qvm::cd> m;             // FP64 block matrix
        int pass;
    };
    std::vector<Block> blocks;
    int n_diag_ops;
    uint64_t id;
    uint64_t pass_table;                    // offset of the PassDesc table in the blob
    bool image;                             // false: built for scoring only (no matrices, no image)
};

namespace qvm {
namespace {

// y = G x for one gate on a small register (block-local bit positions).
void apply_small(std::vector<cd>& v, int k_reg, const cd* u, int k, const int* pos, uint64_t cm) {
    const uint64_t N = 1ull << k_reg;
    const int dim = 1 << k;
    uint64_t tm = 0;
    for (int r = 0; r < k; ++r) tm |= 1ull << pos[r];
    cd in[64];
    uint64_t idx[64];
    for (uint64_t b = 0; b < N; ++b) {
        if ((b & tm) || ((b & cm) != cm)) continue;
        for (int j = 0; j < dim; ++j) {
            uint64_t o = b;
            for (int r = 0; r < k; ++r)
                if ((j >> r) & 1) o |= 1ull << pos[r];
            idx[j] = o;
            in[j] = v[o];
        }
        for (int i = 0; i < dim; ++i) {
            // plain real arithmetic (finite operands; std::complex's product
            // would call the library's NaN-recovering routine per term)
            double sr = 0, si = 0;
            for (int j = 0; j < dim; ++j) {
                const double ar = u[i * dim + j].real(), ai = u[i * dim + j].imag();
                const double br = in[j].real(), bi = in[j].imag();
                sr += ar * br - ai * bi;
                si += ar * bi + ai * br;
            }
            v[idx[i]] = cd(sr, si);
        }
    }
}

// FP64 block matrix over `qubits` (bit r <-> qubits[r]) of the listed gates.
std::vector<cd> block_matrix(const std::vector<PGate>& G, const std::vector<int>& gates,
                             const std::vector<int>& qubits) {
    const int k = (int)qubits.size();
    const int dim = 1 << k;
    std::vector<cd> M((size_t)dim * dim, cd(0, 0));
    std::map<int, int> pos;
    for (int r = 0; r < k; ++r) pos[qubits[r]] = r;
    // each gate's targets and controls in block bit positions, once
    struct Placed { const PGate* g; int p[QVM_MAX_K]; uint64_t cm; };
    std::vector<Placed> pl(gates.size());
    for (size_t i = 0; i < gates.size(); ++i) {
        const PGate& g = G[gates[i]];
        pl[i].g = &g;
        for (int r = 0; r < g.k; ++r) pl[i].p[r] = pos.at(g.t[r]);
        pl[i].cm = 0;
        for (uint64_t m = g.cmask; m; m &= m - 1) pl[i].cm |= 1ull << pos.at(__builtin_ctzll(m));
    }
    std::vector<cd> col(dim);
    for (int c = 0; c < dim; ++c) {
        std::fill(col.begin(), col.end(), cd(0, 0));
        col[c] = 1.0;
        for (const Placed& x : pl) apply_small(col, k, x.g->u.data(), x.g->k, x.p, x.cm);
        for (int r = 0; r < dim; ++r) M[(size_t)r * dim + c] = col[r];
    }
    return M;
}

inline int popc(uint64_t v) { return __builtin_popcountll(v); }

// Dependency tracking over a gate subset: a gate is ready when every earlier
// gate (in the subset) sharing a qubit with it has been consumed.
struct Frontier {
    std::vector<std::vector<int>> per_q;     // per wire: gate indices in order
    std::vector<size_t> ptr;
    Frontier(int nq, const std::vector<PGate>& G, const std::vector<int>& subset)
        : per_q(nq), ptr(nq, 0) {
        for (int gi : subset)
            for (int q = 0; q < nq; ++q)
                if ((G[gi].qmask >> q) & 1) per_q[q].push_back(gi);
    }
    bool ready(const PGate& g, int gi) const {
        for (uint64_t m = g.qmask; m; m &= m - 1) {
            int q = __builtin_ctzll(m);
            if (ptr[q] >= per_q[q].size() || per_q[q][ptr[q]] != gi) return false;
        }
        return true;
    }
    void consume(const PGate& g) {
        for (uint64_t m = g.qmask; m; m &= m - 1) ++ptr[__builtin_ctzll(m)];
    }
};

// Greedy frontier fusion of an ordered gate subset into units.
std::vector<Unit> fuse(const std::vector<PGate>& G, const std::vector<int>& subset, int nq,
                       int k_max, uint64_t allowed) {
    std::vector<Unit> out;
    Frontier F(nq, G, subset);
    std::vector<char> done(subset.size(), 0);
    size_t left = subset.size();
    Unit cur{true, {}, {}};
    uint64_t S = 0;
    auto close = [&]() {
        if (!cur.gates.empty()) {
            for (int q = 0; q < nq; ++q)
                if ((S >> q) & 1) cur.qubits.push_back(q);
            out.push_back(cur);
        }
        cur = Unit{true, {}, {}};
        S = 0;
    };
    size_t first = 0;
    while (left) {
        bool progress = false;
        while (first < subset.size() && done[first]) ++first;
        for (size_t i = first; i < subset.size(); ++i) {
            if (done[i]) continue;
            const int gi = subset[i];
            const PGate& g = G[gi];
            if (!F.ready(g, gi)) continue;
            bool take = false;
            if (g.diag) {
                if (!cur.gates.empty() && (g.qmask & ~S) == 0) {
                    cur.gates.push_back(gi);
                    take = true;
                } else if (!cur.gates.empty() && (g.qmask & S) != 0 && (g.qmask & ~allowed) == 0 &&
                           popc(S | g.qmask) <= std::min(3, k_max)) {
                    // widening the block up to the 3 qubits it is padded to
                    // anyway costs nothing
                    cur.gates.push_back(gi);
                    S |= g.qmask;
                    take = true;
                } else if ((g.qmask & S) == 0) {
                    out.push_back(Unit{false, {gi}, {}});
                    take = true;
                }
            } else if (popc(S | g.qmask) <= k_max && (g.qmask & ~allowed) == 0) {
                cur.gates.push_back(gi);
                S |= g.qmask;
                take = true;
            }
            if (take) {
                F.consume(g);
                done[i] = 1;
                --left;
                progress = true;
            }
        }
        if (!progress) {
            if (cur.gates.empty()) {
                // a diagonal gate that overlaps nothing open is always takeable,
                // so an empty block without progress cannot happen; guard anyway
                break;
            }
            close();
        }
    }
    close();
    return out;
}

// Standalone diagonal units are multiplied into a neighbouring block: into
// the last block before them that touches any of their qubits, else into the
// first block after them that does (diagonal units in between are passed
// over: diagonal gates commute).  The block must cover the unit's qubits or
// be narrower than the 3 qubits every block is padded to anyway, in which case
// it grows by the unit's qubits (at most min(3, k_max), within `allowed`).
// The block matrix takes the phases for free, and per-qubit order is kept up
// to commuting diagonal gates.
void absorb_diagonals(std::vector<Unit>& units, const std::vector<PGate>& G, int k_max,
                      uint64_t allowed) {
    const int grow_to = std::min(3, k_max);
    auto qmask_of = [&](const Unit& u) {
        uint64_t m = 0;
        if (u.block)
            for (int q : u.qubits) m |= 1ull << q;
        else
            for (int gi : u.gates) m |= G[gi].qmask;
        return m;
    };
    auto take = [&](Unit& b, uint64_t m) {
        const uint64_t bm = qmask_of(b);
        if ((m & ~bm) == 0) return true;
        if ((m & ~allowed) != 0 || popc(bm | m) > grow_to) return false;
        for (uint64_t x = m & ~bm; x; x &= x - 1) b.qubits.push_back(__builtin_ctzll(x));
        return true;
    };
    std::vector<char> gone(units.size(), 0);
    // into the block before
    for (size_t i = 0; i < units.size(); ++i) {
        if (units[i].block) continue;
        const uint64_t m = qmask_of(units[i]);
        for (size_t j = i; j-- > 0;) {
            if (gone[j] || !units[j].block || (qmask_of(units[j]) & m) == 0) continue;
            if (take(units[j], m)) {
                for (int gi : units[i].gates) units[j].gates.push_back(gi);
                gone[i] = 1;
            }
            break;
        }
    }
    // into the block after
    for (size_t i = units.size(); i-- > 0;) {
        if (gone[i] || units[i].block) continue;
        const uint64_t m = qmask_of(units[i]);
        for (size_t j = i + 1; j < units.size(); ++j) {
            if (gone[j] || !units[j].block || (qmask_of(units[j]) & m) == 0) continue;
            if (take(units[j], m)) {
                units[j].gates.insert(units[j].gates.begin(), units[i].gates.begin(), units[i].gates.end());
                gone[i] = 1;
            }
            break;
        }
    }
    std::vector<Unit> kept;
    kept.reserve(units.size());
    for (size_t i = 0; i < units.size(); ++i)
        if (!gone[i]) kept.push_back(std::move(units[i]));
    units.swap(kept);
}

struct Builder {
    int n;
    qvm_dtype dt;
    int c;            // low bits always in the tile
    int L;            // tile bits per pass
    std::vector<char>& blob;
    explicit Builder(std::vector<char>& b) : blob(b) {}
    size_t put(const void* p, size_t bytes) {
        size_t off = (blob.size() + 255) & ~size_t(255);
        blob.resize(off + bytes);
        if (bytes) memcpy(blob.data() + off, p, bytes);
        return off;
    }
};

// Runs of at least this many terms take the angle-accumulating path of the
// tile kernel (one integer add per term and thread, then one complex factor
// per element); shorter runs multiply term by term.  Sign-only runs end in a
// sign flip instead of a factor, so they pay off sooner.
constexpr int kTurnsMinTerms = 8;
constexpr int kTurnsMinSignTerms = 4;

// Angle of a unit-modulus factor as a 64-bit fraction of a full turn,
// rounded: exp(2 pi i turns / 2^64) = v.
uint64_t turns_of(cd v) {
    double a = std::atan2(v.imag(), v.real()) / (2.0 * M_PI);      // (-1/2, 1/2]
    if (a < 0) a += 1.0;                                            // [0, 1)
    const double s = std::ldexp(a, 64);
    if (!(s < 18446744073709551616.0)) return 0;                    // rounded up to a full turn
    return (uint64_t)std::nearbyint(s);
}

// Angle-path terms of a diagonal run (layout in tile.hpp): each term's angle
// in the kernel's fixed-point width.  bitmap[b] says where tile bit b sits
// in the code the kernel evaluates: a thread-code bit (0..8: the term's
// lmask / lval) or, as 32 + j, element-code bit j (the groups).  A
// condition h = 0 on an element bit becomes 1 - h, so a term splits into
// +-angle on the supersets of its required ones; terms with equal
// conditions in a group are merged (sums modulo a full turn are exact) and
// zero sums dropped.  off gets 2^h + 1 group offsets (h element bits).
void angle_terms(const std::vector<DSub>& run, int L, qvm_dtype dt, const int8_t* bitmap, int nhb,
                 std::vector<DTerm>& terms, std::vector<uint32_t>& off) {
    const uint32_t ne = 1u << nhb;
    const uint64_t wmask = dt == QVM_C64 ? 0xffffffffull : ~0ull;
    std::vector<std::vector<DTerm>> grp(ne);
    for (const DSub& d : run) {
        const uint64_t w = dt == QVM_C64 ? (d.turns + (1ull << 31)) >> 32 : d.turns;
        uint32_t tm = 0, tv = 0, mh = 0, vh = 0;
        for (int b = 0; b < L; ++b) {
            if (!((d.lmask >> b) & 1)) continue;
            const int to = bitmap[b];
            const uint32_t v = (d.lval >> b) & 1;
            if (to >= 32) {
                mh |= 1u << (to - 32);
                vh |= v << (to - 32);
            } else {
                tm |= 1u << to;
                tv |= v << to;
            }
        }
        const uint32_t ones = mh & vh, zeros = mh & ~vh;
        for (uint32_t T = zeros;; T = (T - 1) & zeros) {
            const uint64_t v = (__builtin_popcount(T) & 1 ? 0 - w : w) & wmask;
            std::vector<DTerm>& g = grp[ones | T];
            auto same = std::find_if(g.begin(), g.end(), [&](const DTerm& e) {
                return e.omask == d.omask && e.oval == d.oval && e.lmask == tm && e.lval == tv;
            });
            if (same != g.end()) same->turns = (same->turns + v) & wmask;
            else g.push_back(DTerm{d.omask, d.oval, v, tm, tv});
            if (T == 0) break;
        }
    }
    terms.clear();
    off.assign(ne + 1, 0);
    for (uint32_t g = 0; g < ne; ++g) {
        for (const DTerm& e : grp[g])
            if (e.turns) terms.push_back(e);
        off[g + 1] = (uint32_t)terms.size();
    }
}

// Bits of x at the zero positions of qmask (the tile's outer bits), packed
// in ascending order: x's bits as bits of the tile (workgroup) index.
static uint32_t outer_bits(uint64_t x, uint64_t qmask) {
    uint32_t r = 0;
    int j = 0;
    for (int p = 0; p < 64 && j < 32; ++p) {
        if ((qmask >> p) & 1) continue;
        if ((x >> p) & 1) r |= 1u << j;
        ++j;
    }
    return r;
}

// Epilogue-run records (ETerm) from the grouped angle-path terms of a run
// over the epilogue layout (four element-code bits): outer conditions over
// the tile index, sign runs with their groups' element-code sets, every
// group padded to an even count.
void epilogue_terms(const std::vector<DTerm>& terms, const std::vector<uint32_t>& off, uint64_t qmask, bool signs,
                    std::vector<ETerm>& et, std::vector<uint32_t>& eoff) {
    et.clear();
    eoff.assign(17, 0);
    for (uint32_t g = 0; g < 16; ++g) {
        uint32_t sup = 0;                                  // element codes containing g
        for (uint32_t i = 0; i < 16; ++i)
            if ((i & g) == g) sup |= 1u << i;
        for (uint32_t q = off[g]; q < off[g + 1]; ++q) {
            const DTerm& d = terms[q];
            ETerm e{};
            e.om = outer_bits(d.omask, qmask);
            e.ov = outer_bits(d.oval, qmask);
            e.lm = d.lmask;
            e.lv = d.lval;
            e.w = signs ? sup : (uint32_t)d.turns;
            et.push_back(e);
        }
        if (et.size() & 1) {
            ETerm pad{};
            pad.ov = 1;                                    // (w & 0) != 1: never matches
            et.push_back(pad);
        }
        eoff[g + 1] = (uint32_t)et.size();
    }
}

// Phase sums of the phase runs a pass applies in block epilogues (layout
// in tile.hpp), built run by run: a run's terms by group and thread
// condition (combos, in order of first appearance), records with equal
// tile-index tests merged and zero sums dropped, each thread condition as
// one lane mask per wave (thread t = 64 wave + lane), every group's combos
// padded to a multiple of 4.
struct PSumBuild {
    std::vector<uint32_t> cb{0};
    std::vector<PRec> recs;
    std::vector<std::array<uint64_t, kTileThreads / 64>> masks;   // per wave
};

void epilogue_psums(const std::vector<DTerm>& terms, const std::vector<uint32_t>& off, uint64_t qmask,
                    PSumBuild& ps, std::vector<uint32_t>& goff) {
    goff.assign(17, (uint32_t)ps.masks.size());
    for (uint32_t g = 0; g < 16; ++g) {
        std::vector<std::pair<uint64_t, std::vector<PRec>>> combos;
        for (uint32_t q = off[g]; q < off[g + 1]; ++q) {
            const DTerm& d = terms[q];
            const uint64_t key = (uint64_t)d.lmask << 32 | d.lval;
            auto c = std::find_if(combos.begin(), combos.end(), [&](const auto& x) { return x.first == key; });
            if (c == combos.end()) c = combos.insert(combos.end(), std::make_pair(key, std::vector<PRec>{}));
            const PRec r{outer_bits(d.omask, qmask), outer_bits(d.oval, qmask), (uint32_t)d.turns, 0};
            auto same = std::find_if(c->second.begin(), c->second.end(),
                                     [&](const PRec& e) { return e.om == r.om && e.ov == r.ov; });
            if (same != c->second.end()) same->w += r.w;
            else c->second.push_back(r);
        }
        for (auto& c : combos) {
            size_t kept = 0;
            for (const PRec& r : c.second)
                if (r.w) {
                    ps.recs.push_back(r);
                    ++kept;
                }
            if (!kept) continue;
            const uint32_t lm = (uint32_t)(c.first >> 32), lv = (uint32_t)c.first;
            std::array<uint64_t, kTileThreads / 64> m{};
            for (uint32_t w = 0; w < kTileThreads / 64; ++w)
                for (uint32_t lane = 0; lane < 64; ++lane)
                    if (((64 * w + lane) & lm) == lv) m[w] |= 1ull << lane;
            ps.cb.push_back((uint32_t)ps.recs.size());
            ps.masks.push_back(m);
        }
        while ((ps.masks.size() - goff[g]) % 4) {
            ps.cb.push_back((uint32_t)ps.recs.size());
            ps.masks.push_back({});
        }
        goff[g + 1] = (uint32_t)ps.masks.size();
    }
}

// Upper bound on the combos a phase run adds to its pass's phase sums,
// whatever block layout it ends up on: a condition h = 0 on an element bit
// splits a term in two (at most four element bits), and each group's
// combos are padded to a multiple of 4.
int psum_bound(const std::vector<DSub>& run, int L) {
    const uint64_t tile = L >= 64 ? ~0ull : (1ull << L) - 1;
    int n = 16 * 3;
    for (const DSub& d : run) n += 1 << std::min(4, __builtin_popcountll(d.lmask & ~d.lval & tile));
    return n;
}

// The standalone run's element layout: thread t holds elements
// t + kTileThreads i, so tile bits below kLogTileThreads are thread bits and
// the ones above are element bits.
int run_bitmap(int L, int8_t* bitmap) {
    for (int b = 0; b < L; ++b) bitmap[b] = (int8_t)(b < kLogTileThreads ? b : 32 + b - kLogTileThreads);
    return L > kLogTileThreads ? L - kLogTileThreads : 0;
}

// Column roles of a block op (layout in tile.hpp): the tile bits outside
// the block, in ascending order, give the lane's four column bits and then
// the bits of the column-tile index ti; with wave bits W (three tile bits
// outside the block), W takes the ti bits above the CT bits (the wave's)
// and the other bits keep ascending order around it.  W = 0 is the default
// layout (every role in ascending order).
struct ColMap {
    int nlane = 0;
    int lane[4] = {0, 0, 0, 0};
    std::vector<int> tib;          // tile bit of ti bit j
};

ColMap col_map(const int32_t* lb, int k, int L, qvm_dtype dt, uint32_t W) {
    uint32_t bmask = 0;
    for (int r = 0; r < k; ++r) bmask |= 1u << lb[r];
    std::vector<int> rest;
    for (int b = 0; b < L; ++b)
        if (!((bmask >> b) & 1) && !((W >> b) & 1)) rest.push_back(b);
    ColMap m;
    m.nlane = std::min(4, (int)rest.size());
    // lane bits: the lowest free bits whose slots are independent in the
    // low slot bits that select the LDS bank (complex64: bits 0..3, the 16
    // lanes of a 64-bit access; complex128: bits 0..2, the 8 lanes of a
    // 128-bit access, lane bits 0..2), picked greedily (a basis of the
    // widest span, lowest bits first), then the lowest remaining bits
    const uint32_t bank = dt == QVM_C128 ? 7u : 15u;
    const int nind = dt == QVM_C128 ? 3 : 4;
    std::vector<int> pick;
    uint32_t basis[4] = {0, 0, 0, 0};         // reduced images, by leading bit
    for (int b : rest) {
        if ((int)pick.size() >= std::min(nind, m.nlane)) break;
        uint32_t v = tile_swizzle(1u << b) & bank;
        for (int j = 3; j >= 0 && v; --j)
            if ((v >> j) & 1) {
                if (!basis[j]) break;
                v ^= basis[j];
            }
        if (!v) continue;
        int lead = 31 - __builtin_clz(v);
        basis[lead] = v;
        pick.push_back(b);
    }
    for (int b : rest)
        if ((int)pick.size() < m.nlane && std::find(pick.begin(), pick.end(), b) == pick.end()) pick.push_back(b);
    std::sort(pick.begin(), pick.begin() + std::min((int)pick.size(), nind));
    for (int i = 0; i < m.nlane; ++i) m.lane[i] = pick[i];
    for (int i = 0; i < m.nlane; ++i) rest.erase(std::find(rest.begin(), rest.end(), pick[i]));
    if (!W) {
        m.tib = rest;
        return m;
    }
    const int ct = block_ct(k, L, dt == QVM_C128);
    int lct = 0;
    while ((1 << lct) < ct) ++lct;
    m.tib.assign(rest.begin(), rest.begin() + lct);
    for (int b = 0; b < L; ++b)
        if ((W >> b) & 1) m.tib.push_back(b);
    m.tib.insert(m.tib.end(), rest.begin() + lct, rest.end());
    return m;
}

// Blocks whose waves may keep their elements across blocks: up to 4 qubits
// (register fragments) and at least one full iteration of column tiles per
// wave (ntile >= 8 CT), so that ti has three wave bits.
bool wave_bits_ok(int k, int L, qvm_dtype dt) {
    if (k > 4 || L - k < 4) return false;
    const int ntile = 1 << (L - k - 4);
    return ntile >= 8 * block_ct(k, L, dt == QVM_C128);
}

// A diagonal run can ride in the epilogue of a complex64 3- or 4-qubit block
// in a 13-qubit tile (one column iteration per wave; tile.hip).
bool epilogue_ok(int k, int L, qvm_dtype dt) { return dt == QVM_C64 && L == 13 && (k == 3 || k == 4); }

// The element layout of such an epilogue: lane l = 0..63, wave w, column
// tile ct < CT (8 for k = 3, 4 for k = 4) and row block rb < K / 16 hold
// column tile CT w + ct, the lane's column l & 15, and complex row
// 8 rb + 2 (l >> 4) + hh of the block, hh = 0, 1.  Thread code:
// (l & 15) | (l >> 4) << 4 | w << 6; element code: hh | ct << 1 | rb << (1 + log2 CT).
// bitmap[b] = thread-code bit of tile bit b, or 32 + its element-code bit.
void epilogue_bitmap(const int32_t* lb, int k, const ColMap& cm, int8_t* bitmap) {
    const int lct = k == 3 ? 3 : 2;
    for (int i = 0; i < cm.nlane; ++i) bitmap[cm.lane[i]] = (int8_t)i;
    for (int j = 0; j < (int)cm.tib.size(); ++j)
        bitmap[cm.tib[j]] = (int8_t)(j < lct ? 32 + 1 + j : 6 + (j - lct));
    for (int r = 0; r < k; ++r)
        bitmap[lb[r]] = (int8_t)(r == 0 ? 32 : r <= 2 ? 4 + (r - 1) : 32 + 1 + lct);
}

// Address table of a block op (layout in tile.hpp): the wave-uniform parts
// of its LDS slots, computed once here instead of per access in the kernel.
std::vector<uint32_t> block_table(const int32_t* lb, int k, int L, qvm_dtype dt, const ColMap& cm) {
    auto rows = [&](int j) {                     // block row index -> tile bits
        uint32_t e = 0;
        for (int q = 0; q < k; ++q)
            if ((j >> q) & 1) e |= 1u << lb[q];
        return e;
    };
    const BlockTabLayout lay(L, k);
    const uint32_t es = dt == QVM_C64 ? 8u : 16u;     // bytes per amplitude
    std::vector<uint32_t> t((size_t)lay.words(), 0u);
    for (int ti = 0; ti < lay.ntile; ++ti) {
        uint32_t e = 0;
        for (int j = 0; j < (int)cm.tib.size(); ++j)
            if ((ti >> j) & 1) e |= 1u << cm.tib[j];
        t[lay.col() + ti] = es * tile_swizzle(e);
    }
    for (int i = 0; i < lay.nb; ++i) t[lay.brow() + i] = es * tile_swizzle(rows(4 * i));
    for (int rb = 0; rb < lay.ne / 4; ++rb)
        for (int r = 0; r < 4; ++r) {
            // complex64: registers (2h, 2h+1) hold output row 8 rb + h (plus
            // the lane's 2 (l / 16)); complex128: register r holds row
            // 8 rb + 2 r (plus the lane's (l / 16) / 2)
            const int j = dt == QVM_C64 ? (r < 2 ? 8 * rb + r : -1) : 8 * rb + 2 * r;
            t[lay.erow() + 4 * rb + r] = j < 0 ? 0u : es * tile_swizzle(rows(j));
        }
    for (int i = 0; i < cm.nlane; ++i) t[lay.lane() + i] = es * tile_swizzle(1u << cm.lane[i]);
    for (int r = 0; r < std::min(k, 4); ++r) t[lay.rbit() + r] = es * tile_swizzle(1u << lb[r]);
    return t;
}

// Real MFMA fragments of a complex 2^k x 2^k matrix: K = 2^(k+1);
// fragment (rb, s), lane l holds Mr[16 rb + l % 16][col(s, l / 16)] with
// Mr = [[Re, -Im], [Im, Re]] per complex entry (real index 2 j + part for
// complex index j).  The contraction index is permuted so that k-steps
// 2t and 2t+1 take the real and imaginary parts of the same complex input
// row: col(s, g) = 2 (4 (s / 2) + g) + (s % 2).  A lane then reads each
// input amplitude as one (re, im) pair.
template <typename R>
std::vector<R> fragments(const std::vector<cd>& M, int k) {
    const int dim = 1 << k, K = 2 * dim, RB = K / 16, KS = K / 4;
    auto mr = [&](int i, int j) -> double {
        cd v = M[(size_t)(i >> 1) * dim + (j >> 1)];
        int a = i & 1, b = j & 1;
        if (a == 0 && b == 0) return v.real();
        if (a == 0 && b == 1) return -v.imag();
        if (a == 1 && b == 0) return v.imag();
        return v.real();
    };
    std::vector<R> f((size_t)RB * KS * 64);
    for (int rb = 0; rb < RB; ++rb)
        for (int s = 0; s < KS; ++s)
            for (int l = 0; l < 64; ++l)
                f[((size_t)rb * KS + s) * 64 + l] =
                    (R)mr(16 * rb + (l & 15), 2 * (4 * (s >> 1) + (l >> 4)) + (s & 1));
    return f;
}

}  // namespace

qvm_status build_plan(const qvm_gate* gates, size_t ng, int n, qvm_dtype dt, int k_max,
                      int tile_qubits, const uint32_t* partition, qvm_plan** out, bool image,
                      const int32_t* k_of_pass = nullptr, int n_k_of_pass = 0, bool defer_narrow = false) {
    if (!out) return fail(QVM_EARG, "NULL out");
    *out = nullptr;
    if (n < 1 || n > QVM_MAX_QUBITS) return fail(QVM_EARG, "n_qubits outside 1..34");
    if (dt != QVM_C64 && dt != QVM_C128) return fail(QVM_EARG, "unknown dtype");
    if (ng && !gates) return fail(QVM_EARG, "NULL gate list");
    if (k_max < 1 || k_max > 6) return fail(QVM_EARG, "k_max outside 1..6");
    if (n < 3) return fail(QVM_EUNSUPPORTED, "fused plans need n >= 3 (blocks are padded to 3 qubits)");
    // LDS per workgroup: the tile plus the widest block's real fragments
    const int Lmax = dt == QVM_C64 ? 13 : (k_max >= 6 ? 11 : 12);
    const int cdef = dt == QVM_C64 ? 4 : 3;
    if (tile_qubits != 0 && (tile_qubits < k_max || tile_qubits > Lmax))
        return fail(QVM_EARG, "tile_qubits must be 0 or in k_max..13 (complex64) / ..12 (complex128, 11 with k_max = 6)");
    // ---- lower gates onto wires
    std::vector<PGate> G;
    G.reserve(ng);
    std::vector<int> wire(n);
    std::iota(wire.begin(), wire.end(), 0);
    std::vector<int> src_of;
    for (size_t i = 0; i < ng; ++i) {
        qvm_status st = validate_gate(gates[i], n, true);
        if (st) return fail(st, "gate " + std::to_string(i) + ": " + std::string(qvm_last_error()));
        const qvm_gate& g = gates[i];
        if (g.kind == QVM_G_SWAP && g.ctrl_mask == 0 && !partition) {
            std::swap(wire[g.targets[0]], wire[g.targets[1]]);
            continue;
        }
        PGate p{};
        p.k = g.k;
        p.cmask = 0;
        p.qmask = 0;
        for (int r = 0; r < g.k; ++r) {
            p.t[r] = wire[g.targets[r]];
            p.qmask |= 1ull << p.t[r];
        }
        for (int q = 0; q < n; ++q)
            if ((g.ctrl_mask >> q) & 1) p.cmask |= 1ull << wire[q];
        p.qmask |= p.cmask;
        st = gate_matrix(g, p.u);
        if (st) return st;
        const int dim = 1 << p.k;
        // diagonal: zero off the diagonal and unit-modulus entries (the
        // diagonal runs apply pure phases); other diagonal matrices are blocks
        p.diag = true;
        for (int r = 0; r < dim && p.diag; ++r)
            for (int cc = 0; cc < dim; ++cc)
                if (r != cc ? p.u[(size_t)r * dim + cc] != cd(0, 0)
                            : std::fabs(std::abs(p.u[(size_t)r * dim + cc]) - 1.0) > 1e-12) {
                    p.diag = false;
                    break;
                }
        p.src = (int)i;
        if (popc(p.qmask) > k_max && !p.diag)
            return fail(QVM_EARG, "gate " + std::to_string(i) + " spans more than k_max qubits");
        G.push_back(p);
    }
    const int ngw = (int)G.size();
    // ---- tile geometry
    int L = tile_qubits ? tile_qubits : Lmax;
    if (L > n) L = n;
    int c = std::min(cdef, L);
    if (L < std::min(n, std::max(k_max, 3)))
        return fail(QVM_EARG, "tile too small for k_max");
    // the lowest c physical bits are in every tile; a tile no wider than
    // them could never take a gate on any other qubit
    if (L < n && L <= c)
        return fail(QVM_EARG, "tile_qubits must exceed " + std::to_string(cdef) +
                                  " (the low bits every tile holds) when the state has more qubits");
    // one workgroup of kTileThreads per tile: the grid must stay below 2^32
    // threads (at 34 qubits, tiles of at least 12 qubits)
    if ((uint64_t)kTileThreads << (n - L) > 0xFFFFFFFFull)
        return fail(QVM_EARG, "tile of " + std::to_string(L) + " qubits too narrow for " + std::to_string(n) +
                                  " qubits: the pass would launch 2^32 or more threads");

    // ---- units for block / partition modes (one pass per block)
    std::vector<int> all(ngw);
    std::iota(all.begin(), all.end(), 0);
    std::vector<Unit> units;
    if (partition) {
        std::map<uint32_t, std::vector<int>> byid;
        for (int gi = 0; gi < ngw; ++gi) byid[partition[G[gi].src]].push_back(gi);
        for (auto& kv : byid) {
            uint64_t S = 0;
            for (int gi : kv.second) S |= G[gi].qmask;
            if (popc(S) > k_max) return fail(QVM_EARG, "partition block spans more than k_max qubits");
            Unit u{true, kv.second, {}};
            for (int q = 0; q < n; ++q)
                if ((S >> q) & 1) u.qubits.push_back(q);
            units.push_back(u);
        }
        std::vector<int> order(ngw);
        int t = 0;
        for (auto& u : units)
            for (int gi : u.gates) order[gi] = t++;
        std::vector<int> last(n, -1);
        for (int gi = 0; gi < ngw; ++gi)
            for (int q = 0; q < n; ++q)
                if ((G[gi].qmask >> q) & 1) {
                    if (last[q] >= 0 && order[last[q]] > order[gi])
                        return fail(QVM_EARG, "partition breaks the gate order on qubit " + std::to_string(q));
                    last[q] = gi;
                }
    } else if (tile_qubits == 0) {
        units = fuse(G, all, n, k_max, ~0ull);
        absorb_diagonals(units, G, k_max, ~0ull);
    }
    const bool tile_mode = !partition && tile_qubits != 0;
    size_t next_unit = 0;
    int idle_passes = 0;             // consecutive tile passes that took no gate

    // ---- schedule, fuse and emit passes
    qvm_plan* P = new (std::nothrow) qvm_plan();
    if (!P) return fail(QVM_ENOMEM, "host allocation failed");
    P->n = n;
    P->dt = dt;
    P->k_max = k_max;
    P->tile_qubits = tile_qubits;
    P->n_diag_ops = 0;
    P->id = g_plan_ids.fetch_add(1);
    P->image = image;
    P->block_of_gate.assign(ng, 0xffffffffu);
    P->exec_pos.assign(ng, -1);
    P->unit_of.assign(ng, -1);
    int32_t exec_counter = 0, unit_counter = 0;
    Builder B(P->blob);
    size_t cis_off = 0;                  // the plan's cis table (put once, when a pass needs it)
    std::vector<int> pos(n), at(n);      // wire -> physical bit, physical bit -> wire
    std::iota(pos.begin(), pos.end(), 0);
    std::iota(at.begin(), at.end(), 0);
    Frontier F(n, G, all);
    std::vector<char> done(ngw, 0);
    int left = ngw;
    int first = 0;
    auto fail_plan = [&](qvm_status st, const std::string& m) {
        delete P;
        return fail(st, m);
    };
    while (tile_mode ? left > 0 : next_unit < units.size()) {
        PassPlan pp;
        uint64_t T = 0;
        for (int b = 0; b < c; ++b) T |= 1ull << at[b];
        if (tile_mode) {
            std::vector<int> taken;
            bool progress = true;
            while (progress) {
                progress = false;
                while (first < ngw && done[first]) ++first;
                for (int gi = first; gi < ngw; ++gi) {
                    if (done[gi] || !F.ready(G[gi], gi)) continue;
                    uint64_t need = G[gi].diag ? 0 : G[gi].qmask;
                    if (popc(T | need) > L) continue;
                    T |= need;
                    F.consume(G[gi]);
                    done[gi] = 1;
                    --left;
                    taken.push_back(gi);
                    progress = true;
                }
            }
            // Nothing fits (the next gate needs more wires outside the low
            // bits than the tile has free slots): this pass runs no ops; it
            // loads the wires needed soonest and its remap moves them onto
            // the low bits (where they stay while still needed soonest), so
            // after at most a few such passes the gate fits.
            if (taken.empty() && ++idle_passes > n) return fail_plan(QVM_EARG, "planner made no progress");
            if (!taken.empty()) idle_passes = 0;
            // fill the tile up to L with the wires needed soonest
            std::vector<std::pair<int, int>> nxt;
            for (int q = 0; q < n; ++q) {
                if ((T >> q) & 1) continue;
                int when = ngw;
                for (int gi = first; gi < ngw; ++gi)
                    if (!done[gi] && !G[gi].diag && ((G[gi].qmask >> q) & 1)) { when = gi; break; }
                nxt.push_back({when, q});
            }
            std::sort(nxt.begin(), nxt.end());
            for (auto& w : nxt) {
                if (popc(T) >= L) break;
                T |= 1ull << w.second;
            }
            // block width of this pass: a pass's gates depend only on the
            // tile width, so each pass may fuse them with its own k
            const int kp = k_of_pass ? k_of_pass[std::min((int)P->passes.size(), n_k_of_pass - 1)] : k_max;
            pp.units = fuse(G, taken, n, kp, T);
            absorb_diagonals(pp.units, G, kp, T);
            // A block narrower than 3 qubits costs a full 3-qubit block.  When
            // such a block's gates are the last this pass takes on each of
            // their wires, they are left to a later pass (which needs those
            // wires for their successors anyway), where they join the block
            // of those successors.  Not in the last pass, and never every
            // block of a pass.
            if (defer_narrow && left > 0 && kp >= 3) {
                std::vector<char> defer(pp.units.size(), 0);
                int nblocks = 0, ndefer = 0;
                for (size_t ui = 0; ui < pp.units.size(); ++ui) {
                    const Unit& u = pp.units[ui];
                    if (!u.block) continue;
                    ++nblocks;
                    if (u.qubits.size() >= 3) continue;
                    std::vector<int> cnt(n, 0);
                    for (int gi : u.gates)
                        for (uint64_t m = G[gi].qmask; m; m &= m - 1) ++cnt[__builtin_ctzll(m)];
                    bool trailing = true;
                    for (int q = 0; q < n && trailing; ++q)
                        for (int j = 1; j <= cnt[q] && trailing; ++j) {
                            const int gj = F.per_q[q][F.ptr[q] - j];
                            trailing = std::find(u.gates.begin(), u.gates.end(), gj) != u.gates.end();
                        }
                    if (trailing) {
                        defer[ui] = 1;
                        ++ndefer;
                    }
                }
                if (ndefer && ndefer < nblocks) {
                    for (size_t ui = 0; ui < pp.units.size(); ++ui) {
                        if (!defer[ui]) continue;
                        for (int gi : pp.units[ui].gates) {
                            for (uint64_t m = G[gi].qmask; m; m &= m - 1) --F.ptr[__builtin_ctzll(m)];
                            done[gi] = 0;
                            ++left;
                            taken.erase(std::find(taken.begin(), taken.end(), gi));
                        }
                    }
                    first = 0;
                    pp.units = fuse(G, taken, n, kp, T);
                    absorb_diagonals(pp.units, G, kp, T);
                }
            }
        } else {
            // diagonal units ride in the pass of the next block
            while (next_unit < units.size()) {
                pp.units.push_back(units[next_unit++]);
                if (pp.units.back().block) break;
            }
            for (auto& u : pp.units)
                if (u.block)
                    for (int q : u.qubits) T |= 1ull << q;
            if (popc(T) > L) return fail_plan(QVM_EARG, "block does not fit the tile");
            for (int b = c; b < n && popc(T) < L; ++b) T |= 1ull << at[b];
        }
        // local bit of each tile wire: ascending physical bit (the c low
        // physical bits come first)
        std::vector<int> phys;
        for (int q = 0; q < n; ++q)
            if ((T >> q) & 1) phys.push_back(pos[q]);
        std::sort(phys.begin(), phys.end());
        if ((int)phys.size() != L) return fail_plan(QVM_EARG, "internal: tile size mismatch");
        for (int b = 0; b < c; ++b)
            if (phys[b] != b) return fail_plan(QVM_EARG, "internal: low bits missing from the tile");
        std::vector<int> local_of_wire(n, -1);
        uint64_t qmask = 0;
        for (int i = 0; i < L; ++i) {
            local_of_wire[at[phys[i]]] = i;
            qmask |= 1ull << phys[i];
        }
        const int pi = (int)P->passes.size();
        std::vector<TOp> ops;
        std::vector<DSub> run;
        // runs that ride in a block's epilogue: encoded once the block's
        // column layout is fixed (after the wave bits are chosen)
        std::vector<std::pair<size_t, std::vector<DSub>>> epi_runs;
        int psum_combos = 0;          // bound on the phase sums' combos so far
        // Diagonal gates commute with each other and with blocks on other
        // wires, so they are held back until a block touches one of their
        // wires (or the pass ends) and then emitted as one run: fewer, longer
        // runs.  Their schedule positions are given when they are emitted.
        std::vector<const Unit*> held;
        uint64_t held_wires = 0;
        auto place = [&](const Unit& u) {
            for (int gi : u.gates) {
                P->exec_pos[G[gi].src] = exec_counter++;
                P->unit_of[G[gi].src] = unit_counter;
            }
            ++unit_counter;
        };
        // widest block of the pass (blocks are padded to 3 qubits)
        int kmax_pass = 0;
        for (const auto& u : pp.units)
            if (u.block) kmax_pass = std::max(kmax_pass, std::max(3, (int)u.qubits.size()));
        auto flush = [&]() {
            for (const Unit* h : held) place(*h);
            held.clear();
            held_wires = 0;
            if (run.empty()) return;
            TOp op{};
            op.type = TOP_DIAGRUN;
            // long runs accumulate angles (one add per term and thread, one
            // factor per element); short ones multiply term by term
            bool signs = true;
            for (const DSub& d : run) signs = signs && d.neg;
            const int at_least = signs ? kTurnsMinSignTerms : kTurnsMinTerms;
            int8_t bitmap[32];
            // (passes with blocks of 5 or more qubits stage fragments in LDS and
            // apply every run on its own)
            // (a phase run's sums share a bounded LDS area with the pass's others)
            const int need = signs ? 0 : psum_bound(run, L);
            const bool fuse_prev = !ops.empty() && ops.back().type == TOP_BLOCK && kmax_pass <= 4 &&
                                   !(ops.back().flags & BLK_RUN) && epilogue_ok(ops.back().k, L, dt) &&
                                   psum_combos + need <= kPSumMax;
            if (fuse_prev) {
                // applied in the block's epilogue (no pass of its own); the
                // default layout tells whether the run's phases cancel
                epilogue_bitmap(ops.back().lb, ops.back().k, col_map(ops.back().lb, ops.back().k, L, dt, 0), bitmap);
                std::vector<DTerm> terms;
                std::vector<uint32_t> off;
                angle_terms(run, L, dt, bitmap, 4, terms, off);
                if (terms.empty()) {
                    run.clear();
                    return;
                }
                op.k = (int32_t)terms.size();
                op.flags = DRUN_TURNS | (signs ? DRUN_SIGNS : 0) | DRUN_EPILOGUE;
                ops.back().flags |= BLK_RUN | (signs ? BLK_RUN_SIGNS : 0);
                psum_combos += need;
                epi_runs.emplace_back(ops.size(), std::move(run));
                run.clear();
            } else if ((int)run.size() >= at_least) {
                // the angle path
                const int nhb = run_bitmap(L, bitmap);
                std::vector<DTerm> terms;
                std::vector<uint32_t> off;
                angle_terms(run, L, dt, bitmap, nhb, terms, off);
                run.clear();
                if (terms.empty()) return;          // the run's phases cancel
                op.k = (int32_t)terms.size();
                op.flags = DRUN_TURNS | (signs ? DRUN_SIGNS : 0);
                op.data = B.put(terms.data(), terms.size() * sizeof(DTerm));
                op.tab = B.put(off.data(), off.size() * sizeof(uint32_t));
            } else {
                op.k = (int32_t)run.size();
                op.data = B.put(run.data(), run.size() * sizeof(DSub));
                run.clear();
            }
            ops.push_back(op);
        };
        for (auto& u : pp.units) {
            TOp op{};
            if (u.block) {
                uint64_t bw = 0;
                for (int w : u.qubits) bw |= 1ull << w;
                if (held_wires & bw) flush();
                place(u);
                std::vector<int> bq = u.qubits;
                const int k_true = (int)bq.size();
                for (int i = 0; (int)bq.size() < 3 && i < L; ++i) {
                    int w = at[phys[i]];
                    if (std::find(bq.begin(), bq.end(), w) == bq.end()) bq.push_back(w);
                }
                const int k = (int)bq.size();
                std::vector<cd> M;
                op.type = TOP_BLOCK;
                op.k = k;
                for (int r = 0; r < k; ++r) op.lb[r] = local_of_wire[bq[r]];
                if (image) {
                    M = block_matrix(G, u.gates, bq);
                    // in a pass whose widest block has 4 qubits the kernel
                    // fetches every block's fragments as 16 values per lane:
                    // 3-qubit fragments are padded with zeros to that size
                    const size_t pad = kmax_pass == 4 ? (size_t)16 * 64 : 0;
                    if (dt == QVM_C64) {
                        auto f = fragments<float>(M, k);
                        if (f.size() < pad) f.resize(pad, 0.f);
                        op.data = B.put(f.data(), f.size() * sizeof(float));
                    } else {
                        auto f = fragments<double>(M, k);
                        if (f.size() < pad) f.resize(pad, 0.0);
                        op.data = B.put(f.data(), f.size() * sizeof(double));
                    }
                }
                qvm_plan::Block blk;
                blk.qubits = bq;
                blk.k_true = k_true;
                for (int gi : u.gates) {
                    blk.gates.push_back(G[gi].src);
                    P->block_of_gate[G[gi].src] = (uint32_t)P->blocks.size();
                }
                blk.m = std::move(M);
                blk.pass = pi;
                P->blocks.push_back(std::move(blk));
            } else {
                // diagonal gate -> phase terms over its target patterns
                const PGate& g = G[u.gates[0]];
                held.push_back(&u);
                held_wires |= g.qmask;
                uint64_t tmask = 0;
                for (int r = 0; r < g.k; ++r) tmask |= 1ull << pos[g.t[r]];
                uint64_t pc = 0;
                for (int q = 0; q < n; ++q)
                    if ((g.cmask >> q) & 1) pc |= 1ull << pos[q];
                const int dim = 1 << g.k;
                for (int j = 0; j < dim; ++j) {
                    const cd v = g.u[(size_t)j * dim + j];
                    if (v == cd(1, 0)) continue;
                    uint64_t pv = pc;
                    for (int r = 0; r < g.k; ++r)
                        if ((j >> r) & 1) pv |= 1ull << pos[g.t[r]];
                    const uint64_t pm = pc | tmask;
                    DSub d{};
                    d.omask = pm & ~qmask;
                    d.oval = pv & ~qmask;
                    for (int i = 0; i < L; ++i) {
                        if ((pm >> phys[i]) & 1) d.lmask |= 1u << i;
                        if ((pv >> phys[i]) & 1) d.lval |= 1u << i;
                    }
                    d.neg = v == cd(-1, 0);
                    d.pr = v.real();
                    d.pi = v.imag();
                    d.turns = d.neg ? 1ull << 63 : turns_of(v);
                    {
                        const uint32_t hi = ~(uint32_t)(kTileThreads - 1);
                        const int nrow = L > 9 ? 1 << (L - 9) : 1;          // elements per thread
                        for (int i = 0; i < nrow; ++i)
                            if ((((uint32_t)kTileThreads * i) & d.lmask & hi) == (d.lval & hi)) d.rows |= 1u << i;
                    }
                    run.push_back(d);
                }
                P->n_diag_ops++;
                continue;
            }
            ops.push_back(op);
        }
        flush();
        // ---- wave bits.  In a pass whose blocks are all of 3 or 4 qubits
        // (register fragments), consecutive blocks that leave three tile bits
        // W untouched form an epoch: every block of it puts W on its wave
        // bits, so each wave owns the elements with one value of W throughout
        // and the blocks after the first need no workgroup barrier
        // (BLK_NOSYNC).  Standalone diagonal runs (their own layout) end an
        // epoch; epilogue runs ride with their block.
        std::vector<uint32_t> wsel(ops.size(), 0u);
        {
            int kmax_ops = 0;
            for (const TOp& o : ops)
                if (o.type == TOP_BLOCK) kmax_ops = std::max(kmax_ops, (int)o.k);
            if (kmax_ops <= 4) {
                const uint32_t tile_bits = (1u << L) - 1;
                std::vector<size_t> members;
                uint32_t allowed = 0;
                auto close = [&]() {
                    if (members.size() >= 2) {
                        uint32_t W = 0;
                        for (int b = L - 1, got = 0; b >= 0 && got < 3; --b)
                            if ((allowed >> b) & 1) {
                                W |= 1u << b;
                                ++got;
                            }
                        for (size_t i = 0; i < members.size(); ++i) {
                            wsel[members[i]] = W;
                            if (i) ops[members[i]].flags |= BLK_NOSYNC;
                        }
                    }
                    members.clear();
                    allowed = 0;
                };
                for (size_t oi = 0; oi < ops.size(); ++oi) {
                    const TOp& o = ops[oi];
                    if (o.type != TOP_BLOCK) {
                        if (!(o.flags & DRUN_EPILOGUE)) close();
                        continue;
                    }
                    if (!wave_bits_ok(o.k, L, dt)) {
                        close();
                        continue;
                    }
                    uint32_t bm = 0;
                    for (int r = 0; r < o.k; ++r) bm |= 1u << o.lb[r];
                    const uint32_t ok = tile_bits & ~bm;
                    if (!members.empty() && __builtin_popcount(allowed & ok) >= 3) {
                        allowed &= ok;
                        members.push_back(oi);
                    } else {
                        close();
                        members.push_back(oi);
                        allowed = ok;
                    }
                }
                close();
            }
        }
        // ---- block address tables and epilogue runs over the final layouts
        if (kmax_pass >= 5 && !epi_runs.empty())
            return fail_plan(QVM_EARG, "internal: epilogue run in a pass of 5- or 6-qubit blocks");
        PSumBuild ps;                          // phase runs in block epilogues
        std::vector<size_t> phase_ops;
        for (auto& er : epi_runs) {
            TOp& o = ops[er.first];
            const TOp& blk = ops[er.first - 1];
            int8_t bitmap[32];
            epilogue_bitmap(blk.lb, blk.k, col_map(blk.lb, blk.k, L, dt, wsel[er.first - 1]), bitmap);
            std::vector<DTerm> terms;
            std::vector<uint32_t> off;
            angle_terms(er.second, L, dt, bitmap, 4, terms, off);
            o.k = (int32_t)terms.size();
            if (o.flags & DRUN_SIGNS) {
                std::vector<ETerm> et;
                std::vector<uint32_t> eoff;
                epilogue_terms(terms, off, qmask, true, et, eoff);
                o.data = B.put(et.data(), et.size() * sizeof(ETerm));
                o.tab = B.put(eoff.data(), eoff.size() * sizeof(uint32_t));
            } else {
                std::vector<uint32_t> goff;
                epilogue_psums(terms, off, qmask, ps, goff);
                o.tab = B.put(goff.data(), goff.size() * sizeof(uint32_t));
                phase_ops.push_back(er.first);
            }
        }
        const bool epi_phases = !phase_ops.empty();
        size_t psum_off = 0;
        const uint32_t ncombo = (uint32_t)ps.masks.size();
        if (epi_phases) {
            if (ncombo > (uint32_t)kPSumMax || ncombo > (uint32_t)psum_combos)
                return fail_plan(QVM_EARG, "internal: phase sums above their bound");
            constexpr int NW = kTileThreads / 64;
            PSumHead h{};
            h.ncombo = ncombo;
            h.nrec = (uint32_t)ps.recs.size();
            h.rec_off = (uint32_t)((sizeof(PSumHead) + 4 * (ncombo + 1) + 15) & ~(size_t)15);
            h.mask_off = h.rec_off + (uint32_t)(sizeof(PRec) * ps.recs.size());
            std::vector<char> t(h.mask_off + sizeof(uint64_t) * NW * ncombo, 0);
            memcpy(t.data(), &h, sizeof h);
            memcpy(t.data() + sizeof h, ps.cb.data(), 4 * ps.cb.size());
            if (!ps.recs.empty()) memcpy(t.data() + h.rec_off, ps.recs.data(), sizeof(PRec) * ps.recs.size());
            uint64_t* m = (uint64_t*)(t.data() + h.mask_off);
            for (uint32_t c = 0; c < ncombo; ++c)
                for (int w = 0; w < NW; ++w) m[(size_t)w * ncombo + c] = ps.masks[c][w];
            psum_off = B.put(t.data(), t.size());
            for (size_t oi : phase_ops) ops[oi].data = psum_off;
        }
        PassDesc pd{};
        if (image && !ops.empty()) {
            // every op's table slot, by op index (zeros for diagonal runs)
            std::vector<uint32_t> tabs(ops.size() * kTabWords, 0u);
            for (size_t oi = 0; oi < ops.size(); ++oi) {
                if (ops[oi].type != TOP_BLOCK) continue;
                const TOp& o = ops[oi];
                const std::vector<uint32_t> tab = block_table(o.lb, o.k, L, dt, col_map(o.lb, o.k, L, dt, wsel[oi]));
                if (tab.size() > (size_t)kTabWords) return fail_plan(QVM_EARG, "internal: block table too long");
                std::copy(tab.begin(), tab.end(), tabs.begin() + oi * kTabWords);
            }
            pd.tabs = B.put(tabs.data(), tabs.size() * sizeof(uint32_t));
            for (size_t oi = 0; oi < ops.size(); ++oi)
                if (ops[oi].type == TOP_BLOCK) ops[oi].tab = pd.tabs + oi * kTabStride;
        }
        pd.L = L;
        pd.c = c;
        pd.nops = (int)ops.size();
        pd.kmax = 0;
        pd.first_block = -1;
        for (int oi = (int)ops.size() - 1; oi >= 0; --oi) {
            ops[oi].next_block = pd.first_block;
            ops[oi].next_data = pd.first_block >= 0 ? ops[pd.first_block].data : 0;
            if (ops[oi].type == TOP_BLOCK) {
                pd.first_block = oi;
                pd.kmax = std::max(pd.kmax, (int32_t)ops[oi].k);
            }
        }
        if (pd.kmax != (pd.first_block >= 0 ? kmax_pass : pd.kmax))
            return fail_plan(QVM_EARG, "internal: pass block width mismatch");
        pd.qmask = qmask;
        pd.ops = ops.empty() ? 0 : B.put(ops.data(), ops.size() * sizeof(TOp));
        if (epi_phases && image) {
            if (!cis_off) {
                std::vector<float> t(2 * kCisEntries);
                for (int j = 0; j < kCisEntries; ++j) {
                    t[2 * j] = (float)std::cos(2.0 * M_PI * j / kCisEntries);
                    t[2 * j + 1] = (float)std::sin(2.0 * M_PI * j / kCisEntries);
                }
                cis_off = B.put(t.data(), t.size() * sizeof(float));
            }
            pd.cistab = cis_off;
            pd.psum = psum_off;
            pd.npsum = (int32_t)ncombo;
        }
        std::vector<uint64_t> ldoff((size_t)1 << (L - c));
        for (size_t ch = 0; ch < ldoff.size(); ++ch) {
            uint64_t off = 0;
            for (int i = c; i < L; ++i)
                if ((ch >> (i - c)) & 1) off |= 1ull << phys[i];
            ldoff[ch] = off;
        }
        pd.ldoff = B.put(ldoff.data(), ldoff.size() * sizeof(uint64_t));
        // ---- remap: put the tile wires needed soonest on the low physical bits
        pd.remap = 0;
        const bool more = tile_mode ? left > 0 : next_unit < units.size();
        if (more && c > 0 && L > c) {
            std::vector<int> nextu(n, 1 << 30);
            if (tile_mode) {
                for (int gi = first; gi < ngw; ++gi)
                    if (!done[gi] && !G[gi].diag)
                        for (uint64_t m = G[gi].qmask; m; m &= m - 1) {
                            int q = __builtin_ctzll(m);
                            if (nextu[q] > gi) nextu[q] = gi;
                        }
            } else {
                for (size_t ui = next_unit; ui < units.size(); ++ui)
                    if (units[ui].block)
                        for (int q : units[ui].qubits)
                            if (nextu[q] > (int)ui) nextu[q] = (int)ui;
            }
            std::vector<int> tw(L);
            for (int i = 0; i < L; ++i) tw[i] = at[phys[i]];
            std::vector<int> want = tw;
            std::stable_sort(want.begin(), want.end(), [&](int a, int b) { return nextu[a] < nextu[b]; });
            want.resize(c);
            auto wanted = [&](int w) { return std::find(want.begin(), want.end(), w) != want.end(); };
            std::vector<int> newat(L, -1);          // destination slot -> wire
            std::vector<char> placed(n, 0);
            for (int i = 0; i < c; ++i)
                if (wanted(tw[i])) {
                    newat[i] = tw[i];
                    placed[tw[i]] = 1;
                }
            for (int w : want)
                if (!placed[w])
                    for (int i = 0; i < c; ++i)
                        if (newat[i] < 0) {
                            newat[i] = w;
                            placed[w] = 1;
                            break;
                        }
            for (int i = c; i < L; ++i)
                if (!placed[tw[i]]) {
                    newat[i] = tw[i];
                    placed[tw[i]] = 1;
                }
            for (int i = 0; i < c; ++i)
                if (!placed[tw[i]])
                    for (int j = c; j < L; ++j)
                        if (newat[j] < 0) {
                            newat[j] = tw[i];
                            placed[tw[i]] = 1;
                            break;
                        }
            bool ident = true;
            for (int i = 0; i < L; ++i)
                if (newat[i] != tw[i]) ident = false;
            if (!ident) {
                // destination slot d receives wire newat[d], found at local
                // slot src[d] of the loaded tile
                std::vector<int> src(L);
                for (int d = 0; d < L; ++d) src[d] = local_of_wire[newat[d]];
                std::vector<uint32_t> hi((size_t)1 << (L - c)), lo((size_t)1 << c);
                // entries are LDS slots of the source elements (the swizzle
                // is linear, so the slot of hi | lo is the XOR of the two)
                for (size_t v = 0; v < hi.size(); ++v) {
                    uint32_t e = 0;
                    for (int d = c; d < L; ++d)
                        if ((v >> (d - c)) & 1) e |= 1u << src[d];
                    hi[v] = tile_swizzle(e);
                }
                for (size_t v = 0; v < lo.size(); ++v) {
                    uint32_t e = 0;
                    for (int d = 0; d < c; ++d)
                        if ((v >> d) & 1) e |= 1u << src[d];
                    lo[v] = tile_swizzle(e);
                }
                pd.remap = 1;
                pd.rmhi = B.put(hi.data(), hi.size() * sizeof(uint32_t));
                pd.rmlo = B.put(lo.data(), lo.size() * sizeof(uint32_t));
                for (int d = 0; d < L; ++d) {
                    pos[newat[d]] = phys[d];
                    at[phys[d]] = newat[d];
                }
            }
        }
        double fl = 0;
        for (const TOp& o : ops)
            if (o.type == TOP_BLOCK) fl += 8.0 * (double)(1 << o.k) * (double)(1ull << n);
        P->pass_flops.push_back(fl);
        {
            // features of the pass for the cost model (layout in qvm.h)
            float f[QVM_PASS_FEATURES] = {};
            f[0] = (float)n;
            f[1] = dt == QVM_C64 ? 0.f : 1.f;
            f[2] = (float)L;
            int nb = 0, nlow = 0, ktrue = 0, ngates = 0, nruns = 0, nterms = 0;
            double pos_sum = 0, pos_min = 64, pos_max = -1, work = 0;
            for (const TOp& o : ops) {
                if (o.type == TOP_BLOCK) {
                    f[3 + (o.k - 3)] += 1.f;
                    work += (double)(1 << o.k);
                    ++nb;
                    for (int r = 0; r < o.k; ++r) {
                        const double ph = phys[o.lb[r]];
                        pos_sum += ph;
                        pos_min = std::min(pos_min, ph);
                        pos_max = std::max(pos_max, ph);
                        if (ph < c) ++nlow;
                    }
                } else {
                    ++nruns;
                    nterms += o.k;
                    if (o.flags & DRUN_TURNS) {
                        f[20] += 1.f;
                        f[21] += (float)o.k;
                    }
                }
            }
            for (auto& u : pp.units) {
                ngates += (int)u.gates.size();
                if (u.block) ktrue += (int)u.qubits.size();
            }
            int high = 0;
            for (int i = 0; i < L; ++i)
                if (phys[i] >= 20) ++high;
            f[7] = (float)work;
            f[8] = (float)nruns;
            f[9] = (float)nterms;
            f[10] = (float)ngates;
            f[11] = pd.remap ? 1.f : 0.f;
            f[12] = (float)high;
            f[13] = nb ? (float)(pos_sum / std::max(1, [&] { int t = 0; for (const TOp& o : ops) if (o.type == TOP_BLOCK) t += o.k; return t; }())) : 0.f;
            f[14] = nb ? (float)pos_min : (float)n;
            f[15] = nb ? (float)pos_max : 0.f;
            f[16] = (float)nlow;
            f[17] = (float)ktrue;
            f[18] = (float)(n + (dt == QVM_C64 ? 3 : 4));     // log2 of state bytes
            f[19] = (float)(n - L);                           // log2 of the tile count
            {
                // workgroup barriers between the pass's ops (tile.hip):
                // register-fragment passes skip them before BLK_NOSYNC
                // blocks; passes with wider blocks take one after every op
                // and one more per staged block fragment
                int bars = 0, execd = 0;
                for (const TOp& o : ops) {
                    if (o.type != TOP_BLOCK && (o.flags & DRUN_EPILOGUE)) continue;
                    if (pd.kmax <= 4) {
                        if (execd && !(o.type == TOP_BLOCK && (o.flags & BLK_NOSYNC))) ++bars;
                    } else {
                        bars += o.type == TOP_BLOCK ? 2 : 1;
                    }
                    ++execd;
                }
                f[22] = (float)bars;
            }
            P->pass_features.insert(P->pass_features.end(), f, f + QVM_PASS_FEATURES);
        }
        P->passes.push_back(pd);
    }
    P->final_perm.resize(n);
    for (int l = 0; l < n; ++l) P->final_perm[l] = pos[wire[l]];
    P->pass_table = P->passes.empty() ? 0 : B.put(P->passes.data(), P->passes.size() * sizeof(PassDesc));
    *out = P;
    return QVM_OK;
}

qvm_status run_plan(qvm_sv* sv, const qvm_plan* P) {
    for (int q = 0; q < sv->n; ++q)
        if (sv->perm[q] != q) return fail(QVM_ESTATE, "run_plan needs the identity layout; call qvm_reset_layout");
    if (P->blob.size() > sv->lay.plan_bytes) return fail(QVM_ENOMEM, "plan data exceeds the workspace plan area");
    char* dblob = sv->work + sv->lay.plan_off;
    if (!P->blob.empty())
        QVM_HIP(sv, hipMemcpyAsync(dblob, P->blob.data(), P->blob.size(), hipMemcpyHostToDevice, sv->stream));
    for (size_t i = 0; i < P->passes.size(); ++i) {
        qvm_status st = launch_tile_pass(sv, P->passes[i], dblob, P->pass_flops[i]);
        if (st) return st;
    }
    for (int q = 0; q < sv->n; ++q) sv->perm[q] = P->final_perm[q];
    return QVM_OK;
}

}  // namespace qvm

using namespace qvm;

extern "C" {

qvm_status qvm_plan_greedy(const qvm_gate* gates, size_t n_gates, int n_qubits, int k_max,
                           int tile_qubits, qvm_dtype dt, qvm_plan** out) {
    return build_plan(gates, n_gates, n_qubits, dt, k_max, tile_qubits, nullptr, out, true);
}

qvm_status qvm_plan_greedy_ex(const qvm_gate* gates, size_t n_gates, int n_qubits, int k_max,
                              int tile_qubits, qvm_dtype dt, uint32_t flags, qvm_plan** out) {
    if (flags & ~(uint32_t)(QVM_PLAN_NO_IMAGE | QVM_PLAN_DEFER_NARROW)) return fail(QVM_EARG, "unknown plan flags");
    return build_plan(gates, n_gates, n_qubits, dt, k_max, tile_qubits, nullptr, out,
                      (flags & QVM_PLAN_NO_IMAGE) == 0, nullptr, 0, (flags & QVM_PLAN_DEFER_NARROW) != 0);
}

qvm_status qvm_plan_tile_per_pass(const qvm_gate* gates, size_t n_gates, int n_qubits, int tile_qubits,
                                  const int32_t* k_of_pass, int32_t n_k, qvm_dtype dt, uint32_t flags,
                                  qvm_plan** out) {
    if (flags & ~(uint32_t)QVM_PLAN_NO_IMAGE) return fail(QVM_EARG, "unknown plan flags");
    if (n_k < 1 || !k_of_pass) return fail(QVM_EARG, "empty per-pass block widths");
    if (tile_qubits == 0) return fail(QVM_EARG, "per-pass block widths need tile passes (tile_qubits > 0)");
    int kmax = 0, kmin = 7;
    for (int i = 0; i < n_k; ++i) {
        kmax = std::max(kmax, (int)k_of_pass[i]);
        kmin = std::min(kmin, (int)k_of_pass[i]);
    }
    if (kmin < 1 || kmax > 6) return fail(QVM_EARG, "per-pass block width outside 1..6");
    // the tile must hold the widest block (and, in complex128, its fragments)
    const int Lmax = dt == QVM_C64 ? 13 : (kmax >= 6 ? 11 : 12);
    if (tile_qubits < std::min(kmax, n_qubits) || tile_qubits > Lmax)
        return fail(QVM_EARG, "tile_qubits must lie in [widest per-pass block width, 13] (complex64) / "
                              "[.., 12] (complex128, 11 with a 6-qubit width)");
    // validation (gate spans, tile width) against the narrowest width used
    return build_plan(gates, n_gates, n_qubits, dt, kmin, tile_qubits, nullptr, out,
                      (flags & QVM_PLAN_NO_IMAGE) == 0, k_of_pass, n_k);
}

qvm_status qvm_plan_from_partition(const qvm_gate* gates, size_t n_gates, const uint32_t* block_of_gate,
                                   int n_qubits, int k_max, qvm_dtype dt, qvm_plan** out) {
    if (n_gates && !block_of_gate) return fail(QVM_EARG, "NULL partition");
    return build_plan(gates, n_gates, n_qubits, dt, k_max, 0, block_of_gate, out, true);
}

qvm_status qvm_plan_pass_features(const qvm_plan* p, float* out, size_t cap, int32_t* n_passes) {
    if (!p) return fail(QVM_EARG, "NULL plan");
    if (n_passes) *n_passes = (int32_t)p->passes.size();
    if (out) {
        if (cap < p->pass_features.size()) return fail(QVM_ENOMEM, "feature buffer too small");
        memcpy(out, p->pass_features.data(), p->pass_features.size() * sizeof(float));
    }
    return QVM_OK;
}

qvm_status qvm_plan_image(const qvm_plan* p, void* out, size_t cap, size_t* bytes,
                          uint64_t* pass_table, int32_t* n_passes) {
    if (!p) return fail(QVM_EARG, "NULL plan");
    if (bytes) *bytes = p->blob.size();
    if (pass_table) *pass_table = p->pass_table;
    if (n_passes) *n_passes = (int32_t)p->passes.size();
    if (out) {
        if (cap < p->blob.size()) return fail(QVM_ENOMEM, "buffer too small for the plan image");
        memcpy(out, p->blob.data(), p->blob.size());
    }
    return QVM_OK;
}

qvm_status qvm_plan_destroy(qvm_plan* p) {
    delete p;
    return QVM_OK;
}

qvm_status qvm_plan_info(const qvm_plan* p, qvm_plan_stats* s) {
    if (!p || !s) return fail(QVM_EARG, "NULL argument");
    memset(s, 0, sizeof(*s));
    s->n_passes = (int32_t)p->passes.size();
    s->n_blocks = (int32_t)p->blocks.size();
    s->n_diag_ops = p->n_diag_ops;
    for (auto& b : p->blocks) s->blocks_by_k[b.k_true]++;
    s->tile_qubits = p->passes.empty() ? 0 : p->passes[0].L;
    s->device_bytes = p->blob.size();
    return QVM_OK;
}

qvm_status qvm_plan_block(const qvm_plan* p, int32_t i, int32_t* k, int32_t* k_true, int32_t* qubits,
                          int32_t* n_gates, int32_t* gate_idx, int32_t* pass, double* m_out) {
    if (!p) return fail(QVM_EARG, "NULL plan");
    if (i < 0 || i >= (int)p->blocks.size()) return fail(QVM_ERANGE, "block index out of range");
    const auto& b = p->blocks[i];
    if (k) *k = (int32_t)b.qubits.size();
    if (k_true) *k_true = b.k_true;
    if (qubits)
        for (size_t r = 0; r < b.qubits.size(); ++r) qubits[r] = b.qubits[r];
    if (n_gates) *n_gates = (int32_t)b.gates.size();
    if (gate_idx)
        for (size_t r = 0; r < b.gates.size(); ++r) gate_idx[r] = b.gates[r];
    if (pass) *pass = b.pass;
    if (m_out && !p->image) return fail(QVM_ESTATE, "plan was built for scoring only (QVM_PLAN_NO_IMAGE)");
    if (m_out)
        for (size_t r = 0; r < b.m.size(); ++r) {
            m_out[2 * r] = b.m[r].real();
            m_out[2 * r + 1] = b.m[r].imag();
        }
    return QVM_OK;
}

qvm_status qvm_plan_schedule(const qvm_plan* p, int32_t* exec_pos, int32_t* unit_of) {
    if (!p) return fail(QVM_EARG, "NULL plan");
    for (size_t i = 0; i < p->exec_pos.size(); ++i) {
        if (exec_pos) exec_pos[i] = p->exec_pos[i];
        if (unit_of) unit_of[i] = p->unit_of[i];
    }
    return QVM_OK;
}

qvm_status qvm_plan_final_layout(const qvm_plan* p, int32_t* perm_out) {
    if (!p || !perm_out) return fail(QVM_EARG, "NULL argument");
    for (int q = 0; q < p->n; ++q) perm_out[q] = p->final_perm[q];
    return QVM_OK;
}

qvm_status qvm_run_plan(qvm_sv* sv, const qvm_plan* p) {
    if (!sv || !p) return fail(QVM_EARG, "NULL argument");
    if (sv->failed) return fail(QVM_ESTATE, "state handle failed earlier");
    if (!p->image) return fail(QVM_ESTATE, "plan was built for scoring only (QVM_PLAN_NO_IMAGE)");
    if (p->n != sv->n || p->dt != sv->dt) return fail(QVM_EARG, "plan built for another n or dtype");
    return run_plan(sv, p);
}

}  // extern "C"
