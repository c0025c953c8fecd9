// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <complex>
#include <cstdint>
#include <string>
#include <vector>

#include "qvm.h"

namespace qvm {

using cd = std::complex<double>;

// ------------------------------------------------------------------ errors
void set_error(const std::string& msg);
qvm_status fail(qvm_status st, const std::string& msg);

// ---------------------------------------------------------- workspace map
// Fixed layout of the caller-provided device workspace.
struct WorkLayout {
    size_t red_off, red_bytes;        // reduction partials + results (doubles)
    size_t chunk_off, chunk_bytes;    // sampling chunk sums + prefix (doubles)
    size_t io_off, io_bytes;          // staging for host <-> device small arrays
    size_t plan_off, plan_bytes;      // plan data (matrices, op tables)
    size_t total;
    int chunk_log;                    // log2 of the sampling chunk length
};
WorkLayout work_layout(int n, qvm_dtype dt);

constexpr int kRedBlocks = 2048;      // fixed grid of reduction kernels
constexpr int kRedSlots = 64;         // doubles per block in the partials table

// Per-launch timing with HIP events (enabled by qvm_profile_begin).
enum ProfKind { PK_DENSE1 = 0, PK_DENSE2, PK_DENSE3, PK_DIAG, PK_PHASE, PK_SWAP, PK_TILE,
                PK_BASIS, PK_RDM1, PK_COUNT };
struct ProfRec {
    int kind;
    int ev;                           // index of the start event; end = ev + 1
    double bytes, flops;              // algorithmic bytes and flops of the launch
};
struct Prof {
    bool on = false;
    std::vector<hipEvent_t> events;   // pool, grows on demand
    std::vector<ProfRec> recs;
    std::vector<double> last_ms;      // per-launch durations of the last interval
    std::vector<int> last_kind;
};

}  // namespace qvm

struct qvm_sv {
    int n;
    qvm_dtype dt;
    void* amps;
    char* work;
    size_t work_bytes;
    hipStream_t stream;
    int perm[QVM_MAX_QUBITS];         // logical -> physical bit
    bool failed;
    qvm::WorkLayout lay;
    qvm::Prof prof;
};

namespace qvm {

// Record a HIP error on the handle (sticky) and return QVM_EDEVICE.
qvm_status device_fail(qvm_sv* sv, hipError_t e, const char* where);
#define QVM_HIP(sv, expr)                                            \
    do {                                                             \
        hipError_t _e = (expr);                                      \
        if (_e != hipSuccess) return ::qvm::device_fail(sv, _e, #expr); \
    } while (0)
#define QVM_LAUNCH_CHECK(sv) QVM_HIP(sv, hipGetLastError())

// Bracket a launch: prof_begin returns a token (-1 when profiling is off).
int prof_begin(qvm_sv* sv);
void prof_end(qvm_sv* sv, int token, int kind, double bytes, double flops);

// Logical mask -> physical mask through the handle's layout.
uint64_t phys_mask(const qvm_sv* sv, uint64_t logical_mask);
// Physical index of a logical index, and back.
uint64_t phys_index(const qvm_sv* sv, uint64_t logical);

// --------------------------------------------------------------- lowering
// A gate after validation and lowering, on physical qubits.
enum OpClass { OP_DENSE = 0, OP_DIAG = 1, OP_PHASE = 2, OP_SWAPPAIR = 3 };
struct LOp {
    OpClass cls;
    int k;
    int t[QVM_MAX_K];                 // physical targets, bit r of matrix <-> t[r]
    uint64_t cmask;                   // physical control mask
    std::vector<cd> m;                // dense: 2^k x 2^k row-major; diag: 2^k
    uint64_t cond_mask, cond_val;     // OP_PHASE / OP_SWAPPAIR index condition
    uint64_t xmask;                   // OP_SWAPPAIR partner = i ^ xmask
    uint64_t hbit;                    // OP_SWAPPAIR: bit of xmask that is 0 in i
    cd phase;                         // OP_PHASE factor
};

// Validate a gate against n qubits (logical).  Returns QVM_OK or an error
// with the message set.
qvm_status validate_gate(const qvm_gate& g, int n, bool allow_k_gt3);
// Full target matrix of a validated gate (FP64, host libm).
qvm_status gate_matrix(const qvm_gate& g, std::vector<cd>& u);
// Lower a validated gate onto the physical layout and classify it.
LOp lower(const qvm_sv* sv, const qvm_gate& g, const std::vector<cd>& u);
// Same, given physical targets directly.
LOp classify(int k, const int* phys_t, uint64_t phys_cmask, const std::vector<cd>& u);

// ----------------------------------------------------- plain-path launchers
qvm_status launch_op(qvm_sv* sv, const LOp& op);
qvm_status launch_init_basis(qvm_sv* sv, uint64_t phys_index);
qvm_status launch_swap_bits(qvm_sv* sv, int a, int b);   // physical bit swap

// ------------------------------------------------------- readout launchers
qvm_status rd_norm(qvm_sv* sv, double* out);
qvm_status rd_scale(qvm_sv* sv, double factor);
qvm_status rd_z_all(qvm_sv* sv, double* out_phys_total, double* out_phys_bit);
// out = {sum |psi_i|^2 over physical bit pbit = 0, the same over bit = 1,
//        Re and Im of sum psi_i conj(psi_{i | 2^pbit})}, FP64; synchronizes
qvm_status rd_rdm1(qvm_sv* sv, int pbit, double* out);
qvm_status rd_pauli_group(qvm_sv* sv, uint64_t x_phys, int nt, const uint64_t* z_phys,
                          double* out);
qvm_status rd_probs_full(qvm_sv* sv, double* out_host);
qvm_status rd_marginal(qvm_sv* sv, int m, const int* phys_q, double* out_host);
qvm_status rd_sample(qvm_sv* sv, size_t ns, const double* u, uint64_t* out_logical);
qvm_status rd_copy(qvm_sv* sv, uint64_t first, uint64_t count, double* out_host);
qvm_status rd_gather(qvm_sv* sv, size_t count, const uint64_t* logical, double* out_host);

}  // namespace qvm
