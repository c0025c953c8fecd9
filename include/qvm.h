/*
 * qvm.h -- C ABI of the MI355X (gfx950) full-amplitude state-vector library.
 *
 * The method: a quantum program is a sequence of gates, each a 2^k x 2^k
 * unitary on k target qubits with optional control qubits, applied as a
 * linear map to the 2^n complex amplitudes of the state (paper, "Multi-
 * simulation methods", noise-free Schroedinger simulation, full-amplitude
 * backend).  The calls follow the paper's user-facing operations: allocate
 * n qubits (init_qvm / qAlloc_many), apply gates with targets and controls
 * (the gate set and .control() of "Structure of QPanda" and "A variety of
 * convenient tools"), fuse gates into unitary blocks (Fusion /
 * aggregate_operations, "Quantum circuit fusion"), and read out
 * probabilities (prob_run_*), expectation values and measurement samples
 * ("A variety of convenient tools").
 *
 * Conventions (the paper fixes none of them):
 *   - qubit q is bit q of the amplitude index (qubit 0 least significant);
 *   - amplitudes are interleaved (re, im): QVM_C64 = 2 x float (8 bytes),
 *     QVM_C128 = 2 x double (16 bytes);
 *   - a k-qubit matrix is row-major 2^k x 2^k complex given as (re, im)
 *     double pairs, and bit r of its row/column index refers to targets[r];
 *   - controls are 1-controls, given as a bit mask over qubits;
 *   - bit strings returned by sampling are amplitude indices in the logical
 *     qubit order above.
 *
 * Ownership: device buffers (amplitudes, workspace) belong to the caller,
 * who keeps them alive until qvm_sv_destroy.  Host arrays passed in are
 * read during the call only.  The library owns only its opaque handles.
 *
 * Streams: every call enqueues on the stream given at creation (a
 * hipStream_t passed as void*; NULL = the null stream).  Calls that return
 * host values synchronise that stream; all others are asynchronous.
 *
 * Errors: every call returns a qvm_status.  Arguments are validated before
 * anything is enqueued (QVM_EARG / QVM_ERANGE).  A HIP error returns
 * QVM_EDEVICE and marks the handle failed; later calls on it return
 * QVM_ESTATE.  qvm_last_error() gives the calling thread's last message.
 * No C++ exception crosses this interface.
 */
#ifndef QVM_H
#define QVM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    QVM_OK = 0,
    QVM_EARG = -1,          /* malformed argument (NULL, duplicate qubit, k out of range) */
    QVM_ERANGE = -2,        /* qubit >= n, basis index >= 2^n, index out of range */
    QVM_ENOMEM = -3,        /* workspace too small, host allocation failed */
    QVM_EDEVICE = -4,       /* HIP runtime or launch error */
    QVM_ESTATE = -5,        /* handle failed earlier, or is in the wrong state */
    QVM_EUNSUPPORTED = -6   /* valid request the library does not implement */
} qvm_status;

typedef enum { QVM_C64 = 1, QVM_C128 = 2 } qvm_dtype;

#define QVM_MAX_QUBITS 34
#define QVM_MAX_K 6

/* Named gates (paper's gate set).  One-target kinds take targets[0]; RZZ and
 * SWAP take two targets; QVM_G_MATRIX takes k targets and the matrix u.
 * Angles in params: RX/RY/RZ/P/RZZ use params[0]; U3 uses (theta, phi,
 * lambda) in the OpenQASM 2 form.  CNOT = X with one control, CZ = Z with one
 * control, CR = P with one control, Toffoli = X with two controls. */
typedef enum {
    QVM_G_MATRIX = 0,
    QVM_G_I = 1, QVM_G_H = 2, QVM_G_X = 3, QVM_G_Y = 4, QVM_G_Z = 5,
    QVM_G_S = 6, QVM_G_SDG = 7, QVM_G_T = 8, QVM_G_TDG = 9,
    QVM_G_RX = 10, QVM_G_RY = 11, QVM_G_RZ = 12, QVM_G_P = 13, QVM_G_U3 = 14,
    QVM_G_RZZ = 15, QVM_G_SWAP = 16
} qvm_gate_kind;

/* One gate.  72 bytes, no padding surprises: int32 x 8, uint64, double x 3,
 * pointer.  `u` is read only for QVM_G_MATRIX (2^k x 2^k, (re, im) doubles,
 * row-major) and must be NULL otherwise. */
typedef struct qvm_gate {
    int32_t kind;
    int32_t k;
    int32_t targets[QVM_MAX_K];
    uint64_t ctrl_mask;
    double params[3];
    const double* u;
} qvm_gate;

typedef struct qvm_sv qvm_sv;       /* a state vector bound to caller memory */

/* ---------------------------------------------------------------- lowering */

/* Gate lowering: writes the gate's 2^k x 2^k target matrix (controls not
 * included) as (re, im) doubles into u_out (room for 2^(2k) complex).
 * Angles are evaluated on the host in double precision.  Host-only; needs no
 * GPU.  QVM_EARG for an unknown kind or a k that does not match the kind. */
qvm_status qvm_gate_matrix(const qvm_gate* g, double* u_out);

/* ------------------------------------------------------------ state vector */

/* Bytes of device workspace a state of n qubits needs (reduction partials,
 * sampling tables, plan data).  Host-only. */
size_t qvm_workspace_bytes(int n_qubits, qvm_dtype dt);

/* Bind a state of n qubits (1..QVM_MAX_QUBITS) to caller memory: amps_dev
 * holds 2^n amplitudes of dtype dt (256-byte aligned), work_dev at least
 * qvm_workspace_bytes(n, dt) bytes.  hip_stream may be NULL.  The amplitudes
 * are not initialised; call qvm_init_basis.  The logical-to-physical qubit
 * layout starts as the identity. */
qvm_status qvm_sv_create(int n_qubits, qvm_dtype dt, void* amps_dev,
                         void* work_dev, size_t work_bytes, void* hip_stream,
                         qvm_sv** out);

/* Release the handle.  Never frees caller buffers.  Accepts NULL. */
qvm_status qvm_sv_destroy(qvm_sv* sv);

/* Replace the stream later calls enqueue on. */
qvm_status qvm_sv_set_stream(qvm_sv* sv, void* hip_stream);

/* Set the state to the basis state |index> (0 = |0..0>) and reset the qubit
 * layout to the identity.  QVM_ERANGE if index >= 2^n.  Asynchronous. */
qvm_status qvm_init_basis(qvm_sv* sv, uint64_t index);

/* Apply one gate (plain per-gate path: one pass over the state).  k <= 3 for
 * dense matrices; any number of controls.  Asynchronous. */
qvm_status qvm_apply(qvm_sv* sv, const qvm_gate* g);

/* Kraus operators of the paper's single-qubit noise channels ("Noise
 * simulation method"), lowered on the host in double precision:
 *   QVM_K_DAMPING         [[1, 0], [0, sqrt(1-p)]], [[0, sqrt(p)], [0, 0]]
 *   QVM_K_DEPHASING       sqrt(1-p) I, sqrt(p) Z (also the phase flip)
 *   QVM_K_DECOHERENCE     K_a(damping, p1) K_b(dephasing, p2), a, b in {1, 2}
 *                         (4 operators, a-major), p1 = 1 - exp(-tgate/T1),
 *                         p2 = (1 - exp(-(tgate/T2 - tgate/(2 T1)))) / 2
 *   QVM_K_DEPOLARIZING    sqrt(1 - 3p/4) I, sqrt(p)/2 X, sqrt(p)/2 Y, sqrt(p)/2 Z
 *   QVM_K_BIT_PHASE_FLIP  sqrt(1-p) I, sqrt(p) Y (the printed "bit or phase
 *                         flip" operator is sqrt(p) Y)
 *   QVM_K_BIT_FLIP        sqrt(1-p) I, sqrt(p) X
 *   QVM_K_PHASE_DAMPING   [[1, 0], [0, sqrt(1-p)]], [[0, 0], [0, sqrt(p)]]
 * Writes *n_ops operators to ops_out (room for QVM_MAX_KRAUS) in the layout
 * qvm_apply_kraus reads.  p is used by every kind except decoherence, which
 * uses t1, t2 and tgate.  QVM_ERANGE: p outside [0, 1]; QVM_EARG: unknown
 * kind, NULL outputs, or decoherence without T1 > 0, T2 > 0, tgate >= 0 and
 * T2 <= 2 T1 (a negative dephasing rate).  Host-only. */
typedef enum {
    QVM_K_DAMPING = 0, QVM_K_DEPHASING = 1, QVM_K_DECOHERENCE = 2, QVM_K_DEPOLARIZING = 3,
    QVM_K_BIT_PHASE_FLIP = 4, QVM_K_BIT_FLIP = 5, QVM_K_PHASE_DAMPING = 6
} qvm_channel;
qvm_status qvm_kraus_ops(qvm_channel kind, double p, double t1, double t2, double tgate,
                         double* ops_out, int32_t* n_ops);

/* One single-qubit Kraus channel by the trajectory method (paper, "Noise
 * simulation method": noise models given as Kraus operators K_1..K_m; a noisy
 * run unravels each channel into one randomly drawn branch).  ops holds
 * n_ops (1..16) 2x2 complex matrices as (re, im) doubles, row-major, 8 per
 * operator (host memory, read during the call).  The branch weights
 * p_i = ||K_i psi||^2 = Tr(K_i^dag K_i rho_q) come from the qubit's reduced
 * density matrix rho_q, accumulated in FP64 in one pass over the state; the
 * branch j is the smallest with p_1 + ... + p_j > u (p_1 + ... + p_m), and
 * psi <- K_j psi sqrt((p_1 + ... + p_m) / p_j), which keeps the state's norm.
 * u is the caller's uniform in [0, 1).  chosen (nullable) receives j
 * (0-based); probs (nullable, n_ops doubles) receives p_i / sum.  Operators
 * need not be unitary or complete (the weights are normalised by their sum).
 * Synchronizes the stream.  QVM_ERANGE: qubit >= n; QVM_EARG: n_ops outside
 * 1..16, NULL ops, u outside [0, 1), or every weight zero. */
#define QVM_MAX_KRAUS 16
qvm_status qvm_apply_kraus(qvm_sv* sv, int32_t qubit, int32_t n_ops, const double* ops, double u,
                           int32_t* chosen, double* probs);

/* Apply a gate list in order with the plain per-gate path, in one call (the
 * per-gate call overhead the paper measures at small n is paid once).
 * The list is validated in full before anything is enqueued. */
qvm_status qvm_run(qvm_sv* sv, const qvm_gate* gates, size_t n_gates);

/* Current logical-to-physical qubit layout: perm_out[q] = physical bit of
 * logical qubit q (n entries).  Host-only. */
qvm_status qvm_get_layout(const qvm_sv* sv, int32_t* perm_out);

/* Physically permute the amplitudes back to the identity layout (one pass
 * per displaced qubit pair).  Asynchronous. */
qvm_status qvm_reset_layout(qvm_sv* sv);

/* -------------------------------------------------------------- readout */

/* Probabilities |psi_i|^2 in double precision (single-precision states are
 * widened before squaring).  m = n and qubits = NULL gives all 2^n values
 * in logical index order; otherwise the marginal over qubits[0..m-1], with
 * bit r of the output index <-> qubits[r].  out_host holds 2^m doubles.
 * m <= 24 for marginals.  Synchronous. */
qvm_status qvm_probabilities(qvm_sv* sv, int m, const int32_t* qubits,
                             double* out_host);

/* <Z_q> for every logical qubit in one pass over the state, double-precision
 * accumulation.  out_host holds n doubles.  Synchronous. */
qvm_status qvm_expect_z_all(qvm_sv* sv, double* out_host);

/* Pauli-string expectations <psi|P_t|psi> for strings in symplectic form
 * (x_mask: qubits carrying X or Y; z_mask: qubits carrying Z or Y; over
 * logical qubits).  Terms sharing an x_mask share one pass.  out_terms_host
 * (n_terms doubles, nullable) receives each term without its coefficient;
 * out_sum_host (nullable) receives sum_t coeff[t] <P_t>; coeff may be NULL
 * when out_sum_host is NULL.  Double-precision accumulation.  Synchronous. */
qvm_status qvm_expect_pauli(qvm_sv* sv, size_t n_terms, const uint64_t* x_mask,
                            const uint64_t* z_mask, const double* coeff,
                            double* out_terms_host, double* out_sum_host);

/* Draw samples: for each uniform u in [0,1), the smallest logical index i
 * with C_i > u * C_{N-1}, where C is the cumulative probability in logical
 * index order accumulated in double precision (the total absorbs norm
 * drift).  Synchronous. */
qvm_status qvm_sample(qvm_sv* sv, size_t n_samples, const double* uniforms_host,
                      uint64_t* out_host);

/* Squared norm sum_i |psi_i|^2 in double precision.  Synchronous. */
qvm_status qvm_norm(qvm_sv* sv, double* out);

/* Scale the state to unit norm (norm computed in double precision).
 * norm_before (nullable) receives the squared norm before scaling.
 * QVM_ESTATE if the norm is zero or not finite.  Synchronous. */
qvm_status qvm_renormalize(qvm_sv* sv, double* norm_before);

/* Copy amplitudes [first, first+count) in logical index order to the host as
 * (re, im) doubles.  Synchronous. */
qvm_status qvm_copy_amplitudes(qvm_sv* sv, uint64_t first, uint64_t count,
                               double* out_host);

/* Copy the amplitudes at the given logical indices to the host as (re, im)
 * doubles.  Synchronous. */
qvm_status qvm_gather_amplitudes(qvm_sv* sv, size_t count,
                                 const uint64_t* logical_idx, double* out_host);

/* --------------------------------------------------------- fused plans */

/* A fused execution plan (paper, "Quantum circuit fusion": Fusion /
 * aggregate_operations rewrites a program into unitary blocks before it is
 * simulated; the paper leaves the algorithm open).  A plan is a list of
 * passes.  Each pass streams every tile of 2^L amplitudes (L tile qubits,
 * always including the lowest physical bits) through LDS once and applies a
 * list of ops to it: fused k-qubit blocks (k = 3..6, blocks spanning fewer
 * qubits are padded) as complex GEMMs on MFMA, and phase/diagonal gates.
 * Controls of fused gates are folded into the block matrices; uncontrolled
 * SWAPs become qubit relabelings.  Block matrices are built on the host in
 * double precision and rounded to the state's dtype.  Plans are host
 * objects; building one needs no GPU. */
typedef struct qvm_plan qvm_plan;

typedef struct qvm_plan_stats {
    int32_t n_passes;        /* HBM round trips */
    int32_t n_blocks;        /* fused blocks */
    int32_t n_diag_ops;      /* standalone phase/diagonal ops */
    int32_t tile_qubits;     /* L of the passes */
    int32_t blocks_by_k[8];  /* blocks by the number of qubits their gates span */
    uint64_t device_bytes;   /* size of the plan's device image */
} qvm_plan_stats;

/* Greedy planner.  k_max (1..6) bounds the qubits a fused block spans.
 * tile_qubits = 0: every block gets its own pass ("one fused block per HBM
 * pass"); otherwise tile_qubits in [k_max, 13] (complex64) or [k_max, 12]
 * (complex128) and passes hold as many blocks as the tile admits; a tile
 * narrower than the state must be wider than the low bits every tile holds
 * (4 for complex64, 3 for complex128).  Gate validation as in qvm_run
 * (k <= 6); a non-diagonal gate spanning more than k_max qubits is
 * QVM_EARG.  n_qubits >= 3 (QVM_EUNSUPPORTED below: blocks are padded to 3
 * qubits). */
qvm_status qvm_plan_greedy(const qvm_gate* gates, size_t n_gates, int n_qubits,
                           int k_max, int tile_qubits, qvm_dtype dt,
                           qvm_plan** out);

/* qvm_plan_greedy with options.  QVM_PLAN_NO_IMAGE builds the plan for
 * scoring only: schedule, statistics, blocks' qubits and gates and the pass
 * features are filled in, but no block matrices and no device image (the
 * expensive part), so qvm_run_plan and a block's matrix return QVM_ESTATE.
 * The learned planner scores candidates this way and builds only the chosen
 * one in full.  QVM_PLAN_DEFER_NARROW (tile passes, k_max >= 3): a block of
 * fewer than 3 qubits costs as much as a 3-qubit block, so when such a
 * block's gates are the last its pass takes on each of their wires they are
 * left to a later pass, where they join their successors' block (not in the
 * last pass, never every block of a pass).  Fewer blocks, sometimes more
 * passes: a choice for the learned planner (paper, "Quantum circuit
 * fusion": the fusion scheme is picked by the cost model).  QVM_EARG for
 * unknown flags. */
#define QVM_PLAN_NO_IMAGE 1u
#define QVM_PLAN_DEFER_NARROW 2u
qvm_status qvm_plan_greedy_ex(const qvm_gate* gates, size_t n_gates, int n_qubits,
                              int k_max, int tile_qubits, qvm_dtype dt, uint32_t flags,
                              qvm_plan** out);

/* Tile passes with a block width per pass.  In tile mode the gates a pass
 * takes depend only on the tile width (the block width only changes how
 * they are fused), so pass i of this plan holds the same gates as pass i of
 * qvm_plan_greedy at the same tile width with any k_max; here they are
 * fused into blocks of at most k_of_pass[i] qubits (passes beyond n_k use
 * k_of_pass[n_k - 1]).  The learned planner picks each pass's width from the
 * cost model's predictions of the candidate passes.  Validation as in
 * qvm_plan_greedy with k_max = the narrowest width given; tile_qubits must
 * hold the widest.  flags as in qvm_plan_greedy_ex. */
qvm_status qvm_plan_tile_per_pass(const qvm_gate* gates, size_t n_gates, int n_qubits,
                                  int tile_qubits, const int32_t* k_of_pass, int32_t n_k,
                                  qvm_dtype dt, uint32_t flags, qvm_plan** out);

/* Plan from an explicit partition: block_of_gate[i] is the block id of gate
 * i; blocks run in ascending id order, one pass each.  QVM_EARG if a block
 * spans more than k_max qubits or the partition breaks the per-qubit gate
 * order. */
qvm_status qvm_plan_from_partition(const qvm_gate* gates, size_t n_gates,
                                   const uint32_t* block_of_gate, int n_qubits,
                                   int k_max, qvm_dtype dt, qvm_plan** out);

qvm_status qvm_plan_info(const qvm_plan* plan, qvm_plan_stats* out);

/* Block i of the plan: k (after padding), k_true, its qubits (k entries;
 * wires, i.e. logical qubits when no relabeling SWAP precedes the block),
 * the input indices of its gates (n_gates entries), its pass and its
 * double-precision matrix (2^k x 2^k, (re, im), row-major; bit r <->
 * qubits[r]).  Any output pointer may be NULL. */
qvm_status qvm_plan_block(const qvm_plan* plan, int32_t i, int32_t* k,
                          int32_t* k_true, int32_t* qubits, int32_t* n_gates,
                          int32_t* gate_idx, int32_t* pass, double* m_out);

/* Execution order of the input gates: exec_pos[i] = rank of gate i in the
 * order the plan applies gates (within a block: the order its matrix
 * multiplies them), unit_of[i] = the unit (fused block or standalone
 * diagonal op, numbered in execution order) that applies it.  SWAPs turned
 * into relabelings get -1 in both.  n_gates entries each; either may be
 * NULL. */
qvm_status qvm_plan_schedule(const qvm_plan* plan, int32_t* exec_pos,
                             int32_t* unit_of);

/* Layout the state is left in by qvm_run_plan: perm_out[q] = physical bit
 * of logical qubit q (n entries). */
qvm_status qvm_plan_final_layout(const qvm_plan* plan, int32_t* perm_out);

/* Execute a plan on a state in the identity layout (QVM_ESTATE otherwise;
 * see qvm_reset_layout).  Uploads the plan image into the workspace, then
 * enqueues one tile kernel per pass.  Afterwards the state's layout is the
 * plan's final layout; readouts account for it.  Asynchronous. */
qvm_status qvm_run_plan(qvm_sv* sv, const qvm_plan* plan);

/* Features of every pass for the learned cost model, QVM_PASS_FEATURES
 * floats per pass in execution order: 0 n, 1 dtype (0 complex64, 1
 * complex128), 2 tile qubits L, 3..6 blocks of k = 3, 4, 5, 6 (after
 * padding), 7 sum of 2^k over blocks, 8 diagonal runs, 9 diagonal phase
 * terms, 10 gates applied, 11 remap (0/1), 12 tile bits at physical
 * positions >= 20, 13 mean, 14 min, 15 max physical position of block
 * qubits, 16 block qubits on the always-tile low bits, 17 qubits spanned by
 * the blocks' gates (before padding), 18 log2 state bytes, 19 log2 tile
 * count, 20 diagonal runs and 21 phase terms that take the angle-
 * accumulating path (standalone or in the epilogue of the block before
 * them), 22 workgroup barriers between the pass's ops.  out needs
 * cap >= n_passes * QVM_PASS_FEATURES floats (NULL: only *n_passes is
 * set). */
#define QVM_PASS_FEATURES 23
qvm_status qvm_plan_pass_features(const qvm_plan* plan, float* out, size_t cap,
                                  int32_t* n_passes);

/* The plan's device image as uploaded by qvm_run_plan (for inspection and
 * emulation): *bytes receives its size; when out is not NULL, cap >= that
 * size bytes are copied to it.  *pass_table receives the byte offset of the
 * pass records inside the image, *n_passes their count.  The record layouts
 * are internal and may change between builds. */
qvm_status qvm_plan_image(const qvm_plan* plan, void* out, size_t cap, size_t* bytes,
                          uint64_t* pass_table, int32_t* n_passes);

qvm_status qvm_plan_destroy(qvm_plan* plan);

/* Peephole pre-pass before fusion (paper, "Quantum circuit optimization",
 * first layer: identity pairs removed, consecutive rotations merged).  Two
 * gates are consecutive when they act on the same qubits and no gate in
 * between touches any of them.  With identical targets and controls:
 * H H, X X, Y Y, Z Z, SWAP SWAP, S SDG, T TDG (either order) cancel; I is
 * dropped; RX, RY, RZ, P and RZZ pairs merge into one gate with the summed
 * angle (dropped when the sum is exactly 0); T T -> S, TDG TDG -> SDG,
 * S S -> Z, SDG SDG -> Z; results are compared again with the gate before,
 * so chains collapse.  Every rule is an exact matrix identity (merged
 * angles are rounded sums).  Host-only.  Writes the kept gates, in order, to
 * out (capacity n_in, must not overlap in) and their count to *n_out; the
 * u pointers of QVM_G_MATRIX gates are copied, so in's matrices must stay
 * alive as long as out is used.  QVM_EARG / QVM_ERANGE for invalid gates. */
qvm_status qvm_simplify(const qvm_gate* in, size_t n_in, int n_qubits, qvm_gate* out,
                        size_t* n_out);

/* ------------------------------------------------------------- gradients */

/* Number of gate groups qvm_adjoint_expect_grad splits a circuit into (each
 * group is one pass over the batch forward and one in reverse; up to 4
 * target qubits per group for complex64, 3 for complex128), for callers
 * that account for the passes the sweep executes.  Same gate, parameter
 * index and error rules as qvm_adjoint_expect_grad.  Host-only. */
qvm_status qvm_adjoint_group_count(int n_qubits, qvm_dtype dt, const qvm_gate* gates, size_t n_gates,
                                   const int32_t* param_index, int n_params, int32_t* n_groups);

/* Bytes of device workspace qvm_adjoint_expect_grad needs. */
size_t qvm_adjoint_workspace_bytes(int n_qubits, int batch, size_t n_gates);

/* Expectation f_b = <psi(theta_b)|H|psi(theta_b)> of H = sum_t coeff[t] P_t
 * (Pauli strings in symplectic form, as in qvm_expect_pauli) for a batch of
 * parameter vectors, and its gradient by the adjoint reverse sweep
 * (Jones & Gacon, arXiv:2009.02823) — the paper's variational circuits
 * ("Variational quantum circuit": parameters updated, circuit re-run, qop
 * expectation) differentiated without finite differences.
 * The circuit starts from |0..0>; every gate has one target (k = 1) and any
 * controls.  param_index[i] = -1 for a fixed gate, else the index of the
 * gate's angle in a parameter row; such gates must be RX, RY or RZ (their
 * stored params are ignored).  params_host is [batch][n_params] row-major.
 * psi_dev and lam_dev each hold batch x 2^n amplitudes of dt (caller-owned,
 * distinct); work_dev at least qvm_adjoint_workspace_bytes.  Outputs on the
 * host: f_out[batch]; grad_out[batch][n_params] (NULL: expectation only).
 * All batch elements run together: the gates are split into groups that
 * target at most 4 (complex64) / 3 (complex128) qubits, and each group is
 * one launch that keeps those amplitudes of psi and lambda in registers
 * while it applies (and, in the reverse sweep, differentiates) every gate
 * of the group, so a group costs one pass over the states.  Sums in double
 * precision.  Synchronous on hip_stream. */
qvm_status qvm_adjoint_expect_grad(int n_qubits, qvm_dtype dt, int batch,
                                   const qvm_gate* gates, size_t n_gates,
                                   const int32_t* param_index, int n_params,
                                   const double* params_host, size_t n_terms,
                                   const uint64_t* x_mask, const uint64_t* z_mask,
                                   const double* coeff, void* psi_dev, void* lam_dev,
                                   void* work_dev, size_t work_bytes, void* hip_stream,
                                   double* f_out, double* grad_out);

/* Size of the library's static adjoint workspace (64 MiB per device). */
#define QVM_ADJ_SCRATCH_BYTES (64u << 20)

/* qvm_adjoint_expect_grad without a workspace argument, for callers that
 * cannot allocate device memory (code under HIP graph capture, serving
 * loops, harnesses that forbid hipMalloc): the workspace is a static array
 * of QVM_ADJ_SCRATCH_BYTES in the library, one per device, allocated when
 * the library's code object is loaded on that device and held until the
 * process ends.  This call allocates no device memory.  The caller still
 * owns psi_dev and lam_dev (batch x 2^n amplitudes each) and the outputs;
 * results are identical to qvm_adjoint_expect_grad's.  A problem whose
 * workspace (matrices 2 x n_gates x batch x 64 bytes, plus reduction
 * partials (trainable gates + 1) x batch x 520 bytes, plus the op table)
 * exceeds QVM_ADJ_SCRATCH_BYTES returns QVM_ENOMEM before anything is
 * enqueued; 20 qubits, 944 gates of which 640 trainable, batch 64 needs
 * about 29 MB.  Every call on one device shares that device's array:
 * calls that overlap on one device (other host threads, or other streams
 * before this one's synchronisation) race and give wrong results.  The
 * call is synchronous on hip_stream, so calls made one after another are
 * safe; no contents carry over between calls. */
qvm_status qvm_adjoint_expect_grad_static(int n_qubits, qvm_dtype dt, int batch,
                                          const qvm_gate* gates, size_t n_gates,
                                          const int32_t* param_index, int n_params,
                                          const double* params_host, size_t n_terms,
                                          const uint64_t* x_mask, const uint64_t* z_mask,
                                          const double* coeff, void* psi_dev, void* lam_dev,
                                          void* hip_stream, double* f_out, double* grad_out);

/* ------------------------------------------------------------ cost model */

/* A three-layer perceptron (d features -> H -> H -> 1, ReLU) that predicts
 * the log time of a fused pass from its features; the learned fusion planner
 * uses it to choose among candidate plans.  FP32, device pointers, all
 * asynchronous on `stream`.  Parameters are packed [W1 (d x H), b1 (H),
 * W2 (H x H), b2 (H), W3 (H x 1), b3 (1)], row-major, count from
 * qvm_mlp_param_count.  X is [B][d] row-major.
 * forward:  act receives Z1, H1, Z2, H2 (4 B H floats), y receives B outputs.
 * backward: loss L = (1/B) sum (y - t)^2; grads (packed like params) get dL;
 *           work holds 2 B H + B floats; loss_dev (nullable) receives L.
 * adam:     one Adam step (Kingma & Ba) with bias correction; step >= 1. */
size_t qvm_mlp_param_count(int d, int hidden);
qvm_status qvm_mlp_forward(int batch, int d, int hidden, const float* X, const float* params,
                           float* act, float* y, void* stream);
qvm_status qvm_mlp_backward(int batch, int d, int hidden, const float* X, const float* t,
                            const float* params, const float* act, const float* y, float* grads,
                            float* work, float* loss_dev, void* stream);
qvm_status qvm_mlp_adam_step(size_t n_params, float* params, const float* grads, float* m,
                             float* v, int step, float lr, float beta1, float beta2, float eps,
                             void* stream);

/* --------------------------------------------------------------- timing */

/* Streaming device copy of `bytes` from src to dst (device pointers, 16-byte
 * aligned, bytes a multiple of 16, not overlapping), asynchronous on
 * `stream`: the measured bandwidth reference that effective GB/s figures are
 * compared with beside the HBM peak (a STREAM-style copy; no paper
 * counterpart).  QVM_EARG for NULL, misaligned or overlapping buffers. */
qvm_status qvm_stream_copy(void* dst, const void* src, size_t bytes, void* stream);


/* Per-launch kernel timing for one state: between qvm_profile_begin and
 * qvm_profile_end every kernel the library launches for the state is
 * bracketed by two HIP events recorded on the state's stream.  The
 * durations are aggregated per kernel class together with the algorithmic
 * bytes (amplitudes the launch must read and write, times their size) and
 * flops (complex multiply-adds of dense and fused matrices, 8 flops each).
 * Used to report achieved bandwidth and throughput against the roofline. */
typedef struct qvm_kernel_stat {
    char name[24];           /* dense1..dense3, diag, phase, swappair, tile, basis, rdm1 */
    int64_t launches;
    double total_ms;
    double bytes;
    double flops;
} qvm_kernel_stat;

qvm_status qvm_profile_begin(qvm_sv* sv);

/* Synchronises the stream, writes up to max aggregated records into out
 * (nullable) and their number into *count, and stops recording.  The
 * individual launches stay readable with qvm_profile_launches until the next
 * qvm_profile_begin. */
qvm_status qvm_profile_end(qvm_sv* sv, qvm_kernel_stat* out, int32_t max, int32_t* count);

/* Per-launch durations (ms) and kernel classes (index into the class list
 * above: 0 dense1 .. 7 basis, 8 rdm1) of the last profiled interval, in launch
 * order; up to max entries, *count = the number recorded. */
qvm_status qvm_profile_launches(const qvm_sv* sv, double* ms, int32_t* kind, int32_t max,
                                int32_t* count);

/* Thread-local message for the last non-OK status returned on this thread. */
const char* qvm_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* QVM_H */
