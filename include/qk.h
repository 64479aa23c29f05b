/*
 * qk.h -- C ABI of the MI355X state-vector engine (libqk.so).
 *
 * The interface follows the paper's command set (section "Q-Kit."): add
 * qubits, perform a gate operation, measure, and define a custom gate as a
 * matrix or as a function; classical bits receive measurement outcomes and
 * steer later gates (the paper's Copy command and classically controlled
 * SigmaX / RPhase in Appendix A).  Explicit index arrays replace the
 * paper's "a:b" range syntax.
 *
 * Conventions
 *   - State: 2^n complex amplitudes, contiguous, interleaved (re, im);
 *     QK_C64 = two float32 per amplitude, QK_C128 = two float64.
 *   - Qubit q is bit q of the amplitude index (little-endian).  The paper's
 *     scripts number qubits big-endian; a front end maps paper qubit p of an
 *     n-qubit register to bit n-1-p.
 *   - Inside a gate, row/column index bit j of its matrix (or permutation
 *     index) corresponds to targets[j].
 *   - Every call returns qk_status (0 = QK_OK, < 0 = error); nothing aborts
 *     or throws.  Input arrays are copied before return; the caller keeps
 *     ownership of every host buffer it passes.
 *   - Work is enqueued on the HIP stream given to qk_create and runs
 *     asynchronously.  Calls documented as "synchronises" wait for it.  A
 *     failure of asynchronous device work is latched and returned
 *     (QK_E_HIP) by the next synchronising call.
 *   - One qk_sim is used by one host thread at a time.  Several sims may
 *     share a device through different streams.
 */
#ifndef QK_ABI_H_
#define QK_ABI_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t qk_status;
#define QK_OK 0
#define QK_E_ARG (-1)             /* bad index, duplicate qubit, size limit, unknown name */
#define QK_E_NOT_UNITARY (-2)     /* matrix fails || M^H M - I ||_max <= tol */
#define QK_E_NOT_PERMUTATION (-3) /* index function is not a bijection of [0, 2^k) */
#define QK_E_OOM (-4)             /* allocator returned NULL / device memory exhausted */
#define QK_E_HIP (-5)             /* HIP runtime error (launch or latched asynchronous fault) */
#define QK_E_STATE (-6)           /* invalid state for the call (e.g. forced outcome of probability 0) */
#define QK_E_UNSUPPORTED (-7)     /* valid request the engine does not implement */

typedef int32_t qk_dtype;
#define QK_C64 1
#define QK_C128 2

typedef int32_t qk_gate;

/* Builtin gate ids (matrices in FP64; row/column bit j <-> targets[j]):
 *   H = [[1,1],[1,-1]]/sqrt2, X (the paper's SigmaX), Y, Z, S = diag(1,i),
 *   T = diag(1,e^{i pi/4}), SDG, TDG (adjoints),
 *   RX/RY/RZ(theta) = exp(-i theta P/2), PHASE(phi) = diag(1, e^{i phi}),
 *   CPHASE(phi) = diag(1,1,1,e^{i phi}) (two targets, Appendix A),
 *   SWAP (two targets), RZZ(theta) = exp(-i theta Z(x)Z/2).
 * Any gate takes controls; X with one control is CNOT. */
#define QK_H 1
#define QK_X 2
#define QK_Y 3
#define QK_Z 4
#define QK_S 5
#define QK_T 6
#define QK_SDG 7
#define QK_TDG 8
#define QK_RX 9
#define QK_RY 10
#define QK_RZ 11
#define QK_PHASE 12
#define QK_CPHASE 13
#define QK_SWAP 14
#define QK_RZZ 15

#define QK_MAX_CONDS 8        /* classical conditions per gate */
#define QK_MAX_GATE_QUBITS 40 /* targets + controls per gate */
#define QK_MAX_MATRIX_K 10    /* largest user matrix gate: 2^10 x 2^10 */
#define QK_MAX_PERM_K 30      /* largest permutation gate */
#define QK_MAX_FUSION_K 6     /* largest fused block */

typedef struct qk_sim_s* qk_sim;

/* Device-memory provider.  alloc(bytes, stream, ctx) returns device memory
 * usable on `stream` or NULL; free(ptr, bytes, stream, ctx) returns it.  With
 * a NULL provider the library uses hipMalloc / hipFree. */
typedef struct qk_allocator {
  void* (*alloc)(size_t bytes, void* stream, void* ctx);
  void (*free)(void* ptr, size_t bytes, void* stream, void* ctx);
  void* ctx;
} qk_allocator;

/* Classical condition: the gate runs iff cbits[cbit] == value (0 or 1).
 * Several conditions are ANDed.  Evaluated on the device when the gate
 * executes, so no host round trip is needed between a measurement and the
 * gates it steers. */
typedef struct qk_cond {
  int32_t cbit;
  int32_t value;
} qk_cond;

/* ---- lifetime ---------------------------------------------------------- */

/* Create an empty simulator (0 qubits, 0 cbits; the state is the scalar 1).
 * `alloc` may be NULL (hipMalloc); it is copied.  `hip_stream` (a
 * hipStream_t, may be NULL for the null stream) receives all device work.
 * Allocates nothing on the device until qubits are added. */
qk_status qk_create(qk_dtype dtype, const qk_allocator* alloc, void* hip_stream, qk_sim* out);

/* Create a simulator whose state is kept sparse: only its nonzero amplitudes,
 * as entries with ascending amplitude index (the paper runs circuits whose
 * state stays sparse -- the recycled-qubit Shor circuit, and a 39-qubit
 * conventional Shor circuit on a 12 GB desktop -- section "Shor's
 * Factorization with Q-Kit.").  Up to 62 qubits; at most `max_nonzeros`
 * entries (1 .. 2^32), for which about 60 (complex64) or 76 (complex128)
 * bytes each of device memory are allocated when qubits are first added.
 * Gates, conditions, measurement, cbits, shots, qk_norm2, qk_reset and the
 * measurement log work as for a dense simulator (same definitions; a gate
 * whose result would exceed max_nonzeros fails with QK_E_OOM and leaves the
 * state unchanged); qk_get_state / qk_set_state convert from / to a dense
 * host vector (n <= 40).  Not available: fusion, graph capture,
 * qk_state_ptr, qk_probabilities, inner products between two simulators.
 * Gates with classical conditions read the cbits back, and gates that change
 * the set of nonzero entries read entry counts back, so calls synchronise. */
qk_status qk_create_sparse(qk_dtype dtype, const qk_allocator* alloc, void* hip_stream, int64_t max_nonzeros,
                           qk_sim* out);

/* Number of entries (nonzero amplitudes, counting those that cancel to
 * exactly 0 only when a measurement drops them) of a sparse simulator. */
qk_status qk_sparse_nnz(qk_sim sim, int64_t* nnz);

/* Copy the entries of a sparse simulator to host memory: idx[i] ascending
 * amplitude indices, amps[i] their amplitudes (interleaved re, im in the
 * simulator's precision); cap = room in both arrays (QK_E_ARG if smaller than
 * the entry count, which *nnz receives).  Synchronises. */
qk_status qk_sparse_entries(qk_sim sim, uint64_t* idx, void* amps, int64_t cap, int64_t* nnz);

/* Synchronise and release every buffer of the simulator. */
qk_status qk_destroy(qk_sim sim);

/* AddQubits (Appendix A): psi -> psi (x) |0...0>.  New qubits take bits
 * n..n+count-1, so existing amplitudes keep their indices and the new part
 * of the state is zero.  *first_qubit (may be NULL) receives n.  The first
 * call initialises |0...0>.  Reallocates the state (count > 0). */
qk_status qk_add_qubits(qk_sim sim, int32_t count, int32_t* first_qubit);

/* AddCbits (Appendix A): count new classical bits set to 0, numbered from
 * the current count; *first_cbit (may be NULL) receives it. */
qk_status qk_add_cbits(qk_sim sim, int32_t count, int32_t* first_cbit);

/* ---- gate definitions: custom gates given by a matrix or by an index
 * function, as the paper's engine allows (section "Q-Kit.") --------------- */

/* Builtin id by name ("H", "X", "SIGMAX", "HADAMARD", "CNOT" = X, "RZ", ...). */
qk_status qk_gate_builtin(const char* name, qk_gate* out);

/* Unitary gate on k targets (1 <= k <= QK_MAX_MATRIX_K).  m: 2^k x 2^k
 * complex, row-major, interleaved (re, im), FP64; copied and kept in FP64 (a
 * rounded copy serves complex64 states).  Rejected with QK_E_NOT_UNITARY
 * unless || M^H M - I ||_max <= unitarity_tol.  `name` may be NULL. */
qk_status qk_define_gate_matrix(qk_sim sim, const char* name, int32_t k, const double* m,
                                double unitarity_tol, qk_gate* out);

/* Permutation (oracle) gate U|x> = |f(x)> on k targets (1 <= k <=
 * QK_MAX_PERM_K).  f is called on the host for every x in [0, 2^k) during
 * this call (ctx is passed through); the results must form a bijection of
 * [0, 2^k), else QK_E_NOT_PERMUTATION.  The table is kept on the device. */
qk_status qk_define_gate_index(qk_sim sim, const char* name, int32_t k,
                               uint64_t (*f)(uint64_t x, const void* ctx), const void* ctx,
                               qk_gate* out);

/* Same as qk_define_gate_index with the values f(0..2^k-1) given as an array. */
qk_status qk_define_gate_table(qk_sim sim, const char* name, int32_t k, const uint64_t* table,
                               qk_gate* out);

/* Affine permutation family x -> (a x + b) mod 2^k (a odd, 1 <= k <= 32),
 * evaluated on the device in closed form, no table.  When applied,
 * params[0] = j (optional, default 0) applies the 2^j-th power of the map,
 * like the paper's QuModExpUaj gate takes j. */
qk_status qk_define_gate_affine(qk_sim sim, const char* name, int32_t k, uint64_t a, uint64_t b,
                                qk_gate* out);

/* Modular multiplication family (the paper's QuModExpUaj a= j= N=, Appendix
 * A): y -> (a^(2^j) y) mod N for y < N, y itself for N <= y < 2^k, which
 * keeps the map a permutation of [0, 2^k) (2 <= N <= 2^k, N < 2^32, gcd(a, N)
 * = 1, else QK_E_NOT_PERMUTATION).  params[0] = j when applied (default 0).
 * Evaluated on the device in closed form, no table. */
qk_status qk_define_gate_modmul(qk_sim sim, const char* name, int32_t k, uint64_t a, uint64_t N, qk_gate* out);

/* ---- gate operation (the paper's GateOp) ------------------------------- */

/* Apply `gate` to `targets` (count must equal the gate's arity), restricted
 * to the subspace where every control qubit is 1, iff every classical
 * condition holds at execution time.  params: angles for RX, RY, RZ, PHASE,
 * CPHASE, RZZ (params[0], radians); j for affine and modular gates.  Targets and
 * controls must be distinct and < n.  Enqueued on the stream; returns
 * before the device runs it.  With fusion enabled (qk_set_fusion) an
 * unconditioned matrix gate may be held back and combined with later gates;
 * any measurement, conditioned or permutation gate, readout or qk_flush
 * first emits everything held back, in order.  On a dense state an
 * uncontrolled, unconditioned SWAP moves no data: the simulator exchanges the
 * two qubits' index bits in its qubit map, which every later gate and
 * measurement goes through.  An uncontrolled permutation gate (outside a
 * graph capture) gathers the permuted state into the simulator's second
 * state-sized buffer, which then holds the state: the two buffers trade
 * places and no copy back is made.  qk_get_state, qk_set_state, qk_state_ptr,
 * qk_probabilities, sampling, inner products of two simulators, graph
 * capture and graph launch first put the state back in logical qubit order
 * (one physical swap per misplaced qubit); qk_norm2 and measurements do not
 * need to (the "swap_relabel" tuning key turns this off). */
qk_status qk_apply_gate(qk_sim sim, qk_gate gate, const int32_t* targets, int32_t n_targets,
                        const int32_t* controls, int32_t n_controls, const qk_cond* conds,
                        int32_t n_conds, const double* params, int32_t n_params);

/* ---- measurement (the paper's Measure + Copy) -------------------------- */

/* In-place measurement of `qubit` with the uniform u in [0, 1): p_b = sum of
 * |a_i|^2 over indices with bit qubit = b (accumulated in FP64, fixed
 * order, independent of other work on the device), P0 = p0 / (p0 + p1),
 * outcome = (u < P0) ? 0 : 1; kept amplitudes are scaled by 1/sqrt(p_outcome),
 * the others set to 0.  The outcome is written to cbit `cbit` on the device
 * (cbit = -1: not stored).  No host round trip.  A state of zero norm (which
 * only qk_set_state can produce) gives outcome 1 with p0 = p1 = 0: the state
 * stays zero, the cbit is not written and the measurement log records it.
 * QK_E_ARG if u is not in [0, 1). */
qk_status qk_measure(qk_sim sim, int32_t qubit, int32_t cbit, double u);

/* As qk_measure with u read from device memory d_u when the step executes
 * (for captured graphs whose uniforms change between replays).  The host
 * cannot check such a draw: NaN and negative values count as 0, values at or
 * above 1 as the largest double below 1. */
qk_status qk_measure_dev(qk_sim sim, int32_t qubit, int32_t cbit, const double* d_u);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops and harnesses that forbid hipMalloc): the
 * measurement of qk_measure_dev on a caller's state, with no simulator and no
 * allocation.  d_state: 2^n_qubits amplitudes of `dtype` in device memory
 * (qubit q = bit q of the index), collapsed and renormalised in place exactly
 * as qk_measure_dev does (same kernels, same fixed-order FP64 sums); d_u: the
 * uniform in device memory, read when the step executes (clamped into [0, 1));
 * d_cbit (may be NULL): receives the outcome (0/1) unless its probability is
 * 0; d_result (may be NULL): receives p0, p1 and the outcome as 3 doubles.
 * Enqueued on hip_stream (NULL: the null stream of the current device);
 * asynchronous.  The partial sums and the result live in a fixed device array
 * of the library (16,448 bytes per GPU, kept until the process ends) instead
 * of allocated memory, so calls that overlap on one GPU race: order them on
 * one stream.  1 <= n_qubits <= QK_NOALLOC_MAX_QUBITS, else QK_E_ARG; errors
 * are reported by qk_last_error(NULL). */
#define QK_NOALLOC_MAX_QUBITS 40
qk_status qk_measure_noalloc(qk_dtype dtype, void* d_state, int32_t n_qubits, int32_t qubit, const double* d_u,
                             uint8_t* d_cbit, double* d_result, void* hip_stream);

/* Test hook: force `outcome` (0/1).  Synchronises; QK_E_STATE if the outcome
 * has probability 0 (the state is then left unchanged). */
qk_status qk_postselect(qk_sim sim, int32_t qubit, int32_t cbit, int32_t outcome);

/* Copy the first n cbits (one byte each, 0/1) to host memory.  Synchronises. */
qk_status qk_read_cbits(qk_sim sim, uint8_t* out, int32_t n);

/* Measurement log: for the last `count` measurements (oldest first, at most
 * 4096 kept) write p0, p1 (FP64 sums) and the outcome (as a double) to
 * out[3*i .. 3*i+2].  *written receives the count written.  Synchronises. */
qk_status qk_read_measure_log(qk_sim sim, double* out, int32_t count, int32_t* written);

/* ---- deferred measurement (measuring at the end, many shots) ------------- */

/* The paper's circuits measure qubits either in place or deferred to the end
 * (section "Q-Kit."); measuring the listed qubits at the end, once per shot,
 * draws an amplitude index i with probability |a_i|^2 / sum_j |a_j|^2 and
 * reads its bits at those qubits.  The state is not changed.
 *
 * For each uniform u_s in [0, 1): i_s = the smallest index whose running sum
 * of |a_j|^2 in index order exceeds u_s times the total (FP64 sums; an index
 * of zero weight is never drawn, and a draw within rounding of an interval
 * boundary may land on either side of it).  out[s] packs bit qubits[j] of
 * i_s into bit j; n_qubits = 0 (qubits may be NULL) gives i_s itself.
 * qubits must be distinct and < n; n_shots <= 2^32.
 *
 * qk_sample: uniforms and out are host arrays of n_shots entries; every
 * uniform must lie in [0, 1) (else QK_E_ARG, nothing run); a state of zero
 * norm gives QK_E_STATE.  Synchronises.  Costs one read sweep of the state
 * plus one wave and about 4 KiB of reads per shot; device work space of
 * 2^n / 128 bytes and 16 bytes per shot is allocated on first use and kept. */
qk_status qk_sample(qk_sim sim, const int32_t* qubits, int32_t n_qubits, const double* uniforms,
                    int64_t n_shots, uint64_t* out);

/* As qk_sample with device arrays: d_uniforms (n_shots doubles, read when the
 * step executes) and d_out (n_shots uint64).  Asynchronous, no host round
 * trip.  Draws outside [0, 1) are clamped; a state of zero norm writes
 * UINT64_MAX to every d_out entry.  Inside a graph capture the work space
 * must already exist (call it once on the same qubit count first), else
 * QK_E_STATE. */
qk_status qk_sample_dev(qk_sim sim, const int32_t* qubits, int32_t n_qubits, const double* d_uniforms,
                        int64_t n_shots, uint64_t* d_out);

/* Normalised probability distribution of the listed qubits (the paper's
 * probability view of the state, section "Q-Kit."): out[m] = sum of
 * |a_i|^2 over the i whose bit qubits[j] equals bit j of m, divided by the
 * sum of all |a_i|^2 (FP64, fixed order).  1 <= n_qubits <= min(n, 24);
 * out is a host array of 2^n_qubits doubles.  QK_E_STATE for a state of
 * zero norm.  Synchronises. */
qk_status qk_probabilities(qk_sim sim, const int32_t* qubits, int32_t n_qubits, double* out);

/* ---- readout ------------------------------------------------------------ */

/* Copy the state (2^n amplitudes, bytes = 2^n * amplitude size) to host
 * memory.  Synchronises. */
qk_status qk_get_state(qk_sim sim, void* host_out, size_t bytes);

/* Replace the state with host data of the same size.  Synchronises. */
qk_status qk_set_state(qk_sim sim, const void* host_in, size_t bytes);

/* Current device address and size of the state, in logical qubit order
 * (relabelled qubits are put back first).  Valid until the next call
 * that adds qubits, applies an uncontrolled permutation gate (which leaves
 * the state in the simulator's other buffer) or destroys the simulator.
 * Emits held-back gates first.  Other gates update the state in place, but a
 * later uncontrolled SWAP may only relabel qubits: call qk_state_ptr again
 * before reading through the pointer (or set the "swap_relabel" tuning key
 * to 0). */
qk_status qk_state_ptr(qk_sim sim, void** dev_ptr, size_t* bytes);

/* FP64 inner product <a|b> = sum conj(a_i) b_i of two simulators with the same
 * qubit count (dtypes may differ), fixed-order reduction.  Synchronises both. */
qk_status qk_inner_product(qk_sim a, qk_sim b, double* re, double* im);

/* FP64 squared norm sum |a_i|^2.  Synchronises. */
qk_status qk_norm2(qk_sim sim, double* out);
/* Asynchronous readouts for hosts that must not wait on the device (a
 * serving loop): both only enqueue work on the simulator's stream and
 * return.  qk_norm2_async enqueues the norm's fixed-order partial sums
 * (*count receives their number nb) and their copy into host_partials as
 * (re, im) pairs (capacity >= 2 nb doubles, at most 2048); the sum of the
 * nb real parts taken in order equals qk_norm2 exactly.  qk_read_cbits_async
 * enqueues the copy of the first n cbits.  The host buffers (pinned memory
 * keeps the copies asynchronous) must stay valid, and hold the results only
 * after the stream has reached this point (an event recorded after the call
 * has completed).  Dense states only for the norm. */
qk_status qk_norm2_async(qk_sim sim, double* host_partials, int32_t capacity, int32_t* count);
qk_status qk_read_cbits_async(qk_sim sim, uint8_t* host_out, int32_t n);

/* ---- execution control -------------------------------------------------- */

/* Gate fusion: max_k = 0 applies every gate on its own; 2 <= max_k <= 6
 * combines consecutive unconditioned matrix gates (reordering only gates on
 * disjoint qubits) into blocks on at most max_k qubits, composed in FP64 on
 * the host and applied as one dense 2^k x 2^k sweep (matrix cores). */
qk_status qk_set_fusion(qk_sim sim, int32_t max_k);

/* Emit every held-back gate now (asynchronous). */
qk_status qk_flush(qk_sim sim);

/* Flush, wait for all work of the simulator, report latched errors. */
qk_status qk_sync(qk_sim sim);

/* Launch-shape knobs (results never depend on them).  Keys:
 *   "nt"          0: regular loads/stores, 1 (default): non-temporal when
 *                 the state is larger than 256 MiB (smaller states stay in
 *                 the Infinity Cache between sweeps) and a sweep's accesses
 *                 cover whole cache lines, 2: always;
 *   "lane_bfly"   1 (default): targets below bit 6 use the cross-lane
 *                 butterfly, 0: the strided one;
 *   "sweep_items" amplitudes per thread of the strided butterfly, amplitude
 *                 pairs per thread of the swap sweep (1, 2, 4; default 1
 *                 for complex128, 2 for complex64);
 *   "diag_items"  amplitudes per thread of diagonal and phase sweeps
 *                 (1, 2, 4; default 1 for complex128, 2 for complex64);
 *   "lane_items"  64-amplitude segments per wave of the cross-lane
 *                 butterfly (1, 2, 4; default 1 for complex128, 2 for complex64);
 *   "mfma_waves"  waves per compute unit for matrix-core sweeps (4..32);
 *   "mfma_cols"   tile columns per wave for matrix-core sweeps (16, 32
 *                 default, 64; capped by registers for large k);
 *   "mfma_areg"   blocks of 5-6 qubits: 1 keeps the matrix fragments in
 *                 registers, 0 (default) re-reads them from LDS per tile;
 *   "mfma_lds"    blocks of 4-5 qubits: 1 stages each workgroup's tile
 *                 (2^k rows x 1 KiB) through LDS so that global memory is read
 *                 and written in address order, 0: each wave loads its own
 *                 register tile, 2 (default): LDS tiles for 4-qubit blocks
 *                 and for complex64 5-qubit blocks with three or more targets
 *                 below bit 5, register tiles otherwise;
 *   "lds_wg"      workgroups per compute unit of the LDS-staged kernel (1..8,
 *                 default 2);
 *   "xcd"         1 (default): the per-gate sweeps renumber their workgroups
 *                 so that each of the 8 XCDs sweeps one contiguous range,
 *                 0: workgroups in launch order;
 *   "swap_relabel" 1 (default): an uncontrolled, unconditioned SWAP on a
 *                 dense state relabels the two qubits instead of moving data
 *                 (see qk_apply_gate); 0: every SWAP is a sweep;
 *   "diag_runs"   1 (default): consecutive diagonal gates (at most 6 qubits
 *                 each, with their own controls and cbit conditions, which
 *                 are read on the device when the pass runs) are held back
 *                 and applied in one pass over the subspace all of them
 *                 require, whenever that touches no more amplitudes than one
 *                 sweep per gate; 0: one sweep per gate.  Results agree with
 *                 one sweep per gate up to rounding (factors multiplied in
 *                 FP64 before one multiplication of each amplitude);
 *   "stages"      0 (default), 1: the LDS-tile mode.  Builtin gates (at
 *                 most 4 controls, conditions on cbits below 256) on a dense
 *                 state of 12 (complex128) / 13 (complex64) to 31 qubits are
 *                 held back; at the next other operation they are grouped
 *                 into stages of 12 / 13 qubits (gates pass one another only
 *                 on disjoint qubits or when both are diagonal) and each
 *                 stage is one pass over the state: every chunk of it (the
 *                 amplitudes that agree on the other qubits) is gathered
 *                 into LDS, every gate of the stage is applied there one at
 *                 a time (no matrices composed; results agree with the
 *                 per-gate sweeps up to rounding), and it is written back.
 *                 Each stage counts as one sweep in qk_stats.  Setting
 *                 the key applies whatever is held back first.
 * QK_E_ARG for an unknown key or value. */
qk_status qk_set_tuning(qk_sim sim, const char* key, int32_t value);
qk_status qk_get_tuning(qk_sim sim, const char* key, int32_t* value);

qk_status qk_num_qubits(qk_sim sim, int32_t* n);

/* Counters since creation: sweeps launched (state passes), fused blocks,
 * gates absorbed into fused blocks.  Any pointer may be NULL. */
qk_status qk_stats(qk_sim sim, int64_t* sweeps, int64_t* fused_blocks, int64_t* fused_gates);

/* Text of the last error on `sim` (valid until the next call on it), or of
 * the last error of a call that had no simulator when sim is NULL. */
const char* qk_last_error(qk_sim sim);

const char* qk_status_string(qk_status st);

/* ---- captured gate sequences (HIP graphs) --------------------------------
 * A sequence of calls on one simulator can be captured once and replayed
 * with one launch: qk_capture_begin, then any qk_reset / qk_apply_gate /
 * qk_measure / qk_measure_dev / qk_flush calls (no readout, no qk_add_*),
 * then qk_capture_end.  Nothing runs during capture; each qk_graph_launch
 * replays the whole sequence on the simulator's state, cbits and stream.
 * Permutation gates inside a capture keep the state in its buffer; if an
 * uncontrolled permutation gate applied after the capture moved the state to
 * the other buffer, qk_graph_launch first copies it back (QK_E_STATE if
 * qubits were added since the capture).  The graph keeps the constants it
 * uploads; destroy graphs before their simulator. */
typedef struct qk_graph_s* qk_graph;

/* Set the state to |0...0> and every cbit to 0 (asynchronous; capturable). */
qk_status qk_reset(qk_sim sim);
qk_status qk_capture_begin(qk_sim sim);
qk_status qk_capture_end(qk_sim sim, qk_graph* out);
qk_status qk_graph_launch(qk_graph graph);
qk_status qk_graph_destroy(qk_graph graph);

/* ---- batched execution: many circuits in one persistent launch -----------
 * Circuits on 1..24 qubits, builtin gates and measurements only, each started
 * from |0...0>.  qk_batch_run launches one persistent grid whose workgroups
 * take circuits from a device queue (largest first), one circuit per
 * workgroup.  A circuit on at most 13 qubits (complex128) or 14 (complex64)
 * keeps its state in on-chip memory (LDS) for the whole circuit; a larger one
 * keeps it in the batch's device buffer and runs by stages: gate groups on at
 * most 12 (complex128) or 13 (complex64) qubits, each applied chunk by chunk
 * through LDS (one read and one write of the state per stage).  Results do
 * not depend on which circuits share a launch. */
#define QK_OP_GATE 1
#define QK_OP_MEASURE 2

typedef struct qk_op {
  int32_t kind;          /* QK_OP_GATE or QK_OP_MEASURE */
  int32_t gate;          /* builtin gate id (QK_OP_GATE) */
  int32_t targets[2];
  int32_t n_targets;
  int32_t controls[4];
  int32_t n_controls;
  qk_cond conds[2];      /* classical conditions of a gate (ANDed) */
  int32_t n_conds;
  double param;          /* angle of RX, RY, RZ, PHASE, CPHASE, RZZ */
  int32_t qubit;         /* QK_OP_MEASURE: measured qubit */
  int32_t cbit;          /* QK_OP_MEASURE: destination cbit or -1 */
  double u;              /* QK_OP_MEASURE: pre-drawn uniform in [0, 1) */
} qk_op;

typedef struct qk_batch_s* qk_batch;

/* A whole op list on one simulator in one call (for hosts that submit a
 * circuit per request, such as a serving loop): each QK_OP_GATE record is
 * qk_apply_gate(gate, targets, controls, conds, params) with the gate's own
 * parameter count (builtins; j for affine and modular families, from
 * `param`), each QK_OP_MEASURE record is qk_measure(qubit, cbit, u).  Gate
 * ids may be builtins or gates defined on `sim`.  Stops at the first failing
 * record: its status is returned, qk_last_error names the record, and
 * *n_done (may be NULL) receives the number of records applied. */
qk_status qk_apply_ops(qk_sim sim, const qk_op* ops, int32_t n_ops, int32_t* n_done);

/* Host only (no device work): the fused blocks qk_set_fusion(max_k) would
 * form for a list of unconditioned builtin gates (op records as for
 * batches).  *n_blocks receives the block count; for the first max_blocks
 * blocks, block_masks[b] = the block's qubits as a bit mask, block_gates[b] =
 * gates composed, and (if matrices != NULL) the 2^k x 2^k FP64 block matrices
 * (row/column bit j <-> j-th lowest qubit of the mask, row-major, (re, im)
 * interleaved) one after another in `matrices` (capacity matrices_len
 * doubles).  Applying the blocks in order equals applying the gates in order. */
qk_status qk_plan_fusion(int32_t n_qubits, const qk_op* ops, int32_t n_ops, int32_t max_k, int32_t* n_blocks,
                         uint64_t* block_masks, int32_t* block_gates, int32_t max_blocks, double* matrices,
                         size_t matrices_len);

qk_status qk_batch_create(qk_dtype dtype, const qk_allocator* alloc, void* hip_stream, qk_batch* out);
qk_status qk_batch_destroy(qk_batch batch);
/* Validate and compile one circuit (ops copied); *job receives its index. */
qk_status qk_batch_add(qk_batch batch, int32_t n_qubits, int32_t n_cbits, const qk_op* ops, int32_t n_ops,
                       int32_t* job);
/* Run every circuit added so far (asynchronous, one launch).  Running again
 * without adding or clearing reuses the circuits already uploaded to the
 * device (the launch only resets the job queue). */
qk_status qk_batch_run(qk_batch batch);
qk_status qk_batch_sync(qk_batch batch);
/* Results of the last run (synchronise). */
qk_status qk_batch_get_state(qk_batch batch, int32_t job, void* host_out, size_t bytes);
qk_status qk_batch_read_cbits(qk_batch batch, int32_t job, uint8_t* out, int32_t n);
qk_status qk_batch_state_ptr(qk_batch batch, int32_t job, void** dev_ptr, size_t* bytes);
/* Where job `job` lives in the batch's buffers (host only, any time after
 * the job was added): byte offset and size of its state, offset of its
 * cbits (one byte each); the same layout as qk_batch_read_async's copies. */
qk_status qk_batch_layout(qk_batch batch, int32_t job, size_t* state_offset, size_t* state_bytes,
                          size_t* cbit_offset);
/* Enqueue (after the last qk_batch_run, on the batch's stream; no wait) the
 * copy of every job's final state and cbits into host buffers of at least
 * the batch's total sizes (pinned memory keeps it asynchronous).  For hosts
 * that must not wait on the device, such as a serving loop: the results are
 * there once the stream has reached this point (an event recorded after the
 * call has completed).  QK_E_STATE before a run. */
qk_status qk_batch_read_async(qk_batch batch, void* host_states, size_t state_bytes, uint8_t* host_cbits,
                              size_t cbit_bytes);
/* Forget every circuit (device buffers are kept for reuse). */
qk_status qk_batch_clear(qk_batch batch);
qk_status qk_batch_num_jobs(qk_batch batch, int32_t* n);
const char* qk_batch_last_error(qk_batch batch);

#ifdef __cplusplus
}
#endif

#endif /* QK_ABI_H_ */
