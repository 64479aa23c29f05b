// Internal declarations shared by the runtime (api.hip), the sweep kernels
// (kernels.hip), the matrix-core kernel (fused.hip) and the fusion planner
// (fusion.cpp).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <complex>
#include <cstdint>
#include <string>
#include <vector>

#include "qk.h"

namespace qk {

using cd = std::complex<double>;

constexpr int kMaxSpecial = 48;        // zero-insertion positions per launch (gate qubits + tile column bits)
constexpr int kBlock = 256;            // threads per block of the sweep kernels
constexpr int kReduceBlocks = 1024;    // fixed first-level reduction grid (max)
constexpr int kMeasLog = 4096;         // measurement log entries kept on device

// A measurement draw read from device memory cannot be checked by the host:
// NaN and negative draws count as 0, draws at or above 1 as the largest
// double below 1.  In [0, 1) the outcome u < P0 ? 0 : 1 always has positive
// probability when the state's norm is positive.
__device__ __forceinline__ double meas_draw(double u) {
  if (!(u >= 0.0)) return 0.0;
  if (!(u < 1.0)) return 0x1.fffffffffffffp-1;
  return u;
}

// Ascending bit positions at which zero bits are inserted into a compact
// counter to enumerate a subspace (the positions of targets, controls and,
// for the matrix-core kernel, column bits).
struct Special {
  int n;
  int pos[kMaxSpecial];
};

// Classical conditions, evaluated on the device at kernel start.
struct CondArgs {
  const uint8_t* cbits;
  int n;
  int cbit[QK_MAX_CONDS];
  int val[QK_MAX_CONDS];
};

// Dense matrix for the one-target butterfly: u00 u01 u10 u11 as (re, im).
struct Mat2 {
  double v[8];
};

// Diagonal of up to 6 target qubits (64 entries).
struct Diag64 {
  double v[128];
};

// Launch-shape choices (set per simulator; the autotuner sweeps them).  The
// defaults are the measured best on MI355X at 30 qubits for complex128; a
// complex64 simulator starts with diag_items, lane_items and sweep_items = 2
// (8-byte amplitudes want two per thread to keep 16 bytes per load in flight).
struct Tuning {
  int nt = 1;            // non-temporal sweeps: 0 never, 1 when accesses cover whole lines, 2 always
  int lane_bfly = 1;     // targets below bit 6 use the cross-lane butterfly
  int sweep_items = 1;   // amplitudes per thread in the strided butterfly, pairs per thread in the swap (1, 2 or 4)
  int diag_items = 1;    // amplitudes per thread in the diagonal and phase sweeps (1, 2 or 4)
  int lane_items = 1;    // 64-amplitude segments per wave in the cross-lane butterfly (1, 2 or 4)
  int mfma_waves = 8;    // waves per CU for the matrix-core kernel
  int mfma_cols = 32;    // tile columns per wave for the matrix-core kernel (16, 32, 64; capped per k)
  int mfma_areg = 0;     // blocks of 5-6 qubits: 1 keeps the A fragments in registers, 0 re-reads them from LDS
  int xcd = 1;           // sweeps: 1 renumbers workgroups so each XCD sweeps a contiguous range
  int diag_runs = 1;     // 1: consecutive diagonal gates are held back and applied in one pass
  int swap_relabel = 1;  // 1: an uncontrolled SWAP on a dense state relabels the two qubits instead of moving data
  int mfma_lds = 2;      // blocks of 4-5 qubits: 0 register tiles, 1 LDS-staged tiles, 2 chosen per block
  int lds_wg = 2;        // workgroups per CU of the LDS-staged kernel
  int stages = 0;        // 1: runs of builtin gates are held back and applied by stages through LDS chunks
};

// Where device work goes and what it works on.
struct Launch {
  hipStream_t stream;
  int n;           // qubits
  bool c64;        // complex64 (else complex128)
  void* psi;       // state
  CondArgs cond;
  Tuning tune;
};

// Non-temporal (streaming) accesses pay off only for states larger than the
// 256 MiB Infinity Cache.  A smaller state stays cached from one sweep to the
// next when sweeps use regular loads and stores: measured 9-17 % faster per
// sweep at 21-24 qubits (complex128), while at 25-26 qubits streaming is
// 3-7 % faster.
constexpr uint64_t kCachedStateBytes = 256ull << 20;
inline bool state_streams(const Launch& L) {
  return ((uint64_t)1 << L.n) * (L.c64 ? 8u : 16u) > kCachedStateBytes;
}

// Sorted, de-duplicated zero-insertion positions.
Special make_special(const int* a, int na, const int* b, int nb, const int* c = nullptr, int nc = 0);

// ---- sweep kernels (kernels.hip) ---------------------------------------------
hipError_t launch_fill_zero(void* p, uint64_t from, uint64_t to, bool c64, hipStream_t s);
hipError_t launch_set_one(void* p, uint64_t idx, bool c64, hipStream_t s);
hipError_t launch_copy(void* dst, const void* src, uint64_t count, bool c64, hipStream_t s);
hipError_t launch_butterfly(const Launch& L, int t, const int* controls, int nc, const Mat2& u);
hipError_t launch_diag(const Launch& L, const int* targets, int k, const int* controls, int nc, const Diag64& d);
hipError_t launch_phase_all1(const Launch& L, const int* bits, int nb, double zr, double zi);
hipError_t launch_swap(const Launch& L, int a, int b, const int* controls, int nc);

// Consecutive diagonal gates applied in one pass.  Term t acts on amplitude i
// when every bit of its qubit set (targets and controls, at most 6 qubits) that
// its mask requires is 1 and its classical conditions hold (evaluated on the
// device); it then multiplies a_i by d_t[m_t(i)], m_t(i) being the bit of i at
// its first target (k = 1), the bits at both targets (k = 2), or 0 (k = 0: one
// factor on the mask subspace).  The host packs the terms into groups whose
// qubit sets together span at most 6 bits; the kernel tabulates each group's
// combined factor over those bits (up to 64 entries) and multiplies an amplitude by
// one table entry per group.  The pass enumerates only the subspace where the
// `common` bits (required by every term) are 1.
constexpr int kDiagRunTerms = 24;
constexpr int kDiagRunConds = 32;
constexpr int kDiagRunGroups = 8;
constexpr int kDiagRunGroupBits = 6;
struct DiagRunTerm {
  uint8_t g;        // group
  uint8_t lmask;    // group-index bits that must all be 1
  int8_t k, l0, l1; // target count (0, 1, 2) and the targets' group-index bits
  uint8_t c0, c1;   // the term's conditions are entries [c0, c1) of the run's list
  uint8_t pad;
  double d[8];      // (re, im) of the factors for m = 0 .. 2^k - 1
};
struct DiagRunGroup {
  int8_t nb;                        // bits spanned
  int8_t pos[kDiagRunGroupBits];    // amplitude-index bit of group-index bit j
  int8_t pad;
};
struct DiagRunArgs {
  const uint8_t* cbits;
  int n;                            // terms
  int ng;                           // groups
  int ncond;                        // conditions
  int cb[kDiagRunConds];            // condition: cbit index ...
  uint8_t cv[kDiagRunConds];        // ... and the value it must hold
  DiagRunGroup grp[kDiagRunGroups];
  DiagRunTerm t[kDiagRunTerms];
};
// Device work space of a run: the group tables (complex, the state's
// precision, 64 entries per group) and, in its last 16 bytes, the word that
// says whether any term is active.
constexpr size_t kDiagRunTableBytes = (size_t)kDiagRunGroups * (1 << kDiagRunGroupBits) * 16 + 16;
hipError_t launch_diag_run(const Launch& L, const DiagRunArgs& run, const int* common, int ncommon, void* table);
hipError_t launch_dense_generic(const Launch& L, const int* targets, int k, const int* controls, int nc,
                                const void* d_matrix);
// mode 0: table d_finv; 1: affine x = Ainv (y - B) mod 2^k; 2: modular
// multiplication x = Ainv y mod N for y < N (identity above N, N < 2^32).
// out_of_place (no controls only): the permuted state is written to `scratch`
// (a whole second state buffer), which the caller then takes as the state;
// otherwise the controlled subspace goes through `scratch` and back.
hipError_t launch_perm(const Launch& L, void* scratch, const int* targets, int k, const int* controls, int nc,
                       const uint32_t* d_finv, int mode, uint64_t A, uint64_t B, uint64_t Ainv, uint64_t N,
                       bool out_of_place);

// Measurement: partial sums -> finalize (outcome, cbit, scale, log) -> collapse.
struct MeasBuffers {
  double* partials = nullptr;     // 2 * kReduceBlocks
  double* result = nullptr;       // p0, p1, scale, outcome
  double* log = nullptr;          // 3 * kMeasLog (nullptr: no log)
  uint32_t* log_count = nullptr;  // entries written so far
  uint8_t* cbits = nullptr;
  double* out = nullptr;          // if set: p0, p1, outcome
};
int reduce_blocks_for(uint64_t count);
hipError_t launch_measure(const Launch& L, int qubit, int cbit, double u, const double* d_u, int forced,
                          const MeasBuffers& mb);
// The same measurement with its scratch in a file-scope device array (no
// allocation); the outcome goes to d_cbit[0] and p0, p1, outcome to d_out
// (either may be NULL).  Calls that overlap on one device share the array.
hipError_t launch_measure_noalloc(int device, hipStream_t stream, void* psi, int n, bool c64, int qubit,
                                  const double* d_u, uint8_t* d_cbit, double* d_out);
hipError_t launch_inner_partials(const void* a, bool a64, const void* b, bool b64, uint64_t dim,
                                 double* partials, int nblocks, hipStream_t s);

// ---- deferred measurement (sample.hip) ---------------------------------------
// Shots drawn from the state without collapse: launch_cdf fills `work`
// (sample_layout(n).doubles FP64 values: segment sums, chunk sums, chunk
// prefix with the total last); launch_draw turns device uniforms into indices
// projected onto the listed qubits (nq = 0: the index itself).
struct SampleLayout {
  uint64_t nseg, nchunk, doubles;
};
SampleLayout sample_layout(int n);
hipError_t launch_cdf(const Launch& L, double* work);
hipError_t launch_draw(const Launch& L, const double* work, const int* qubits, int nq, const double* d_u,
                       uint64_t nshots, uint64_t* d_out);
// The same over an arbitrary amplitude array of `dim` entries (the sparse
// engine's amplitudes); draws are positions in that array (nq = 0 only).
SampleLayout sample_layout_dim(uint64_t dim);
hipError_t launch_cdf_dim(const void* psi, uint64_t dim, bool c64, hipStream_t s, double* work);
hipError_t launch_draw_dim(const void* psi, uint64_t dim, bool c64, hipStream_t s, const double* work,
                           const double* d_u, uint64_t nshots, uint64_t* d_out);
// Marginal distribution (unnormalised) of nq >= 1 listed qubits into d_out
// (2^nq doubles); `partial` holds marginal_layout(n, nq).partial_doubles.
struct MarginalLayout {
  uint64_t nrows, nslabs, partial_doubles;
  int slab_bits;
};
MarginalLayout marginal_layout(int n, int nq);
hipError_t launch_marginal(const Launch& L, const int* qubits, int nq, double* partial, double* d_out);

// ---- sparse state engine (sparse.hip) -------------------------------------------
// The state as nnz entries with ascending indices idx[] and amplitudes amp[];
// every array holds `cap` entries.  Operations that reorder or resize the
// state synchronise the stream once or twice to read entry counts back.
struct SpTargets {
  int k;
  int pos[64];
};
enum SpPermMode { SP_PERM_TABLE = 0, SP_PERM_AFFINE = 1, SP_PERM_MODMUL = 2, SP_PERM_SWAP = 3 };
struct SpBufs {
  uint64_t cap = 0, nnz = 0;
  uint64_t* idx = nullptr;     // the state: ascending indices
  void* amp = nullptr;         //            and their amplitudes
  uint64_t* idx_b = nullptr;   // spare pair
  void* amp_b = nullptr;
  uint64_t* key = nullptr;     // sort keys, gate outputs
  uint32_t* cnt = nullptr;     // per-entry counts or flags
  uint64_t* off = nullptr;     // their exclusive scan
  uint64_t* scal = nullptr;    // device scalars: [0] total, [1] exact-zero outputs, [2] keys out of order
  void* temp = nullptr;        // sort and scan work space
  size_t temp_bytes = 0;
};
size_t sp_temp_bytes(uint64_t cap, bool c64);
hipError_t sp_init(SpBufs& b, bool c64, hipStream_t st);
// Dense 2^k x 2^k gate (d_mat in the state's precision, row-major) on targets
// t, restricted to the entries whose bits in cmask are all 1.  Returns
// hipErrorOutOfMemory (state unchanged) if the result could exceed cap.
hipError_t sp_dense_gate(SpBufs& b, int n, bool c64, const SpTargets& t, uint64_t cmask, const void* d_mat,
                         hipStream_t st);
// Uncontrolled one-qubit gate u (row-major 2x2) on target t, by split and
// merges instead of sorts (same result as sp_dense_gate).
hipError_t sp_one_qubit(SpBufs& b, int n, bool c64, int t, const Mat2& u, hipStream_t st);
hipError_t sp_diag(SpBufs& b, bool c64, const SpTargets& t, uint64_t cmask, const Diag64& d, hipStream_t st);
// A run of diagonal gates of at most 2 targets, applied in order in one pass.
struct SpDiagTerm {
  int k;
  int pos[2];
  uint64_t cmask;
  double d[8];
};
constexpr int kSpDiagRun = 24;
struct SpDiagRun {
  int n;
  SpDiagTerm t[kSpDiagRun];
};
hipError_t sp_diag_run(SpBufs& b, bool c64, const SpDiagRun& run, hipStream_t st);
// Modular multiplication (mode SP_PERM_MODMUL) takes B = floor((2^64 - 1) / N).
hipError_t sp_permute(SpBufs& b, int n, bool c64, const SpTargets& t, uint64_t cmask, int mode, const uint32_t* ftab,
                      uint64_t A, uint64_t B, uint64_t N, hipStream_t st);
// Renumber index bits: bit j of every new index is bit phys.pos[j] of the old
// one (phys.k = n), then sort.
hipError_t sp_relabel(SpBufs& b, int n, bool c64, const SpTargets& phys, hipStream_t st);
hipError_t sp_measure(SpBufs& b, bool c64, int q, int cbit, double u, const double* d_u, int forced,
                      const MeasBuffers& mb, hipStream_t st);
hipError_t sp_norm_partials(const SpBufs& b, bool c64, double* partials, int nblocks, hipStream_t st);
hipError_t sp_project(const SpBufs& b, const uint64_t* pos, uint64_t nshots, const SpTargets& ql, uint64_t* d_out,
                      hipStream_t st);

// ---- matrix-core kernel (fused.hip) -----------------------------------------
// Dense 2^k x 2^k gate (2 <= k <= 6) on targets, restricted to controls = 1,
// as a complex GEMM per 16-column tile on 16x16x4 MFMA (f32 for complex64,
// f64 for complex128).  Needs at least 4 qubits outside targets and controls.
bool mfma_supported(int n, int k, int nc, bool c64);
// The same GEMM with workgroup tiles staged through LDS (global memory in
// address order, 1 KiB per wave access); blocks of 4 or 5 qubits.
bool mfma_lds_supported(int n, int k, const int* controls, int nc, bool c64);
bool mfma_lds_auto(int k, const int* targets, bool c64);
hipError_t launch_dense_lds(const Launch& L, const int* targets, int k, const int* controls, int nc,
                            const void* d_matrix, int wg_per_cu);
hipError_t launch_dense_mfma(const Launch& L, const int* targets, int k, const int* controls, int nc,
                             const void* d_matrix, int waves_per_cu);

// ---- builtin gates (api.hip) --------------------------------------------------
// Sweep class of a builtin gate and its FP64 data: BG_DENSE1 (2x2 matrix in m,
// row-major), BG_PHASE (factor z on the all-ones subspace of targets and
// controls), BG_DIAG (diagonal in m over the targets), BG_SWAP.
enum BuiltinClass { BG_DENSE1 = 1, BG_PHASE = 2, BG_DIAG = 3, BG_SWAP = 4 };
struct BuiltinGate {
  int cls = 0;
  std::vector<cd> m;
  cd z = 1.0;
};
bool builtin_info(int id, int* arity, int* nparams);
BuiltinGate builtin_gate(int id, double param);

// ---- fusion planner (fusion.cpp) --------------------------------------------
struct FGate {
  std::vector<int> qubits;   // ascending: union of targets and controls
  std::vector<cd> m;         // 2^q x 2^q, row-major, bit j <-> qubits[j]
  bool diag;
};
struct FBlock {
  std::vector<int> qubits;   // ascending
  std::vector<cd> m;         // 2^k x 2^k
  int ngates;
  bool diag;
  std::vector<int> members;  // indices of the gates composed, in application order
};
// Dense matrix on sorted(targets u controls) of a gate with matrix g on targets.
FGate make_fgate(const int* targets, int k, const int* controls, int nc, const std::vector<cd>& g);
// Greedy commutation-aware grouping into blocks of at most kmax qubits.
std::vector<FBlock> plan_blocks(const std::vector<FGate>& gates, int kmax);

// ---- the LDS-tile mode (batch.hip) ---------------------------------------------
// Held-back builtin gates (op records on physical qubits, n of them, cbit
// conditions below 256) compiled and grouped into stages of
// stage_chunk_qubits() qubits; recs is the device record image, headers the
// record index of each stage's header, in order.  launch_stage applies one
// stage to every chunk of the state (n from stage_chunk_qubits() to 31).
int stage_chunk_qubits(bool c64);
qk_status stage_plan(bool c64, int n, int ncbits, const std::vector<qk_op>& ops, std::vector<unsigned char>& recs,
                     std::vector<uint32_t>& headers, std::string& err);
void launch_stage(bool c64, void* psi, int n, const void* d_recs, uint32_t hrec, const uint8_t* d_cbits, int ncbits,
                  hipStream_t stream);

}  // namespace qk
