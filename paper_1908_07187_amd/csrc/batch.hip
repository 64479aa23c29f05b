// Batched execution: many circuits of uneven qubit counts in one persistent
// launch, and the stage kernel of the simulator's LDS-tile mode.
//
// Each circuit ("job") is compiled on the host into compact device records:
// builtin gates with their FP64 matrices, controls as a bit mask, up to two
// classical conditions, measurements with their pre-drawn uniform.  One-qubit,
// diagonal and phase gates are packed into passes: a pass names three target
// qubits and carries up to eleven gates whose dense targets are among them
// (diagonal and phase gates may act on any qubits).  One persistent grid
// runs all jobs: every workgroup takes the next job from a device counter
// (largest jobs first), builds |0...0> in LDS and runs the job's items one
// after another, a barrier after each.  In a pass every thread loads the 8
// amplitudes of its group (the 2^3 combinations of the pass's targets) from
// LDS, applies the pass's gates in registers and stores them back, so a pass
// costs one LDS round trip whatever its gate count; swaps and measurements
// run over the whole LDS state.  A job's state stays in LDS for its whole
// circuit, so a 12-qubit, 360-gate circuit costs one HBM write instead of 360
// sweeps and 360 launches.  Every workgroup leaves the loop once the counter
// passes the job count.
//
// Jobs too large for LDS (above 13 qubits complex128, 14 complex64; up to
// 24) run in the same launch with their state in global memory.  The host
// splits such a job into stages: runs of gates, reordered only where they
// commute, whose qubits fit one LDS chunk (12 qubits complex128, 13
// complex64), and measurements between them.  A stage's chunks (the
// amplitudes that share the values of the qubits outside the stage) are
// independent, so any free workgroup claims a run of them: it gathers each
// into LDS, runs the stage's items on it exactly as for a small job, and
// scatters it back; the workgroup that completes a stage's last chunk opens
// the next stage.  A stage costs one read and one write of the state
// whatever its gate count; a measurement runs over the state in global
// memory on one workgroup.  Workgroups take staged chunks first and small
// jobs when no chunk is free, and leave once every staged job has finished
// and the small-job counter has passed the job count.
//
// The simulator's LDS-tile mode (k_stage) runs one stage of a single state
// per launch with the same chunk code.
//
// Measurement inside a job uses the same rule as the per-gate path (FP64
// sums, outcome 0 iff u < P0, renormalise by 1/sqrt(p_outcome)), reduced in a
// fixed order that depends only on the job, so a job's result does not depend
// on which other jobs share the launch.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>
#include <string>
#include <vector>

#include "qk_internal.h"

using namespace qk;

namespace {

// One-qubit dense gates come in three kinds by their matrix: BK_X (the bit
// flip: a pair exchange, no arithmetic), BK_U1R (real entries: half the
// multiplications), BK_U1 (general complex).
enum BKind { BK_U1 = 1, BK_DIAG1 = 2, BK_DIAG2 = 3, BK_PHASE = 4, BK_SWAP = 5, BK_MEAS = 6, BK_PASS = 7, BK_X = 8,
             BK_U1R = 9, BK_STAGE = 10 };

__host__ __device__ constexpr bool is_one_qubit_dense(int kind) {
  return kind == BK_U1 || kind == BK_X || kind == BK_U1R;
}

struct BJob {
  uint64_t state_off;   // amplitudes
  uint32_t op_begin, op_end;   // record range of the job's items
  int32_t n, ncbits;
  uint32_t cbit_off;
  uint32_t st_begin, nst;   // staged jobs: their stages in the launch's stage table
  int32_t pad;
};

// One record, 20 dwords.  An item is one record (swap, measurement) or a pass
// header followed by its gate records.  BK_PASS header: head = kind | K << 8 |
// ngates << 16, cmask = target qubits of slots 0..K-1 (8 bits each), conds =
// the same qubits in ascending order, dwords 4..11 = the LDS byte offset of
// each of the 8 group members relative to the group base.  A gate inside a
// pass names its dense target by slot (head bits 8..15), other qubits by
// position; its cmask keeps only the controls off the pass's targets, and
// cbit holds the member bits the others need (bits 16..18) and, for a
// diagonal gate, each member's factor bits from pass targets (2 bits per
// member, bits 0..15).
struct BOp {
  uint32_t head;    // kind | t0 << 8 | t1 << 16 | ncond << 24
  uint32_t cmask;   // control mask (BK_PHASE: the all-ones mask of targets and controls)
  uint32_t conds;   // cb0 | cv0 << 8 | cb1 << 16 | cv1 << 24
  int32_t cbit;     // BK_MEAS: cbit receiving the outcome, or -1
  double m[8];      // BK_U1: 2x2 matrix row-major (re, im); BK_DIAG*: diagonal; BK_PHASE: factor; BK_MEAS: m[0] = u
};
static_assert(sizeof(BOp) == 80, "op record layout");
constexpr int kOpWords = (int)(sizeof(BOp) / 4);
constexpr int kPassGates = 11;                 // gates per pass at most
constexpr int kPassSlots = 3;                  // target qubits of every pass (8 amplitudes per group)
constexpr int kItemWords = 4 * 64;             // dwords an item read brings in (>= (1 + kPassGates) * kOpWords)
static_assert((1 + kPassGates) * kOpWords <= kItemWords, "an item fits one read");
constexpr int kPadRecords = kItemWords / kOpWords + 1;   // zero records after the last job, so item reads stay in bounds

constexpr int kBatchThreads = 512;
constexpr int kMaxJobCbits = 256;
// Items per thread whose LDS reads are issued together in the whole-state
// loops (swap, measurement).
constexpr int kBU = 2;

typedef uint32_t QkU4 __attribute__((ext_vector_type(4)));

template <typename R> struct EVb;
template <> struct EVb<float> { typedef float T __attribute__((ext_vector_type(2))); };
template <> struct EVb<double> { typedef double T __attribute__((ext_vector_type(2))); };

__device__ __forceinline__ double bwave_sum(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// An item's records (at most kItemWords dwords) are read from global memory
// one item ahead, lane l of every wave holding dwords l, 64 + l, 128 + l and
// 192 + l; wave 0 copies them into one of two LDS buffers before the barrier
// that ends the current item, and the next item reads its fields from there
// as broadcast LDS loads (all lanes read the same address).
struct ItemRegs {
  uint32_t w[kItemWords / 64];
};

__device__ __forceinline__ ItemRegs load_item(const uint32_t* __restrict__ opw, uint32_t rec, int lane) {
  const uint32_t* p = opw + (size_t)rec * kOpWords;
  ItemRegs it;
#pragma unroll
  for (int j = 0; j < kItemWords / 64; ++j) it.w[j] = p[64 * j + lane];
  return it;
}

__device__ __forceinline__ void stage_item(uint32_t* buf, const ItemRegs& it, int lane) {
#pragma unroll
  for (int j = 0; j < kItemWords / 64; ++j) buf[64 * j + lane] = it.w[j];
}

__device__ __forceinline__ double ldbl(const uint32_t* buf, int d) {
  const uint64_t lo = buf[d], hi = buf[d + 1];
  return __longlong_as_double((long long)(lo | (hi << 32)));
}

__device__ __forceinline__ uint32_t ins0(uint32_t p, uint32_t q) { return ((p >> q) << (q + 1)) | (p & ((1u << q) - 1)); }

// LDS position of amplitude i.  A pass whose targets include the lowest
// qubits gives consecutive lanes groups 8 (or more) amplitudes apart, all in
// the same banks; XOR-ing the next bits into the position within a 128-byte
// row (3 bits for 16-byte amplitudes, 4 for 8-byte) spreads them, and keeps
// contiguous runs contiguous within each row.  A bijection on [0, 2^n).
template <typename R>
__device__ __forceinline__ uint32_t swz(uint32_t i) {
  constexpr uint32_t b = sizeof(R) == 8 ? 3 : 4, m = (1u << b) - 1;
  return i ^ ((i >> b) & m);
}

template <typename R>
__device__ __forceinline__ typename EVb<R>::T cmul(R ar, R ai, typename EVb<R>::T x) {
  typename EVb<R>::T r;
  r.x = ar * x.x - ai * x.y;
  r.y = ar * x.y + ai * x.x;
  return r;
}

// Pair (lo, hi) of a group under a one-qubit gate: [x_lo, x_hi] <- U [x_lo, x_hi]
// where every control bit of the pair's index is 1.  KIND selects the form:
// general complex U, real U (u holds the four real entries in u[0], u[2],
// u[4], u[6]), or the bit flip.
// The 2x2 matrix (re, im interleaved), passed by value so that it stays in
// registers (a pointer to a local array puts the array in scratch memory).
template <typename R> struct U2 {
  R v[8];
};

template <typename R, int KIND>
__device__ __forceinline__ void bfly(typename EVb<R>::T& p, typename EVb<R>::T& q, bool act, const U2<R> m) {
  const R* u = m.v;
  if (!act) return;
  typename EVb<R>::T r0, r1;
  if constexpr (KIND == BK_X) {
    r0 = q;
    r1 = p;
  } else if constexpr (KIND == BK_U1R) {
    r0.x = u[0] * p.x + u[2] * q.x;
    r0.y = u[0] * p.y + u[2] * q.y;
    r1.x = u[4] * p.x + u[6] * q.x;
    r1.y = u[4] * p.y + u[6] * q.y;
  } else {
    r0.x = u[0] * p.x - u[1] * p.y + u[2] * q.x - u[3] * q.y;
    r0.y = u[0] * p.y + u[1] * p.x + u[2] * q.y + u[3] * q.x;
    r1.x = u[4] * p.x - u[5] * p.y + u[6] * q.x - u[7] * q.y;
    r1.y = u[4] * p.y + u[5] * p.x + u[6] * q.y + u[7] * q.x;
  }
  p = r0;
  q = r1;
}

// The pairs of a group that differ in slot `a` (the gate's target), updated
// by bfly<R, KIND> when the pair's member number has the bits of rmask set
// (its controls among the pass's targets: a uniform test) and ACT holds (the
// lane's controls outside them).  Expanded in the kernel body on the
// kernel's own register array with constant indices: passing the array to a
// function (by reference) made the compiler keep part of it in scratch
// memory.
#define QK_PASS_GATE(KIND, U, ACT, RMASK)                                               \
  do {                                                                                  \
    if (a == 0) {                                                                       \
      _Pragma("unroll") for (int r = 0; r < 8; r += 2)                                  \
        if ((r & (RMASK)) == (RMASK)) bfly<R, KIND>(x[r], x[r + 1], ACT, U);              \
    } else if (a == 1) {                                                                \
      _Pragma("unroll") for (int r = 0; r < 8; ++r)                                     \
        if (!(r & 2) && (r & (RMASK)) == (RMASK))                                        \
          bfly<R, KIND>(x[r], x[r + 2], ACT, U);                                        \
    } else {                                                                            \
      _Pragma("unroll") for (int r = 0; r < 4; ++r)                                     \
        if ((r & (RMASK)) == (RMASK)) bfly<R, KIND>(x[r], x[r + 4], ACT, U);              \
    }                                                                                   \
  } while (0)

// A diagonal or phase gate on every member of the group: member r takes
// factor k = kb | (its bits at the gate's qubits among the pass's targets),
// a 16-byte read at the lane's record address fb plus a uniform offset.
#define QK_PASS_DIAG(ACT, RMASK)                                                        \
  do {                                                                                  \
    _Pragma("unroll") for (int r = 0; r < 8; ++r) {                                     \
      if ((r & (RMASK)) == (RMASK)) {                                                  \
        const uint32_t kr = (aux >> (2 * r)) & 3u;                                     \
        const typename EVb<double>::T f = *reinterpret_cast<const typename EVb<double>::T*>(fb + 4 * kr); \
        const C p = cmul<R>((R)f.x, (R)f.y, x[r]);                                      \
        x[r] = (ACT) ? p : x[r];                                                        \
      }                                                                                 \
    }                                                                                   \
  } while (0)

// Waves per SIMD to keep resident: complex128, two 512-thread workgroups per
// CU (the most the 64 KiB states of 12-qubit jobs allow in LDS); complex64,
// four (32 KiB states).
template <typename R> constexpr int batch_waves_per_simd() { return sizeof(R) == 8 ? 4 : 8; }

// Staged (mid-size) jobs: qubits of the LDS chunk a stage works on, and the
// amplitudes each thread moves per chunk.
template <typename R> constexpr int stage_qubits() { return sizeof(R) == 8 ? 12 : 13; }
template <typename R> constexpr int stage_per_thread() { return (1 << stage_qubits<R>()) / kBatchThreads; }
// Records of a stage kept in LDS beside its chunk by the stage kernel (12 KiB:
// 153 records; two workgroups of 64 + 12 KiB and their static arrays fit a
// compute unit).
constexpr uint32_t kStageLdsWords = 3072;
// The stage kernel's residency: two workgroups per CU (the LDS they hold
// allows no more), so four waves per SIMD and 128 registers per lane for
// either amplitude type.
constexpr int kStageWavesPerSimd = 4;
static_assert(stage_per_thread<double>() % 8 == 0 && stage_per_thread<float>() % 8 == 0, "chunk moves go 8 at a time");
static_assert(kBatchThreads == 512, "a staged chunk maps the thread to the stage's lowest 9 qubits");

// Measurement of qubit mask qb over a state of dim amplitudes (in LDS, read
// through the swizzle, or the job's state in global memory): FP64 sums of
// |x|^2 by outcome in a fixed order (thread-strided, then wave, then the
// waves in order), outcome 0 iff u < P0, the outcome's half scaled by
// 1/sqrt(p), the other half zeroed; cbit (>= 0) receives the outcome.  A
// zero-probability outcome leaves the state and the cbit as they are.
template <typename R, bool LDS>
__device__ __forceinline__ void meas_run(typename EVb<R>::T* st, uint32_t dim, uint32_t qb, double u, int cbit,
                                         uint8_t* cb, double (*red)[kBatchThreads / 64], double* meas) {
  using C = typename EVb<R>::T;
  const uint32_t tid = threadIdx.x, bd = blockDim.x;
  const int lane = tid & 63, w = tid >> 6;
  auto at = [](uint32_t i) { return LDS ? swz<R>(i) : i; };
  double s0 = 0, s1 = 0;
  for (uint32_t i0 = tid; i0 < dim; i0 += kBU * bd) {
    C x[kBU];
#pragma unroll
    for (int k = 0; k < kBU; ++k)
      if (i0 + k * bd < dim) x[k] = st[at(i0 + k * bd)];
#pragma unroll
    for (int k = 0; k < kBU; ++k) {
      const uint32_t i = i0 + k * bd;
      if (i < dim) {
        const double pr = (double)x[k].x * (double)x[k].x + (double)x[k].y * (double)x[k].y;
        if (i & qb) s1 += pr; else s0 += pr;
      }
    }
  }
  s0 = bwave_sum(s0);
  s1 = bwave_sum(s1);
  if (lane == 0) {
    red[0][w] = s0;
    red[1][w] = s1;
  }
  __syncthreads();
  if (tid == 0) {
    double q0 = 0, q1 = 0;
    for (int k = 0; k < (int)(bd / 64); ++k) {
      q0 += red[0][k];
      q1 += red[1][k];
    }
    const double P0 = q0 / (q0 + q1);
    const int oc = (u < P0) ? 0 : 1;
    const double po = oc ? q1 : q0;
    meas[0] = po > 0 ? 1.0 / sqrt(po) : 0.0;
    meas[1] = (double)oc;
    if (cbit >= 0 && po > 0) cb[cbit] = (uint8_t)oc;
  }
  __syncthreads();
  const double sc = meas[0];
  const uint32_t oc = (uint32_t)meas[1];
  if (sc != 0.0) {
    const R scale = (R)sc;
    for (uint32_t i0 = tid; i0 < dim; i0 += kBU * bd) {
      C x[kBU];
#pragma unroll
      for (int k = 0; k < kBU; ++k)
        if (i0 + k * bd < dim) x[k] = st[at(i0 + k * bd)];
#pragma unroll
      for (int k = 0; k < kBU; ++k) {
        const uint32_t i = i0 + k * bd;
        if (i < dim) {
          C v = x[k];
          if (((i & qb) != 0) == (oc != 0)) {
            v.x *= scale;
            v.y *= scale;
          } else {
            v.x = 0;
            v.y = 0;
          }
          st[at(i)] = v;
        }
      }
    }
  }
}

// Runs items [rec, end) over a state of dim amplitudes in LDS.  The first
// item's records must already sit in items[0], staged before a barrier; every
// item ends with a barrier.
// Where run_items reads the records: a double-buffered LDS copy of each
// item staged one item ahead (REC_STAGED), a copy of the whole range in LDS
// (REC_LDS), or global memory at a uniform address, which the compiler turns
// into scalar loads (REC_SCALAR).
enum { REC_STAGED = 0, REC_LDS = 1, REC_SCALAR = 2 };

template <typename R, int RM = REC_STAGED>
__device__ __forceinline__ void run_items(typename EVb<R>::T* st, uint32_t dim, uint32_t rec, uint32_t end,
                                          const uint32_t* __restrict__ opw, uint8_t* cb,
                                          uint32_t (*items)[kItemWords], double (*red)[kBatchThreads / 64],
                                          double* meas, const uint32_t* lrec = nullptr, uint32_t lbase = 0) {
  using C = typename EVb<R>::T;
  constexpr bool LREC = RM != REC_STAGED;
  const uint32_t tid = threadIdx.x, bd = blockDim.x;
  const int lane = tid & 63, w = tid >> 6;
  int buf = 0;
  while (rec < end) {
    const uint32_t* cur = RM == REC_SCALAR ? opw + (size_t)rec * kOpWords
                        : (RM == REC_LDS ? lrec + (size_t)(rec - lbase) * kOpWords : items[buf]);
    const uint32_t head = __builtin_amdgcn_readfirstlane(cur[0]);
    const int kind = head & 0xff;
    const int ngates = kind == BK_PASS ? (int)((head >> 16) & 0xff) : 0;
    const uint32_t next = rec + 1 + (uint32_t)ngates;
    ItemRegs nxt;   // (unused when the records are in LDS: no registers to clear)
    if constexpr (!LREC) {
      if (w == 0) nxt = load_item(opw, next, lane);   // the record array ends with padding
    }
    if (kind == BK_PASS) {
      // every pass has three slots (the host fills them with qubits above
      // the job's own for jobs of one or two qubits, whose groups then run
      // into the padding of an LDS state of at least 8 amplitudes), so the
      // member tests below are compile-time constants
      constexpr int K = kPassSlots, G = 1 << K;
      const uint32_t sw = __builtin_amdgcn_readfirstlane(cur[2]);
      const uint32_t p0 = sw & 0xff, p1 = (sw >> 8) & 0xff, p2 = (sw >> 16) & 0xff;
      // member r of a group sits at LDS byte offset swz(base) * sizeof(C) ^
      // off[r]: the swizzle is linear over XOR and the group base has zeros
      // at the pass's targets, so the host gives each member's part once
      uint32_t off[G];
#pragma unroll
      for (int r = 0; r < G; ++r) off[r] = __builtin_amdgcn_readfirstlane(cur[4 + r]);
      unsigned char* const sp = reinterpret_cast<unsigned char*>(st);
      const uint32_t ngroups = dim >= (uint32_t)G ? dim >> K : 1u;
      for (uint32_t g = tid; g < ngroups; g += bd) {
        const uint32_t base = ins0(ins0(ins0(g, p0), p1), p2);
        const uint32_t sb = swz<R>(base) * (uint32_t)sizeof(C);
        C x[8];
#pragma unroll
        for (int r = 0; r < 8; ++r) x[r] = *reinterpret_cast<const C*>(sp + (sb ^ off[r]));
        // complex128: a gate's first four dwords (head, cmask, conds, aux)
        // are read one gate ahead, so their LDS latency overlaps the previous
        // gate's work (complex64, whose kernel keeps twice the waves within
        // half the registers, was slower so)
        constexpr bool kAhead = sizeof(R) == 8;
        QkU4 hn{};
        if (kAhead) hn = *reinterpret_cast<const QkU4*>(cur + kOpWords);
        for (int o = 1; o <= ngates; ++o) {
          const uint32_t* g0 = cur + o * kOpWords;
          QkU4 hc;
          if (kAhead) {
            hc = hn;
            if (o < ngates) hn = *reinterpret_cast<const QkU4*>(g0 + kOpWords);
          } else {
            hc = *reinterpret_cast<const QkU4*>(g0);
          }
          const uint32_t oh = __builtin_amdgcn_readfirstlane(hc.x);
          const int okind = oh & 0xff, ncond = oh >> 24;
          const uint32_t a = (oh >> 8) & 0xff, b = (oh >> 16) & 0xff;
          if (ncond > 0) {
            const uint32_t cw = __builtin_amdgcn_readfirstlane(hc.z);
            if ((uint32_t)__builtin_amdgcn_readfirstlane(cb[cw & 0xff]) != ((cw >> 8) & 0xff)) continue;
            if (ncond > 1 && (uint32_t)__builtin_amdgcn_readfirstlane(cb[(cw >> 16) & 0xff]) != (cw >> 24)) continue;
          }
          // the host split the controls into those on the pass's targets
          // (rmask: the member bits they need, a uniform test per member)
          // and the rest (cout: the same for the whole group, one test per
          // lane); with neither, no tests at all
          const uint32_t cout = __builtin_amdgcn_readfirstlane(hc.y);
          const uint32_t aux = __builtin_amdgcn_readfirstlane(hc.w);
          const int rmask = (int)((aux >> 16) & 7u);
          const bool plain = cout == 0u && rmask == 0;
          const bool gact = (base & cout) == cout;
          if (okind == BK_X) {
            if (plain) QK_PASS_GATE(BK_X, U2<R>{}, true, 0);
            else QK_PASS_GATE(BK_X, U2<R>{}, gact, rmask);
          } else if (okind == BK_U1R) {
            U2<R> u{};
#pragma unroll
            for (int e = 0; e < 8; e += 2) u.v[e] = (R)ldbl(g0, 4 + 2 * e);
            if (plain) QK_PASS_GATE(BK_U1R, u, true, 0);
            else QK_PASS_GATE(BK_U1R, u, gact, rmask);
          } else if (okind == BK_U1) {
            U2<R> u;
#pragma unroll
            for (int e = 0; e < 8; ++e) u.v[e] = (R)ldbl(g0, 4 + 2 * e);
            if (plain) QK_PASS_GATE(BK_U1, u, true, 0);
            else QK_PASS_GATE(BK_U1, u, gact, rmask);
          } else {
            // BK_DIAG1 / BK_DIAG2 on qubits a (, b); BK_PHASE: one factor where
            // every control bit is 1.  Factor k = 2 m1 + m0 (two doubles at
            // dwords 4 + 4k of the record, in LDS): the bits of the lane's
            // group base give kb (zero at pass targets), the member's bits
            // at pass targets the rest (2 bits per member in aux).
            const uint32_t s0 = okind == BK_PHASE ? 31u : a, s1 = okind == BK_DIAG2 ? b : 31u;
            const uint32_t kb = ((base >> s0) & 1u) | (((base >> s1) & 1u) << 1);
            const uint32_t* fb = g0 + 4 + 4 * kb;
            if (plain) QK_PASS_DIAG(true, 0);
            else QK_PASS_DIAG(gact, rmask);
          }
        }
#pragma unroll
        for (int r = 0; r < 8; ++r) *reinterpret_cast<C*>(sp + (sb ^ off[r])) = x[r];
      }
    } else if (kind == BK_SWAP) {
      // quarter-space enumeration: bit t0 set, bit t1 clear, exchanged with the mirror
      const uint32_t t0 = (head >> 8) & 0xff, t1 = (head >> 16) & 0xff, cm = __builtin_amdgcn_readfirstlane(cur[1]);
      const uint32_t ab = 1u << t0, bb = 1u << t1, q = dim >> 2;
      const uint32_t plo = t0 < t1 ? t0 : t1, phi = t0 < t1 ? t1 : t0;
      bool ok = true;
      const int ncond = head >> 24;
      if (ncond > 0) {
        const uint32_t cw = __builtin_amdgcn_readfirstlane(cur[2]);
        if (cb[cw & 0xff] != (uint8_t)((cw >> 8) & 0xff)) ok = false;
        if (ncond > 1 && cb[(cw >> 16) & 0xff] != (uint8_t)(cw >> 24)) ok = false;
      }
      if (ok) {
        for (uint32_t p0 = tid; p0 < q; p0 += kBU * bd) {
          C x[kBU], y[kBU];
          uint32_t ia[kBU];
#pragma unroll
          for (int k = 0; k < kBU; ++k) {
            const uint32_t pp = p0 + k * bd;
            ia[k] = ins0(ins0(pp, plo), phi) | ab;
            if (pp < q) {
              x[k] = st[swz<R>(ia[k])];
              y[k] = st[swz<R>(ia[k] ^ ab ^ bb)];
            }
          }
#pragma unroll
          for (int k = 0; k < kBU; ++k) {
            if (p0 + k * bd < q && (ia[k] & cm) == cm) {
              st[swz<R>(ia[k])] = y[k];
              st[swz<R>(ia[k] ^ ab ^ bb)] = x[k];
            }
          }
        }
      }
    } else if (kind == BK_MEAS) {
      meas_run<R, true>(st, dim, 1u << ((head >> 8) & 0xff), ldbl(cur, 4), (int)cur[3], cb, red, meas);
    }
    // the next item's records into the other buffer (its last readers
    // finished before the barrier that ended the previous item)
    if constexpr (!LREC) {
      if (w == 0) stage_item(items[buf ^ 1], nxt, lane);
    }
    __syncthreads();
    buf ^= 1;
    rec = next;
  }
}

// Bits of v deposited, lowest first, at the set bits of mask.
__device__ __forceinline__ uint32_t deposit(uint32_t v, uint32_t mask) {
  uint32_t out = 0;
  for (uint32_t m = mask; m; m &= m - 1, v >>= 1)
    if (v & 1u) out |= m & (~m + 1u);
  return out;
}

// The chunk layout of a stage whose header record is h (record index rec):
// its item range, the qubits outside it (cmask: where the chunk number goes),
// and this thread's part of the local index.  Local index tid + k * 512: its
// low 9 bits (the thread) land on the stage's lowest 9 qubits, k on the
// others (the same for every thread).
struct ChunkMap {
  uint32_t it_begin, it_end, cmask, shigh, base;
};

template <int LQ>
__device__ __forceinline__ ChunkMap chunk_map(const uint32_t* h, uint32_t rec, uint32_t dim, uint32_t tid) {
  ChunkMap m;
  m.it_begin = rec + 1;
  m.it_end = m.it_begin + (uint32_t)__builtin_amdgcn_readfirstlane(h[1]);
  uint32_t smask = 0;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const uint32_t wq = (uint32_t)__builtin_amdgcn_readfirstlane(h[4 + q]);
#pragma unroll
    for (int e = 0; e < 4; ++e)
      if (4 * q + e < LQ) smask |= 1u << ((wq >> (8 * e)) & 0xff);
  }
  m.cmask = (dim - 1) & ~smask;
  uint32_t slow = 0, shigh = smask;
  for (int e = 0; e < 9; ++e) {
    slow |= shigh & (~shigh + 1u);
    shigh &= shigh - 1;
  }
  m.shigh = shigh;
  m.base = deposit(tid, slow);
  return m;
}

// One chunk of a stage: gathered from the state into LDS (or, with zero,
// made |0...0>'s slice), the stage's items run on it, scattered back.
// Starts after and ends with a barrier.
template <typename R, int RM = REC_STAGED>
__device__ __forceinline__ void stage_chunk(typename EVb<R>::T* st, typename EVb<R>::T* gst, const ChunkMap& cm,
                                            uint32_t ch, bool zero, const uint32_t* __restrict__ opw, uint8_t* cb,
                                            uint32_t (*items)[kItemWords], double (*red)[kBatchThreads / 64],
                                            double* meas, const uint32_t* lrec = nullptr) {
  using C = typename EVb<R>::T;
  constexpr int LQ = stage_qubits<R>(), PT = stage_per_thread<R>();
  const uint32_t tid = threadIdx.x, bd = blockDim.x;
  const int lane = tid & 63, w = tid >> 6;
  const uint32_t cpart = deposit(ch, cm.cmask);
  if (RM == REC_STAGED && w == 0) stage_item(items[0], load_item(opw, cm.it_begin, lane), lane);
#pragma unroll 1
  for (int k0 = 0; k0 < PT; k0 += 8) {   // 8 loads in flight per thread
    C x[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const uint32_t g = cm.base | deposit((uint32_t)(k0 + k), cm.shigh) | cpart;
      if (zero) {
        x[k].x = g == 0 ? (R)1 : (R)0;
        x[k].y = 0;
      } else {
        x[k] = gst[g];
      }
    }
#pragma unroll
    for (int k = 0; k < 8; ++k) st[swz<R>(tid + (uint32_t)(k0 + k) * bd)] = x[k];
  }
  __syncthreads();
  run_items<R, RM>(st, 1u << LQ, cm.it_begin, cm.it_end, opw, cb, items, red, meas, lrec, cm.it_begin);
#pragma unroll 1
  for (int k0 = 0; k0 < PT; k0 += 8)
#pragma unroll
    for (int k = 0; k < 8; ++k)
      gst[cm.base | deposit((uint32_t)(k0 + k), cm.shigh) | cpart] = st[swz<R>(tid + (uint32_t)(k0 + k) * bd)];
  __syncthreads();   // the next chunk's gather overwrites LDS
}

// Scheduling state of a batch launch.  Staged jobs: per job a 64-bit word
// (current stage << 32 | chunks claimed in it), the chunks completed in the
// current stage and a finished flag.  sched[0]: every staged job below it has
// finished (a scan hint); sched[1]: small jobs taken; sched[2]: set when a
// workgroup found no work for stall_ticks of the wall clock, 10 s (the host
// reports it).
struct BStage {
  uint32_t rec;       // record of the stage header or measurement
  uint32_t nchunks;   // chunks of the stage (1 for a measurement)
};
struct JobCtl {
  unsigned long long word;
  unsigned int done;
  unsigned int finished;
};
constexpr uint32_t kScanWindow = 128;                   // staged jobs a workgroup looks at for a free chunk

__device__ __forceinline__ unsigned ld_acq(const unsigned* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ unsigned long long ld_acq64(const unsigned long long* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Where the small jobs' records come from.
// Staged one item ahead: reading the records as scalar loads from global
// memory instead measured 8-11 % slower (2048 12-qubit circuits) and 6 %
// slower on mid-size staged jobs.
constexpr int RM_SMALL = REC_STAGED;

template <typename R>
__global__ __launch_bounds__(kBatchThreads, batch_waves_per_simd<R>()) void k_batch(
    const BJob* __restrict__ jobs, int njobs, int nstaged, const BStage* __restrict__ stages, JobCtl* ctl,
    unsigned* sched, const uint32_t* __restrict__ opw, typename EVb<R>::T* __restrict__ states,
    uint8_t* __restrict__ cbits, unsigned long long stall_ticks, uint32_t run_max) {
  using C = typename EVb<R>::T;
  constexpr int LQ = stage_qubits<R>();
  extern __shared__ __align__(16) unsigned char smem_raw[];
  C* st = reinterpret_cast<C*>(smem_raw);
  __shared__ uint8_t cb[kMaxJobCbits];
  __shared__ double red[2][kBatchThreads / 64];
  __shared__ double meas[2];
  __shared__ int task[5];
  __shared__ __align__(16) uint32_t items[2][kItemWords];
  const uint32_t tid = threadIdx.x, bd = blockDim.x;
  const int lane = tid & 63, w = tid >> 6;
  unsigned long long idle_since = 0;
  for (;;) {
    // ---- find work (wave 0): a free chunk of a staged job, oldest first,
    // 64 jobs looked at per load round; else the next small job; else wait
    // for the stages in flight, or leave once every staged job has finished
    if (w == 0) {
      int job = -1, stage = 0, chunk = 0, count = 1, status = 0;   // status 0: work, 1: wait, 2: leave
      const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane(ld_acq(&sched[0]));
      for (uint32_t b0 = lo; job < 0 && b0 < (uint32_t)nstaged && b0 < lo + kScanWindow; b0 += 64) {
        const uint32_t j = b0 + lane;
        bool fin = true, avail = false;
        if (j < (uint32_t)nstaged) {
          fin = ld_acq(&ctl[j].finished) != 0;
          if (!fin) {
            const BJob& jb = jobs[j];
            const unsigned long long wd = ld_acq64(&ctl[j].word);
            const uint32_t s0 = (uint32_t)(wd >> 32);
            avail = s0 < jb.nst && (uint32_t)wd < stages[jb.st_begin + s0].nchunks;
          }
        }
        const unsigned long long fm = __ballot(fin);
        if (b0 == lo && (fm & 1ull)) {   // a finished prefix: move the hint past it
          const uint32_t np = ~fm == 0 ? 64u : (uint32_t)__builtin_ctzll(~fm);
          if (lane == 0) atomicMax(&sched[0], b0 + np);
        }
        unsigned long long av = __ballot(avail);
        while (av) {
          const int l = __builtin_ctzll(av);
          int got = 0, s2 = 0, c2 = 0, cnt = 0;
          if (lane == l) {
            // a run of chunks per claim: fewer claims and fences on large stages
            const BJob& jb = jobs[j];
            const uint32_t nck = stages[jb.st_begin + (uint32_t)(ld_acq64(&ctl[j].word) >> 32) % jb.nst].nchunks;
            const uint32_t want = min(run_max, max(1u, nck >> 4));
            const unsigned long long old = atomicAdd(&ctl[j].word, (unsigned long long)want);
            s2 = (int)(old >> 32);
            c2 = (int)(uint32_t)old;
            if ((uint32_t)s2 < jb.nst) {
              const uint32_t n2 = stages[jb.st_begin + s2].nchunks;
              got = (uint32_t)c2 < n2;
              cnt = got ? (int)min(want, n2 - (uint32_t)c2) : 0;
            }
          }
          if (__ballot(got)) {
            job = (int)(b0 + l);
            stage = __shfl(s2, l, 64);
            chunk = __shfl(c2, l, 64);
            count = __shfl(cnt, l, 64);
            break;
          }
          av &= av - 1;
        }
      }
      if (job >= 0) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");   // pairs with the release that opened the stage
      if (lane == 0) {
        if (job < 0 && ld_acq(&sched[1]) < (unsigned)(njobs - nstaged)) {
          const unsigned q = atomicAdd(&sched[1], 1u);
          if (q < (unsigned)(njobs - nstaged)) job = nstaged + (int)q;
        }
        if (job < 0) {
          if (ld_acq(&sched[0]) >= (unsigned)nstaged) {
            status = 2;
          } else {
            const unsigned long long t = wall_clock64();
            if (idle_since == 0) idle_since = t;
            if (t - idle_since > stall_ticks) {
              atomicOr(&sched[2], 1u);
              status = 2;
            } else {
              status = 1;
            }
          }
        } else {
          idle_since = 0;
        }
        task[0] = job;
        task[1] = stage;
        task[2] = chunk;
        task[3] = status;
        task[4] = count;
      }
    }
    __syncthreads();
    const int job = __builtin_amdgcn_readfirstlane(task[0]);
    const uint32_t stage = (uint32_t)__builtin_amdgcn_readfirstlane(task[1]);
    const uint32_t chunk = (uint32_t)__builtin_amdgcn_readfirstlane(task[2]);
    const int status = __builtin_amdgcn_readfirstlane(task[3]);
    const uint32_t count = (uint32_t)__builtin_amdgcn_readfirstlane(task[4]);
    __syncthreads();   // task[] is rewritten by the next search
    if (status == 2) break;
    if (status == 1) {
      __builtin_amdgcn_s_sleep(8);
      continue;
    }
    const BJob jb = jobs[job];
    const uint32_t dim = 1u << jb.n;
    C* gst = states + jb.state_off;
    if (job >= nstaged) {
      // ---- a small job: |0...0> in LDS, every item, written out once
      for (int c = tid; c < jb.ncbits; c += bd) cb[c] = 0;
      if (RM_SMALL == REC_STAGED && w == 0) stage_item(items[0], load_item(opw, jb.op_begin, lane), lane);
      for (uint32_t i = tid; i < dim; i += bd) {
        C z;
        z.x = (i == 0) ? (R)1 : (R)0;
        z.y = 0;
        st[swz<R>(i)] = z;
      }
      __syncthreads();
      run_items<R, RM_SMALL>(st, dim, jb.op_begin, jb.op_end, opw, cb, items, red, meas);
      for (uint32_t i = tid; i < dim; i += bd) gst[i] = st[swz<R>(i)];
      for (int c = tid; c < jb.ncbits; c += bd) cbits[jb.cbit_off + c] = cb[c];
      __syncthreads();
      continue;
    }
    // ---- a run of chunks of a stage (or a measurement) of a staged job.
    // Wave 0 acquired after its claim (the invalidation covers this compute
    // unit's caches), and the barrier above orders every wave after it, so
    // every chunk of the earlier stages, written by any workgroup, is visible.
    const BStage bs = stages[jb.st_begin + stage];
    for (int c = tid; c < jb.ncbits; c += bd) cb[c] = cbits[jb.cbit_off + c];
    __syncthreads();
    const uint32_t* h = opw + (size_t)bs.rec * kOpWords;
    const uint32_t head = __builtin_amdgcn_readfirstlane(h[0]);
    if ((head & 0xff) == BK_MEAS) {
      // readfirstlane returns a signed int: widen through uint32_t
      const uint64_t ulo = (uint32_t)__builtin_amdgcn_readfirstlane(h[4]);
      const uint64_t uhi = (uint32_t)__builtin_amdgcn_readfirstlane(h[5]);
      const double u = __longlong_as_double((long long)(ulo | (uhi << 32)));
      const int cbit = (int)__builtin_amdgcn_readfirstlane(h[3]);
      meas_run<R, false>(gst, dim, 1u << ((head >> 8) & 0xff), u, cbit, cb, red, meas);
      if (tid == 0 && cbit >= 0) cbits[jb.cbit_off + cbit] = cb[cbit];
    } else {
      // BK_STAGE: cmask word = records in the stage, bytes of m = the global
      // qubit of each local bit, ascending; the first stage starts from |0...0>
      const ChunkMap cm = chunk_map<LQ>(h, bs.rec, dim, tid);
#pragma unroll 1
      for (uint32_t ch = chunk; ch < chunk + count; ++ch)
        stage_chunk<R>(st, gst, cm, ch, stage == 0, opw, cb, items, red, meas);
    }
    // Release: every wave's stores have completed (waitcnt) before the
    // barrier, then one agent-scope release (the write-back of this XCD's
    // L2) before the chunks count as done; the workgroup that completes a
    // stage opens the next one.
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (tid == 0) {
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");   // the whole workgroup's stores, through the barrier
      const unsigned d = atomicAdd(&ctl[job].done, count) + count;
      if (d == bs.nchunks) {
        atomicExch(&ctl[job].done, 0u);
        __threadfence();
        if (stage + 1 == jb.nst) atomicExch(&ctl[job].finished, 1u);
        __threadfence();
        atomicExch(&ctl[job].word, (unsigned long long)(stage + 1) << 32);
      }
    }
  }
}

// Clears a launch's scheduling state and every cbit (a staged job's cbits
// are read by each of its chunks).  A kernel rather than a memset so that a
// captured batch launch replays correctly.
__global__ void k_batch_reset(JobCtl* ctl, int nctl, unsigned* sched, uint8_t* cbits, uint32_t ncbits) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x, stride = gridDim.x * blockDim.x;
  for (uint32_t k = i; k < (uint32_t)nctl; k += stride) {
    ctl[k].word = 0;
    ctl[k].done = 0;
    ctl[k].finished = 0;
  }
  for (uint32_t k = i; k < ncbits; k += stride) cbits[k] = 0;
  if (i < 4) sched[i] = 0;
}

// The chunk that the i-th position of the stage kernel's chunk loop takes:
// i with its low 3 bits rotated to the top.  Workgroups go to the 8 XCDs in
// turn (workgroup b to XCD b mod 8) and the grid is a multiple of 8, so XCD
// x takes the chunks [x R, (x + 1) R), R = nchunks / 8, and the workgroups
// of one XCD hold consecutive chunks at any time: chunks that differ only
// in the lowest qubits outside the stage share cache lines when the stage
// leaves out some of qubits 0..2, and then meet in that XCD's L2.
__device__ __forceinline__ uint32_t xcd_chunk(uint32_t i, uint32_t nchunks) {
  return nchunks >= 8 ? ((i & 7u) * (nchunks >> 3)) | (i >> 3) : i;
}

// One stage of a simulator's held-back gates (the LDS-tile mode): every
// chunk of the state, a chunk per workgroup at a time.  The stage's header
// is record hrec of opw; the gates' cbit conditions read cbits.
template <typename R>
__global__ __launch_bounds__(kBatchThreads, kStageWavesPerSimd) void k_stage(
    typename EVb<R>::T* __restrict__ psi, int n, const uint32_t* __restrict__ opw, uint32_t hrec,
    const uint8_t* __restrict__ cbits, int ncbits) {
  constexpr int LQ = stage_qubits<R>();
  extern __shared__ __align__(16) unsigned char smem_raw[];
  typename EVb<R>::T* st = reinterpret_cast<typename EVb<R>::T*>(smem_raw);
  __shared__ uint8_t cb[kMaxJobCbits];
  __shared__ double red[2][kBatchThreads / 64];
  __shared__ double meas[2];
  __shared__ __align__(16) uint32_t items[2][kItemWords];
  const uint32_t tid = threadIdx.x, dim = 1u << n;
  for (int c = tid; c < ncbits && c < kMaxJobCbits; c += blockDim.x) cb[c] = cbits[c];
  const ChunkMap cm = chunk_map<LQ>(opw + (size_t)hrec * kOpWords, hrec, dim, tid);
  const uint32_t nchunks = dim >> LQ;
  const uint32_t nwords = (cm.it_end - cm.it_begin) * kOpWords;
  if (nwords <= kStageLdsWords) {
    // the stage's records once into LDS beside the chunk, for all of this
    // workgroup's chunks (2 % faster than staging each item per chunk;
    // scalar loads from global memory were 8 % slower)
    uint32_t* lrec = reinterpret_cast<uint32_t*>(smem_raw + (sizeof(typename EVb<R>::T) << LQ));
    for (uint32_t i = tid; i < nwords; i += blockDim.x) lrec[i] = opw[(size_t)cm.it_begin * kOpWords + i];
    __syncthreads();
    if constexpr (sizeof(R) == 4) {
      // complex64: the next chunk's amplitudes are loaded into registers
      // while this chunk's passes run (16 per thread; complex128 has no
      // registers to spare for its 8)
      using C = typename EVb<R>::T;
      constexpr int PT = stage_per_thread<R>();
      const uint32_t bd = blockDim.x;
      C pre[PT];
      uint32_t i = blockIdx.x;
      if (i < nchunks) {
        const uint32_t cpart = deposit(xcd_chunk(i, nchunks), cm.cmask);
#pragma unroll
        for (int k = 0; k < PT; ++k) pre[k] = psi[cm.base | deposit((uint32_t)k, cm.shigh) | cpart];
      }
      for (; i < nchunks; i += gridDim.x) {
        const uint32_t cpart = deposit(xcd_chunk(i, nchunks), cm.cmask);
#pragma unroll
        for (int k = 0; k < PT; ++k) st[swz<R>(tid + (uint32_t)k * bd)] = pre[k];
        __syncthreads();
        const uint32_t inext = i + gridDim.x;
        if (inext < nchunks) {
          const uint32_t npart = deposit(xcd_chunk(inext, nchunks), cm.cmask);
#pragma unroll
          for (int k = 0; k < PT; ++k) pre[k] = psi[cm.base | deposit((uint32_t)k, cm.shigh) | npart];
        }
        run_items<R, REC_LDS>(st, 1u << LQ, cm.it_begin, cm.it_end, opw, cb, items, red, meas, lrec, cm.it_begin);
#pragma unroll 1
        for (int k0 = 0; k0 < PT; k0 += 8)
#pragma unroll
          for (int k = 0; k < 8; ++k)
            psi[cm.base | deposit((uint32_t)(k0 + k), cm.shigh) | cpart] = st[swz<R>(tid + (uint32_t)(k0 + k) * bd)];
        __syncthreads();   // the next chunk's amplitudes overwrite LDS
      }
    } else {
      for (uint32_t i = blockIdx.x; i < nchunks; i += gridDim.x)
        stage_chunk<R, REC_LDS>(st, psi, cm, xcd_chunk(i, nchunks), false, opw, cb, items, red, meas, lrec);
    }
  } else {
    for (uint32_t i = blockIdx.x; i < nchunks; i += gridDim.x)
      stage_chunk<R>(st, psi, cm, xcd_chunk(i, nchunks), false, opw, cb, items, red, meas);
  }
}

// Packs a job's gate records into items: one-qubit, diagonal and phase gates
// into passes over three target qubits (the targets of its one-qubit gates,
// filled up with the lowest other qubits) and at most kPassGates gates; swaps
// and measurements stay single records.  Gates keep their order except where
// a later gate commutes with the ones it passes.
uint32_t op_mask(const BOp& o);
bool op_diag(const BOp& o);
constexpr int kPassWindow = 64;   // gates a pass looks at past its first

// The LDS swizzle of the pass kernel (swz), for the host.
uint32_t swz_host(uint32_t i, bool c64) {
  const uint32_t b = c64 ? 4 : 3, m = (1u << b) - 1;
  return i ^ ((i >> b) & m);
}

std::vector<BOp> build_items(const std::vector<BOp>& ops, bool c64) {
  const int K = kPassSlots;
  std::vector<BOp> out, cur;
  std::vector<int> T;
  auto close = [&]() {
    if (cur.empty()) return;
    // below three qubits the remaining slots take qubits n, n + 1, ...: no
    // gate names them, and their amplitudes lie in the LDS state's padding
    for (int q = 0; (int)T.size() < K; ++q)
      if (std::find(T.begin(), T.end(), q) == T.end()) T.push_back(q);
    std::vector<int> sorted(T);
    std::sort(sorted.begin(), sorted.end());
    BOp h{};
    h.head = (uint32_t)BK_PASS | ((uint32_t)K << 8) | ((uint32_t)cur.size() << 16);
    for (int i = 0; i < K; ++i) {
      h.cmask |= (uint32_t)T[i] << (8 * i);
      h.conds |= (uint32_t)sorted[i] << (8 * i);
    }
    // dwords 4..11: member r's LDS byte offset within a group
    uint32_t* hw = reinterpret_cast<uint32_t*>(h.m);
    for (int r = 0; r < (1 << K); ++r) {
      uint32_t rb = 0;
      for (int i = 0; i < K; ++i) rb |= (uint32_t)((r >> i) & 1) << T[i];
      hw[r] = swz_host(rb, c64) * (c64 ? 8u : 16u);
    }
    out.push_back(h);
    auto slot_of = [&](int q) { return (int)(std::find(T.begin(), T.end(), q) - T.begin()); };   // K: none
    uint32_t smask = 0;
    for (int i = 0; i < K; ++i) smask |= 1u << T[i];
    for (BOp o : cur) {
      const int okind = o.head & 0xff;
      if (is_one_qubit_dense(okind)) {
        const int slot = slot_of((o.head >> 8) & 0xff);
        o.head = (o.head & ~0xff00u) | ((uint32_t)slot << 8);
      }
      // a pass member's controls: those on pass targets as the member bits
      // they need (rmask), the others kept as a mask (cmask); a diagonal or
      // phase gate also gets, for each member r, its factor bits from pass
      // targets (2 bits per member), so the kernel does no slot lookups
      uint32_t rmask = 0, ktab = 0;
      for (int i = 0; i < K; ++i)
        if ((o.cmask >> T[i]) & 1u) rmask |= 1u << i;
      if (okind == BK_DIAG1 || okind == BK_DIAG2) {
        const int j0 = slot_of((o.head >> 8) & 0xff), j1 = okind == BK_DIAG2 ? slot_of((o.head >> 16) & 0xff) : K;
        for (int r = 0; r < (1 << K); ++r) {
          const uint32_t kr = (j0 < K ? (uint32_t)(r >> j0) & 1u : 0u) | (j1 < K ? ((uint32_t)(r >> j1) & 1u) << 1 : 0u);
          ktab |= kr << (2 * r);
        }
      }
      o.cmask &= ~smask;
      o.cbit = (int32_t)(ktab | (rmask << 16));
      out.push_back(o);
    }
    cur.clear();
    T.clear();
  };
  // A pass starts at the first unplaced gate and takes every later gate (up
  // to kPassWindow looked at) that fits its slots and may move up to it: a
  // gate passes the skipped ones only where they commute (no shared qubit,
  // or both diagonal).  Swaps and measurements end the look-ahead.
  std::vector<char> used(ops.size(), 0);
  size_t first = 0;
  while (first < ops.size()) {
    if (used[first]) {
      ++first;
      continue;
    }
    const int kind0 = ops[first].head & 0xff;
    if (kind0 == BK_SWAP || kind0 == BK_MEAS) {
      out.push_back(ops[first]);
      used[first++] = 1;
      continue;
    }
    uint32_t blocked = 0, blocked_diag = 0;   // qubits of skipped gates (non-diagonal / diagonal)
    int seen = 0;
    for (size_t i = first; i < ops.size() && (int)cur.size() < kPassGates && seen < kPassWindow; ++i) {
      if (used[i]) continue;
      ++seen;
      const BOp& o = ops[i];
      const int kind = o.head & 0xff;
      if (kind == BK_SWAP || kind == BK_MEAS) break;
      const uint32_t m = op_mask(o);
      const bool dg = op_diag(o);
      bool ok = (m & blocked) == 0 && (dg || (m & blocked_diag) == 0);
      if (ok && is_one_qubit_dense(kind)) {
        const int t = (o.head >> 8) & 0xff;
        const bool in = std::find(T.begin(), T.end(), t) != T.end();
        if (!in && (int)T.size() == K) ok = false;
        else if (!in) T.push_back(t);
      }
      if (ok) {
        cur.push_back(o);
        used[i] = 1;
      } else if (dg) {
        blocked_diag |= m;
      } else {
        blocked |= m;
      }
    }
    close();
  }
  return out;
}

// Qubits an op record touches (targets and controls) as a bit mask.
uint32_t op_mask(const BOp& o) {
  const int kind = o.head & 0xff;
  const uint32_t t0 = (o.head >> 8) & 0xff, t1 = (o.head >> 16) & 0xff;
  if (kind == BK_PHASE) return o.cmask;   // already holds targets and controls
  if (kind == BK_DIAG2 || kind == BK_SWAP) return o.cmask | (1u << t0) | (1u << t1);
  return o.cmask | (1u << t0);
}

bool op_diag(const BOp& o) {
  const int kind = o.head & 0xff;
  return kind == BK_DIAG1 || kind == BK_DIAG2 || kind == BK_PHASE;
}

// The record with its qubits renumbered through loc (global -> local).
BOp to_local(BOp o, const std::vector<int>& loc) {
  const int kind = o.head & 0xff;
  const uint32_t t0 = (o.head >> 8) & 0xff, t1 = (o.head >> 16) & 0xff;
  const bool two = kind == BK_DIAG2 || kind == BK_SWAP;
  uint32_t cm = 0;
  for (uint32_t m = o.cmask; m; m &= m - 1) cm |= 1u << loc[__builtin_ctz(m)];
  const uint32_t l0 = kind == BK_PHASE ? 0u : (uint32_t)loc[t0], l1 = two ? (uint32_t)loc[t1] : 0u;
  o.head = (o.head & 0xff0000ffu) | (l0 << 8) | (l1 << 16);
  o.cmask = cm;
  return o;
}

// Stages of a job whose state stays in global memory (n above what LDS
// holds).  Measurements split the list; between them, gates are grouped into
// stages of at most L qubits by a ready frontier (a gate is ready once every
// earlier gate on its qubits is scheduled, except that diagonal gates pass
// one another, since they commute; gates on disjoint qubits commute too, so
// any order of ready gates is valid).  A stage grows by the ready gate that
// adds the fewest new qubits (the earliest among equals) while the union
// stays within L qubits, then takes the lowest unused qubits up to L.  Each
// stage becomes a BK_STAGE header (record count, the L qubits ascending)
// followed by its items over local qubits 0..L-1.
std::vector<BOp> plan_stages(int n, int L, const std::vector<BOp>& ops, bool c64) {
  std::vector<BOp> out;
  const int kScan = 8;   // diagonal gates looked at behind the first unscheduled gate of a qubit
  // the first stage writes |0...0> (its chunks start from it instead of
  // reading the state): when the list is empty or starts with a measurement,
  // an empty stage on the lowest L qubits comes first
  if (ops.empty() || (ops[0].head & 0xff) == BK_MEAS) {
    BOp h{};
    h.head = (uint32_t)BK_STAGE | ((uint32_t)L << 8);
    uint8_t* q = reinterpret_cast<uint8_t*>(h.m);
    for (int j = 0; j < L; ++j) q[j] = (uint8_t)j;
    out.push_back(h);
  }
  size_t i0 = 0;
  while (i0 < ops.size()) {
    if ((ops[i0].head & 0xff) == BK_MEAS) {
      out.push_back(ops[i0++]);
      continue;
    }
    size_t i1 = i0;
    while (i1 < ops.size() && (ops[i1].head & 0xff) != BK_MEAS) ++i1;
    const int N = (int)(i1 - i0);
    std::vector<uint32_t> gm(N);
    std::vector<char> dg(N), done(N, 0);
    std::vector<std::vector<int>> onq(n);
    for (int i = 0; i < N; ++i) {
      gm[i] = op_mask(ops[i0 + i]);
      dg[i] = op_diag(ops[i0 + i]);
      for (uint32_t m = gm[i]; m; m &= m - 1) onq[__builtin_ctz(m)].push_back(i);
    }
    std::vector<size_t> head(n, 0);
    auto ready = [&](int i) {
      for (uint32_t m = gm[i]; m; m &= m - 1) {
        const int q = __builtin_ctz(m);
        for (size_t p = head[q]; p < onq[q].size(); ++p) {
          const int j = onq[q][p];
          if (j == i) break;
          if (done[j] || (dg[i] && dg[j])) continue;
          return false;
        }
      }
      return true;
    };
    int left = N;
    while (left > 0) {
      uint32_t S = 0;
      std::vector<int> members;
      for (;;) {
        int best = -1, best_new = 64;
        for (int q = 0; q < n; ++q) {
          while (head[q] < onq[q].size() && done[onq[q][head[q]]]) ++head[q];
          int seen = 0;
          for (size_t p = head[q]; p < onq[q].size() && seen <= kScan; ++p) {
            const int j = onq[q][p];
            if (done[j]) continue;
            ++seen;
            if (seen > 1 && !dg[j]) break;
            const int nw = __builtin_popcount(gm[j] & ~S);
            if (__builtin_popcount(S | gm[j]) <= L && (nw < best_new || (nw == best_new && j < best)) && ready(j)) {
              best = j;
              best_new = nw;
            }
            if (!dg[j]) break;
          }
        }
        if (best < 0) break;
        S |= gm[best];
        done[best] = 1;
        members.push_back(best);
        --left;
      }
      for (int q = 0; q < n && __builtin_popcount(S) < L; ++q) S |= 1u << q;
      std::vector<int> loc(n, -1);
      std::vector<uint8_t> qs;
      for (int q = 0; q < n; ++q)
        if ((S >> q) & 1) {
          loc[q] = (int)qs.size();
          qs.push_back((uint8_t)q);
        }
      std::vector<BOp> local;
      local.reserve(members.size());
      for (int i : members) local.push_back(to_local(ops[i0 + i], loc));
      std::vector<BOp> items = build_items(local, c64);
      BOp h{};
      h.head = (uint32_t)BK_STAGE | ((uint32_t)L << 8);
      h.cmask = (uint32_t)items.size();
      std::memcpy(h.m, qs.data(), qs.size());
      out.push_back(h);
      out.insert(out.end(), items.begin(), items.end());
    }
    i0 = i1;
  }
  return out;
}

qk_status cfail(std::string& err, qk_status st, const std::string& m) {
  err = m;
  return st;
}

// One op record compiled to a device record (qubits as given, n of them;
// cbit indices below ncbits).  Errors name the problem in err.
qk_status compile_op(const qk_op& o, int n, int ncbits, BOp& d, std::string& err) {
  d = BOp{};
  if (o.n_conds < 0 || o.n_conds > 2) return cfail(err, QK_E_ARG, "at most 2 conditions");
  for (int c = 0; c < o.n_conds; ++c) {
    if (o.conds[c].cbit < 0 || o.conds[c].cbit >= ncbits) return cfail(err, QK_E_ARG, "condition cbit out of range");
    if (o.conds[c].value != 0 && o.conds[c].value != 1) return cfail(err, QK_E_ARG, "condition value must be 0 or 1");
  }
  int kind = 0, t0 = 0, t1 = 0;
  d.cbit = -1;
  if (o.n_conds > 0) d.conds = (uint32_t)o.conds[0].cbit | ((uint32_t)o.conds[0].value << 8);
  if (o.n_conds > 1) d.conds |= ((uint32_t)o.conds[1].cbit << 16) | ((uint32_t)o.conds[1].value << 24);
  if (o.kind == QK_OP_MEASURE) {
    if (o.qubit < 0 || o.qubit >= n) return cfail(err, QK_E_ARG, "qubit out of range");
    if (o.cbit < -1 || o.cbit >= ncbits) return cfail(err, QK_E_ARG, "cbit out of range");
    if (!(o.u >= 0.0 && o.u < 1.0)) return cfail(err, QK_E_ARG, "u must be in [0, 1)");
    if (o.n_conds) return cfail(err, QK_E_ARG, "measurements take no conditions");
    kind = BK_MEAS;
    t0 = o.qubit;
    d.cbit = o.cbit;
    d.m[0] = o.u;
  } else if (o.kind == QK_OP_GATE) {
    int arity = 0, np = 0;
    if (!builtin_info(o.gate, &arity, &np)) return cfail(err, QK_E_UNSUPPORTED, "batched circuits take builtin gates only");
    if (o.n_targets != arity) return cfail(err, QK_E_ARG, "target count does not match the gate");
    if (o.n_controls < 0 || o.n_controls > 4) return cfail(err, QK_E_ARG, "at most 4 controls");
    uint32_t seen = 0;
    for (int q = 0; q < o.n_targets + o.n_controls; ++q) {
      const int x = q < o.n_targets ? o.targets[q] : o.controls[q - o.n_targets];
      if (x < 0 || x >= n) return cfail(err, QK_E_ARG, "qubit index out of range");
      if (seen & (1u << x)) return cfail(err, QK_E_ARG, "qubit used twice in one gate");
      seen |= 1u << x;
    }
    uint32_t cm = 0;
    for (int q = 0; q < o.n_controls; ++q) cm |= 1u << o.controls[q];
    const BuiltinGate g = builtin_gate(o.gate, np ? o.param : 0.0);
    t0 = o.targets[0];
    t1 = arity > 1 ? o.targets[1] : 0;
    switch (g.cls) {
      case BG_DENSE1: {
        d.cmask = cm;
        bool real = true;
        for (int e = 0; e < 4; ++e) {
          d.m[2 * e] = g.m[e].real();
          d.m[2 * e + 1] = g.m[e].imag();
          real = real && g.m[e].imag() == 0.0;
        }
        const bool flip = g.m[0] == cd(0.0) && g.m[1] == cd(1.0) && g.m[2] == cd(1.0) && g.m[3] == cd(0.0);
        kind = flip ? BK_X : (real ? BK_U1R : BK_U1);
        break;
      }
      case BG_DIAG:
        kind = arity == 1 ? BK_DIAG1 : BK_DIAG2;
        d.cmask = cm;
        for (size_t e = 0; e < g.m.size(); ++e) {
          d.m[2 * e] = g.m[e].real();
          d.m[2 * e + 1] = g.m[e].imag();
        }
        break;
      case BG_PHASE:
        kind = BK_PHASE;
        d.cmask = cm | (1u << t0) | (arity > 1 ? (1u << t1) : 0u);
        d.m[0] = g.z.real();
        d.m[1] = g.z.imag();
        break;
      case BG_SWAP:
        kind = BK_SWAP;
        d.cmask = cm;
        break;
      default:
        return cfail(err, QK_E_UNSUPPORTED, "gate class not supported in batches");
    }
  } else {
    return cfail(err, QK_E_ARG, "unknown op kind");
  }
  d.head = (uint32_t)kind | ((uint32_t)t0 << 8) | ((uint32_t)t1 << 16) | ((uint32_t)o.n_conds << 24);
  return QK_OK;
}

struct HostJob {
  int n, ncbits;
  bool staged = false;    // state in global memory, run by stages
  std::vector<BOp> ops;   // items (passes and single records), or stages and measurements, ready to upload
  uint64_t state_off = 0;
  uint32_t cbit_off = 0;
};

std::string g_batch_error;

}  // namespace

struct qk_batch_s {
  qk_dtype dtype = QK_C128;
  bool c64 = false;
  qk_allocator alloc{};
  bool has_alloc = false;
  hipStream_t stream = nullptr;
  std::vector<HostJob> jobs;
  void* d_states = nullptr;
  size_t states_bytes = 0;
  void* d_cbits = nullptr;
  size_t cbits_bytes = 0;
  void* d_ops = nullptr;
  size_t ops_bytes = 0;
  void* d_jobs = nullptr;
  size_t jobs_bytes = 0;
  void* d_stages = nullptr;   // stage table of the staged jobs
  size_t stages_bytes = 0;
  void* d_ctl = nullptr;      // per staged job scheduling state
  size_t ctl_bytes = 0;
  void* d_sched = nullptr;    // scan hint, small-job counter, stall flag
  size_t sched_bytes = 0;
  size_t nstaged = 0;
  size_t ncbits_total = 0;
  uint32_t run_max = 1;       // longest run of chunks one claim takes
  bool ran = false;
  bool uploaded = false;   // the device job table and ops match `jobs` (a rerun only relaunches)
  size_t njobs_dev = 0;
  size_t shm = 0;
  unsigned grid = 0;
  std::string err;
};

namespace {

qk_status bfail(qk_batch b, qk_status st, const std::string& m) {
  if (b) b->err = m;
  else g_batch_error = m;
  return st;
}

void* balloc(qk_batch b, size_t bytes) {
  if (bytes == 0) bytes = 256;
  if (b->has_alloc) return b->alloc.alloc(bytes, (void*)b->stream, b->alloc.ctx);
  void* p = nullptr;
  if (hipMalloc(&p, bytes) != hipSuccess) {
    (void)hipGetLastError();
    return nullptr;
  }
  return p;
}

void bfree(qk_batch b, void*& p, size_t& bytes) {
  if (!p) return;
  if (b->has_alloc) b->alloc.free(p, bytes, (void*)b->stream, b->alloc.ctx);
  else (void)hipFree(p);
  p = nullptr;
  bytes = 0;
}

qk_status bensure(qk_batch b, void*& p, size_t& cur, size_t need, const char* what) {
  if (p && cur >= need) return QK_OK;
  bfree(b, p, cur);
  p = balloc(b, need);
  if (!p) return bfail(b, QK_E_OOM, std::string("device allocation failed: ") + what);
  cur = need;
  return QK_OK;
}

// Jobs up to these sizes keep their whole state in LDS; larger ones, up to
// kMaxStagedQubits, keep it in global memory and run by stages of
// stage_qubits() qubits through LDS.
int max_lds_qubits(bool c64) { return c64 ? 14 : 13; }
constexpr int kMaxStagedQubits = 24;

}  // namespace

extern "C" {

qk_status qk_batch_create(qk_dtype dtype, const qk_allocator* alloc, void* hip_stream, qk_batch* out) {
  if (!out) return bfail(nullptr, QK_E_ARG, "out is NULL");
  *out = nullptr;
  if (dtype != QK_C64 && dtype != QK_C128) return bfail(nullptr, QK_E_ARG, "dtype must be QK_C64 or QK_C128");
  if (alloc && (!alloc->alloc || !alloc->free)) return bfail(nullptr, QK_E_ARG, "allocator needs alloc and free");
  qk_batch b = new qk_batch_s;
  b->dtype = dtype;
  b->c64 = dtype == QK_C64;
  if (alloc) {
    b->alloc = *alloc;
    b->has_alloc = true;
  }
  b->stream = (hipStream_t)hip_stream;
  *out = b;
  return QK_OK;
}

qk_status qk_batch_destroy(qk_batch b) {
  if (!b) return bfail(nullptr, QK_E_ARG, "batch is NULL");
  if (b->d_states || b->d_ops) (void)hipStreamSynchronize(b->stream);
  bfree(b, b->d_states, b->states_bytes);
  bfree(b, b->d_cbits, b->cbits_bytes);
  bfree(b, b->d_ops, b->ops_bytes);
  bfree(b, b->d_jobs, b->jobs_bytes);
  bfree(b, b->d_stages, b->stages_bytes);
  bfree(b, b->d_ctl, b->ctl_bytes);
  bfree(b, b->d_sched, b->sched_bytes);
  delete b;
  return QK_OK;
}

const char* qk_batch_last_error(qk_batch b) { return b ? b->err.c_str() : g_batch_error.c_str(); }

qk_status qk_batch_add(qk_batch b, int32_t n, int32_t ncbits, const qk_op* ops, int32_t nops, int32_t* job) {
  if (!b) return bfail(nullptr, QK_E_ARG, "batch is NULL");
  if (n < 1 || n > kMaxStagedQubits)
    return bfail(b, QK_E_ARG, "qubit count outside the batched range (1.." + std::to_string(kMaxStagedQubits) + ")");
  if (ncbits < 0 || ncbits > kMaxJobCbits) return bfail(b, QK_E_ARG, "cbit count outside 0..256");
  if (nops < 0 || (nops > 0 && !ops)) return bfail(b, QK_E_ARG, "bad op array");
  HostJob hj;
  hj.n = n;
  hj.ncbits = ncbits;
  hj.ops.reserve(nops);
  for (int i = 0; i < nops; ++i) {
    BOp d;
    std::string err;
    const qk_status st = compile_op(ops[i], n, ncbits, d, err);
    if (st) return bfail(b, st, "op " + std::to_string(i) + ": " + err);
    hj.ops.push_back(d);
  }
  hj.staged = n > max_lds_qubits(b->c64);
  hj.ops = hj.staged ? plan_stages(n, b->c64 ? stage_qubits<float>() : stage_qubits<double>(), hj.ops, b->c64)
                     : build_items(hj.ops, b->c64);
  b->jobs.push_back(std::move(hj));
  if (job) *job = (int32_t)b->jobs.size() - 1;
  b->ran = false;
  b->uploaded = false;
  return QK_OK;
}

}  // extern "C"

template <typename R>
static void launch_batch_t(qk_batch b) {
  static bool set = false;
  if (!set) {
    (void)hipFuncSetAttribute((const void*)k_batch<R>, hipFuncAttributeMaxDynamicSharedMemorySize, 128 * 1024);
    set = true;
  }
  hipLaunchKernelGGL(k_batch_reset, dim3(64), dim3(256), 0, b->stream, (JobCtl*)b->d_ctl, (int)b->nstaged,
                     (unsigned*)b->d_sched, (uint8_t*)b->d_cbits, (uint32_t)b->ncbits_total);
  static unsigned long long stall = 0;   // 10 s of the device wall clock
  if (!stall) {
    int khz = 0, dev = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess || khz <= 0)
      khz = 100000;
    stall = 10000ull * (unsigned long long)khz;
  }
  hipLaunchKernelGGL(k_batch<R>, dim3(b->grid), dim3(kBatchThreads), b->shm, b->stream, (const BJob*)b->d_jobs,
                     (int)b->njobs_dev, (int)b->nstaged, (const BStage*)b->d_stages, (JobCtl*)b->d_ctl,
                     (unsigned*)b->d_sched, (const uint32_t*)b->d_ops, (typename EVb<R>::T*)b->d_states,
                     (uint8_t*)b->d_cbits, stall, b->run_max);
}

static void launch_batch(qk_batch b) {
  if (b->c64) launch_batch_t<float>(b);
  else launch_batch_t<double>(b);
}

extern "C" {

qk_status qk_batch_run(qk_batch b) {
  if (!b) return bfail(nullptr, QK_E_ARG, "batch is NULL");
  if (b->jobs.empty()) return QK_OK;
  if (b->uploaded) {   // same jobs as the last run: only the scheduling state is reset
    launch_batch(b);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return bfail(b, QK_E_HIP, std::string("batch launch: ") + hipGetErrorString(e));
    b->ran = true;
    return QK_OK;
  }
  const size_t amp = b->c64 ? 8 : 16;
  const int lq = b->c64 ? stage_qubits<float>() : stage_qubits<double>();
  // layout: states and cbits in job order; the device table lists the staged
  // jobs first, then the small ones, each part largest first
  uint64_t soff = 0;
  uint32_t coff = 0, ooff = 0;
  int nmax = 0;   // largest job kept in LDS, or the stage chunk when larger
  for (auto& j : b->jobs) {
    j.state_off = soff;
    j.cbit_off = coff;
    soff += 1ull << j.n;
    coff += (uint32_t)j.ncbits;
    nmax = std::max(nmax, j.staged ? lq : j.n);
  }
  std::vector<int> order(b->jobs.size());
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int x, int y) {
    const auto& a = b->jobs[x];
    const auto& c = b->jobs[y];
    if (a.staged != c.staged) return a.staged;
    return ((uint64_t)a.ops.size() << a.n) > ((uint64_t)c.ops.size() << c.n);
  });
  std::vector<BOp> all_ops;
  std::vector<BJob> table;
  std::vector<BStage> stab;
  size_t nstaged = 0;
  for (int id : order) {
    const auto& j = b->jobs[id];
    BJob t{};
    t.state_off = j.state_off;
    t.op_begin = ooff;
    all_ops.insert(all_ops.end(), j.ops.begin(), j.ops.end());
    t.op_end = ooff + (uint32_t)j.ops.size();
    t.n = j.n;
    t.ncbits = j.ncbits;
    t.cbit_off = j.cbit_off;
    if (j.staged) {
      ++nstaged;
      t.st_begin = (uint32_t)stab.size();
      for (uint32_t r = 0; r < (uint32_t)j.ops.size();) {
        const BOp& o = j.ops[r];
        if ((o.head & 0xff) == BK_MEAS) {
          stab.push_back({ooff + r, 1u});
          ++r;
        } else {
          stab.push_back({ooff + r, 1u << (j.n - lq)});
          r += 1 + o.cmask;
        }
      }
      t.nst = (uint32_t)stab.size() - t.st_begin;
    }
    ooff = t.op_end;
    table.push_back(t);
  }
  all_ops.resize(all_ops.size() + kPadRecords);   // padding: the kernel reads the next item before knowing its size
  qk_status st;
  if ((st = bensure(b, b->d_states, b->states_bytes, soff * amp, "batch states"))) return st;
  if ((st = bensure(b, b->d_cbits, b->cbits_bytes, std::max<size_t>(coff, 1), "batch cbits"))) return st;
  if ((st = bensure(b, b->d_ops, b->ops_bytes, all_ops.size() * sizeof(BOp), "batch ops"))) return st;
  if ((st = bensure(b, b->d_jobs, b->jobs_bytes, table.size() * sizeof(BJob), "batch job table"))) return st;
  if ((st = bensure(b, b->d_stages, b->stages_bytes, std::max<size_t>(stab.size(), 1) * sizeof(BStage), "batch stages")))
    return st;
  if ((st = bensure(b, b->d_ctl, b->ctl_bytes, std::max<size_t>(nstaged, 1) * sizeof(JobCtl), "batch scheduling")))
    return st;
  if ((st = bensure(b, b->d_sched, b->sched_bytes, 4 * sizeof(unsigned), "batch scheduling"))) return st;
  hipError_t e = hipMemcpyAsync(b->d_ops, all_ops.data(), all_ops.size() * sizeof(BOp), hipMemcpyHostToDevice, b->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(b->d_jobs, table.data(), table.size() * sizeof(BJob), hipMemcpyHostToDevice, b->stream);
  if (e == hipSuccess && !stab.empty())
    e = hipMemcpyAsync(b->d_stages, stab.data(), stab.size() * sizeof(BStage), hipMemcpyHostToDevice, b->stream);
  if (e != hipSuccess) return bfail(b, QK_E_HIP, std::string("batch upload: ") + hipGetErrorString(e));
  const size_t shm = ((size_t)1 << std::max(nmax, kPassSlots)) * amp;   // a pass group's 8 amplitudes at least
  int ncu = 256, dev = 0;
  if (hipGetDevice(&dev) == hipSuccess) (void)hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
  const int per_cu = std::max<int>(1, std::min(4, (int)(160 * 1024 / (shm + 4096))));
  // staged jobs spread their chunks over every workgroup that fits; small
  // jobs need at most one workgroup each
  const size_t want = nstaged ? (size_t)ncu * per_cu : std::min<size_t>(table.size(), (size_t)ncu * per_cu);
  b->shm = shm;
  b->grid = (unsigned)std::max<size_t>(1, want);
  b->njobs_dev = table.size();
  b->nstaged = nstaged;
  b->ncbits_total = coff;
  // Runs of chunks per claim amortise the claim's fences when the staged
  // work is plentiful (about two claims per workgroup per round of stages),
  // and shrink to single chunks when a few jobs must spread over the grid.
  uint64_t chunks = 0;
  for (const BJob& t : table)
    if (t.nst) chunks += 1ull << (t.n - lq);
  b->run_max = (uint32_t)std::min<uint64_t>(16, std::max<uint64_t>(1, chunks / (2ull * b->grid)));
  launch_batch(b);
  e = hipGetLastError();
  if (e != hipSuccess) return bfail(b, QK_E_HIP, std::string("batch launch: ") + hipGetErrorString(e));
  b->ran = true;
  b->uploaded = true;
  return QK_OK;
}

qk_status qk_batch_sync(qk_batch b) {
  if (!b) return bfail(nullptr, QK_E_ARG, "batch is NULL");
  hipError_t e = hipStreamSynchronize(b->stream);
  if (e != hipSuccess) return bfail(b, QK_E_HIP, std::string("batch: ") + hipGetErrorString(e));
  if (b->ran && b->nstaged && b->d_sched) {
    unsigned flags[4] = {0, 0, 0, 0};
    e = hipMemcpy(flags, b->d_sched, sizeof(flags), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return bfail(b, QK_E_HIP, std::string("batch: ") + hipGetErrorString(e));
    if (flags[2]) return bfail(b, QK_E_HIP, "batch: a workgroup found no work for 10 s while stages were open (scheduler stall)");
  }
  return QK_OK;
}

qk_status qk_batch_get_state(qk_batch b, int32_t job, void* host_out, size_t bytes) {
  if (!b) return bfail(nullptr, QK_E_ARG, "batch is NULL");
  if (job < 0 || job >= (int)b->jobs.size()) return bfail(b, QK_E_ARG, "job index out of range");
  if (!b->ran) return bfail(b, QK_E_STATE, "batch has not run since the job was added");
  const size_t amp = b->c64 ? 8 : 16;
  const auto& j = b->jobs[job];
  const size_t need = ((size_t)1 << j.n) * amp;
  if (!host_out || bytes != need) return bfail(b, QK_E_ARG, "buffer size must be 2^n * amplitude size");
  hipError_t e = hipMemcpyAsync(host_out, (char*)b->d_states + j.state_off * amp, need, hipMemcpyDeviceToHost, b->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
  if (e != hipSuccess) return bfail(b, QK_E_HIP, std::string("batch readback: ") + hipGetErrorString(e));
  return QK_OK;
}

qk_status qk_batch_read_cbits(qk_batch b, int32_t job, uint8_t* out, int32_t n) {
  if (!b) return bfail(nullptr, QK_E_ARG, "batch is NULL");
  if (job < 0 || job >= (int)b->jobs.size()) return bfail(b, QK_E_ARG, "job index out of range");
  if (!b->ran) return bfail(b, QK_E_STATE, "batch has not run since the job was added");
  const auto& j = b->jobs[job];
  if (n < 0 || n > j.ncbits || (n > 0 && !out)) return bfail(b, QK_E_ARG, "bad cbit count");
  hipError_t e = hipSuccess;
  if (n > 0) e = hipMemcpyAsync(out, (char*)b->d_cbits + j.cbit_off, (size_t)n, hipMemcpyDeviceToHost, b->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
  if (e != hipSuccess) return bfail(b, QK_E_HIP, std::string("batch readback: ") + hipGetErrorString(e));
  return QK_OK;
}

qk_status qk_batch_state_ptr(qk_batch b, int32_t job, void** dev_ptr, size_t* bytes) {
  if (!b) return bfail(nullptr, QK_E_ARG, "batch is NULL");
  if (job < 0 || job >= (int)b->jobs.size()) return bfail(b, QK_E_ARG, "job index out of range");
  if (!b->ran) return bfail(b, QK_E_STATE, "batch has not run since the job was added");
  const size_t amp = b->c64 ? 8 : 16;
  const auto& j = b->jobs[job];
  if (dev_ptr) *dev_ptr = (char*)b->d_states + j.state_off * amp;
  if (bytes) *bytes = ((size_t)1 << j.n) * amp;
  return QK_OK;
}

qk_status qk_batch_layout(qk_batch b, int32_t job, size_t* state_offset, size_t* state_bytes, size_t* cbit_offset) {
  if (!b) return bfail(nullptr, QK_E_ARG, "batch is NULL");
  if (job < 0 || job >= (int)b->jobs.size()) return bfail(b, QK_E_ARG, "job index out of range");
  uint64_t soff = 0, coff = 0;   // the layout qk_batch_run uses: states and cbits in job order
  for (int32_t i = 0; i < job; ++i) {
    soff += 1ull << b->jobs[i].n;
    coff += (uint64_t)b->jobs[i].ncbits;
  }
  const size_t amp = b->c64 ? 8 : 16;
  if (state_offset) *state_offset = soff * amp;
  if (state_bytes) *state_bytes = ((size_t)1 << b->jobs[job].n) * amp;
  if (cbit_offset) *cbit_offset = coff;
  return QK_OK;
}

qk_status qk_batch_read_async(qk_batch b, void* host_states, size_t state_bytes, uint8_t* host_cbits,
                              size_t cbit_bytes) {
  if (!b) return bfail(nullptr, QK_E_ARG, "batch is NULL");
  if (!b->ran || !b->uploaded) return bfail(b, QK_E_STATE, "batch has not run since the last job was added");
  uint64_t samps = 0, cbytes = 0;
  for (const auto& j : b->jobs) {
    samps += 1ull << j.n;
    cbytes += (uint64_t)j.ncbits;
  }
  const size_t need = samps * (b->c64 ? 8 : 16);
  if (!host_states || state_bytes < need) return bfail(b, QK_E_ARG, "state buffer smaller than the batch's states");
  if (cbytes && (!host_cbits || cbit_bytes < cbytes)) return bfail(b, QK_E_ARG, "cbit buffer smaller than the batch's cbits");
  hipError_t e = hipMemcpyAsync(host_states, b->d_states, need, hipMemcpyDeviceToHost, b->stream);
  if (e == hipSuccess && cbytes) e = hipMemcpyAsync(host_cbits, b->d_cbits, cbytes, hipMemcpyDeviceToHost, b->stream);
  if (e != hipSuccess) return bfail(b, QK_E_HIP, std::string("batch asynchronous read: ") + hipGetErrorString(e));
  return QK_OK;
}

qk_status qk_batch_clear(qk_batch b) {
  if (!b) return bfail(nullptr, QK_E_ARG, "batch is NULL");
  b->jobs.clear();
  b->ran = false;
  b->uploaded = false;
  return QK_OK;
}

qk_status qk_batch_num_jobs(qk_batch b, int32_t* n) {
  if (!b || !n) return bfail(b, QK_E_ARG, "NULL argument");
  *n = (int32_t)b->jobs.size();
  return QK_OK;
}

}  // extern "C"

// ---- the simulator's LDS-tile mode ---------------------------------------------

namespace qk {

int stage_chunk_qubits(bool c64) { return c64 ? stage_qubits<float>() : stage_qubits<double>(); }

qk_status stage_plan(bool c64, int n, int ncbits, const std::vector<qk_op>& ops, std::vector<unsigned char>& recs,
                     std::vector<uint32_t>& headers, std::string& err) {
  std::vector<BOp> bops;
  bops.reserve(ops.size());
  for (size_t i = 0; i < ops.size(); ++i) {
    BOp d;
    const qk_status st = compile_op(ops[i], n, std::min(ncbits, kMaxJobCbits), d, err);
    if (st) {
      err = "op " + std::to_string(i) + ": " + err;
      return st;
    }
    if ((d.head & 0xff) == BK_MEAS) {
      err = "measurements are not staged";
      return QK_E_ARG;
    }
    bops.push_back(d);
  }
  std::vector<BOp> planned = plan_stages(n, stage_chunk_qubits(c64), bops, c64);
  headers.clear();
  for (uint32_t r = 0; r < (uint32_t)planned.size(); r += 1 + planned[r].cmask) headers.push_back(r);
  planned.resize(planned.size() + kPadRecords);   // the item prefetch reads past a stage's last record
  recs.resize(planned.size() * sizeof(BOp));
  std::memcpy(recs.data(), planned.data(), recs.size());
  return QK_OK;
}

template <typename R>
static void launch_stage_t(void* psi, int n, const void* d_recs, uint32_t hrec, const uint8_t* d_cbits, int ncbits,
                           hipStream_t stream) {
  static int ncu = 0;
  if (!ncu) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
      ncu = 256;
    (void)hipFuncSetAttribute((const void*)k_stage<R>, hipFuncAttributeMaxDynamicSharedMemorySize, 128 * 1024);
  }
  const size_t shm = (sizeof(typename EVb<R>::T) << stage_qubits<R>()) + kStageLdsWords * 4;   // 64 + 12 KiB
  const uint32_t nchunks = 1u << (n - stage_qubits<R>());
  const unsigned grid = (unsigned)std::min<uint32_t>(nchunks, (uint32_t)ncu * 2);   // two 64 KiB chunks per CU
  hipLaunchKernelGGL(k_stage<R>, dim3(grid), dim3(kBatchThreads), shm, stream, (typename EVb<R>::T*)psi, n,
                     (const uint32_t*)d_recs, hrec, d_cbits, ncbits);
}

void launch_stage(bool c64, void* psi, int n, const void* d_recs, uint32_t hrec, const uint8_t* d_cbits, int ncbits,
                  hipStream_t stream) {
  if (c64) launch_stage_t<float>(psi, n, d_recs, hrec, d_cbits, ncbits, stream);
  else launch_stage_t<double>(psi, n, d_recs, hrec, d_cbits, ncbits, stream);
}

}  // namespace qk
