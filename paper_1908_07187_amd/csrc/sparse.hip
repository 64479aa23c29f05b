// Sparse state engine for gfx950: the state as its nonzero amplitudes, kept as
// ascending amplitude indices idx[0..nnz) with amplitudes amp[0..nnz).  The
// paper's engine keeps the state of the recycled-qubit Shor circuit "relatively
// sparse" and runs a 39-qubit conventional Shor circuit on 12 GB (section
// "Shor's Factorization with Q-Kit."), which a dense vector (8 TiB) cannot;
// this engine applies the same gate definitions to such states.
//
//   dense k-qubit gate   key = (index with the target bits removed) << k | m,
//                        m = the target bits in gate order; a radix sort by key
//                        brings each group (same non-target bits) together with
//                        its members in m order.  One thread per group: if the
//                        group's control bits are all 1 it writes all 2^k
//                        outputs w = M v (exact zeros get a sentinel index past
//                        every real one), else it copies its members.  Output
//                        slots come from an exclusive scan of the per-group
//                        counts; a second radix sort by index restores the
//                        ascending order and pushes the sentinels to the end.
//                        Either sort is skipped when a pass over its keys
//                        finds them already ascending (e.g. a gate on a qubit
//                        that no entry has set yet).
//   diagonal / phase     in place, no reordering; a run of up to 24 diagonal
//                        gates of at most 2 targets is one pass.
//   permutation / swap   every entry whose controls are all 1 gets its target
//                        bits mapped forward (table, affine, modular
//                        multiplication, bit swap); a radix sort by index
//                        restores the order, unless the mapped indices are
//                        already ascending (e.g. a map of low bits when every
//                        run of equal high bits holds one entry).
//   measurement          FP64 sums of |a|^2 split by the measured bit over
//                        fixed ranges of entries (index order), outcome and
//                        1/sqrt(p) on the device as in the dense path, then an
//                        order-preserving compaction of the kept entries.
//
// Every kernel is deterministic: sorts and scans are exact integer work, each
// output slot is written by one thread, and every floating-point sum runs in a
// fixed order.  The host reads back only entry counts (to size the next step).
#include <rocprim/device/device_radix_sort.hpp>
#include <rocprim/device/device_merge.hpp>
#include <rocprim/device/device_scan.hpp>

#include <algorithm>

#include "qk_internal.h"

namespace qk {
namespace {

template <typename R> struct SpT;
template <> struct SpT<float> { using V = float2; };
template <> struct SpT<double> { using V = double2; };
template <typename R> using SpV = typename SpT<R>::V;

constexpr int kSpBlock = 256;
constexpr uint64_t kSpMaxGrid = 1u << 20;

inline unsigned sp_grid(uint64_t items) {
  return (unsigned)std::min<uint64_t>(kSpMaxGrid, std::max<uint64_t>(1, (items + kSpBlock - 1) / kSpBlock));
}

// Insert zero bits at the ascending positions of s (compact counter -> index).
__device__ __forceinline__ uint64_t sp_insert(uint64_t x, const Special& s) {
  for (int i = 0; i < s.n; ++i) {
    const int p = s.pos[i];
    x = ((x >> p) << (p + 1)) | (x & ((1ull << p) - 1));
  }
  return x;
}
// Remove the bits at the ascending positions of s (index -> compact counter).
__device__ __forceinline__ uint64_t sp_remove(uint64_t x, const Special& s) {
  for (int i = s.n - 1; i >= 0; --i) {
    const int p = s.pos[i];
    x = ((x >> (p + 1)) << p) | (x & ((1ull << p) - 1));
  }
  return x;
}
__device__ __forceinline__ uint64_t sp_ext(uint64_t i, const SpTargets& t) {
  uint64_t m = 0;
  for (int j = 0; j < t.k; ++j) m |= ((i >> t.pos[j]) & 1ull) << j;
  return m;
}
__device__ __forceinline__ uint64_t sp_dep(uint64_t m, const SpTargets& t) {
  uint64_t i = 0;
  for (int j = 0; j < t.k; ++j) i |= ((m >> j) & 1ull) << t.pos[j];
  return i;
}

__device__ __forceinline__ double sp_wave_sum(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

}  // namespace

// ---- dense k-qubit gate ----------------------------------------------------------

__global__ __launch_bounds__(kSpBlock) void k_sp_keys(const uint64_t* __restrict__ idx, uint64_t nnz, Special tsorted,
                                                      SpTargets t, uint64_t* __restrict__ key) {
  for (uint64_t i = (uint64_t)blockIdx.x * kSpBlock + threadIdx.x; i < nnz; i += (uint64_t)gridDim.x * kSpBlock) {
    const uint64_t x = idx[i];
    key[i] = (sp_remove(x, tsorted) << t.k) | sp_ext(x, t);
  }
}

// *unsorted = 1 when some key exceeds the next one (the sort is then needed;
// else it is skipped).
__global__ __launch_bounds__(kSpBlock) void k_sp_check_order(const uint64_t* __restrict__ key, uint64_t n,
                                                             uint64_t* __restrict__ unsorted) {
  for (uint64_t i = (uint64_t)blockIdx.x * kSpBlock + threadIdx.x; i + 1 < n; i += (uint64_t)gridDim.x * kSpBlock)
    if (key[i] > key[i + 1]) *unsorted = 1;
}

__global__ void k_sp_clear(uint64_t* __restrict__ p, int n) {
  if (blockIdx.x == 0 && (int)threadIdx.x < n) p[threadIdx.x] = 0;
}

__global__ __launch_bounds__(kSpBlock) void k_sp_group_count(const uint64_t* __restrict__ skey, uint64_t nnz,
                                                             Special tsorted, int k, uint64_t cmask,
                                                             uint32_t* __restrict__ cnt) {
  for (uint64_t i = (uint64_t)blockIdx.x * kSpBlock + threadIdx.x; i < nnz; i += (uint64_t)gridDim.x * kSpBlock) {
    const uint64_t pre = skey[i] >> k;
    const bool head = i == 0 || (skey[i - 1] >> k) != pre;
    uint32_t c = 0;
    if (head) {
      const uint64_t base = sp_insert(pre, tsorted);
      if ((base & cmask) == cmask) {
        c = 1u << k;
      } else {
        uint64_t j = i + 1;
        while (j < nnz && (skey[j] >> k) == pre) ++j;
        c = (uint32_t)(j - i);
      }
    }
    cnt[i] = c;
  }
}

__global__ void k_sp_total(const uint32_t* __restrict__ cnt, const uint64_t* __restrict__ off, uint64_t nnz,
                           uint64_t* __restrict__ scal) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    scal[0] = nnz ? off[nnz - 1] + cnt[nnz - 1] : 0;
    scal[1] = 0;
    scal[2] = 0;
  }
}

template <typename R>
__global__ __launch_bounds__(kSpBlock) void k_sp_group_apply(const uint64_t* __restrict__ skey,
                                                             const SpV<R>* __restrict__ samp, uint64_t nnz,
                                                             Special tsorted, SpTargets t, uint64_t cmask,
                                                             const SpV<R>* __restrict__ mat,
                                                             const uint64_t* __restrict__ off, uint64_t sentinel,
                                                             uint64_t* __restrict__ out_idx,
                                                             SpV<R>* __restrict__ out_amp,
                                                             unsigned long long* __restrict__ zeros) {
  const int k = t.k;
  const uint32_t D = 1u << k;
  for (uint64_t i = (uint64_t)blockIdx.x * kSpBlock + threadIdx.x; i < nnz; i += (uint64_t)gridDim.x * kSpBlock) {
    const uint64_t pre = skey[i] >> k;
    if (i > 0 && (skey[i - 1] >> k) == pre) continue;     // not the head of its group
    uint64_t g = 1;
    while (i + g < nnz && (skey[i + g] >> k) == pre) ++g;
    const uint64_t base = sp_insert(pre, tsorted);
    const uint64_t o = off[i];
    if ((base & cmask) != cmask) {                        // controls not all 1: members unchanged
      for (uint64_t j = 0; j < g; ++j) {
        out_idx[o + j] = base | sp_dep(skey[i + j] & (D - 1), t);
        out_amp[o + j] = samp[i + j];
      }
      continue;
    }
    unsigned long long nz = 0;
    for (uint32_t r = 0; r < D; ++r) {
      R wr = 0, wi = 0;
      for (uint64_t j = 0; j < g; ++j) {
        const uint32_t m = (uint32_t)(skey[i + j] & (D - 1));
        const SpV<R> a = mat[(size_t)r * D + m];
        const SpV<R> v = samp[i + j];
        wr += a.x * v.x - a.y * v.y;
        wi += a.x * v.y + a.y * v.x;
      }
      const bool zero = (wr == (R)0 && wi == (R)0);
      out_idx[o + r] = zero ? sentinel : (base | sp_dep(r, t));
      SpV<R> w;
      w.x = wr;
      w.y = wi;
      out_amp[o + r] = w;
      nz += zero ? 1 : 0;
    }
    if (nz) atomicAdd(zeros, nz);
  }
}

// ---- uncontrolled one-qubit gates by merging ------------------------------------
// Entries with target bit 0 and those with bit 1 are each already in key
// order, so a stable split and a merge replace the first sort; the outputs
// with bit 0 and those with bit 1 are again each in index order, so a merge
// replaces the second.

__global__ __launch_bounds__(kSpBlock) void k_sp_bit_flags(const uint64_t* __restrict__ idx, uint64_t nnz, int t,
                                                           uint32_t* __restrict__ cnt) {
  for (uint64_t i = (uint64_t)blockIdx.x * kSpBlock + threadIdx.x; i < nnz; i += (uint64_t)gridDim.x * kSpBlock)
    cnt[i] = (uint32_t)((idx[i] >> t) & 1ull);
}

// Entries with the bit clear go to [0, nA) in order, those with it set to [nA, nnz).
template <typename R>
__global__ __launch_bounds__(kSpBlock) void k_sp_split(const uint64_t* __restrict__ key, const SpV<R>* __restrict__ amp,
                                                       const uint32_t* __restrict__ cnt,
                                                       const uint64_t* __restrict__ off, uint64_t nnz,
                                                       uint64_t* __restrict__ out_key, SpV<R>* __restrict__ out_amp) {
  const uint64_t nB = off[nnz - 1] + cnt[nnz - 1];
  const uint64_t nA = nnz - nB;
  for (uint64_t i = (uint64_t)blockIdx.x * kSpBlock + threadIdx.x; i < nnz; i += (uint64_t)gridDim.x * kSpBlock) {
    const uint64_t dst = cnt[i] ? nA + off[i] : i - off[i];
    out_key[dst] = key[i];
    out_amp[dst] = amp[i];
  }
}

__global__ __launch_bounds__(kSpBlock) void k_sp_head_flags(const uint64_t* __restrict__ skey, uint64_t nnz,
                                                            uint32_t* __restrict__ cnt) {
  for (uint64_t i = (uint64_t)blockIdx.x * kSpBlock + threadIdx.x; i < nnz; i += (uint64_t)gridDim.x * kSpBlock)
    cnt[i] = (i == 0 || (skey[i - 1] >> 1) != (skey[i] >> 1)) ? 1u : 0u;
}

// One thread per group (head at i, group number off[i]): w = U v, the bit-0
// output to o0[g], the bit-1 output to o1[g].
template <typename R>
__global__ __launch_bounds__(kSpBlock) void k_sp_apply1(const uint64_t* __restrict__ skey,
                                                        const SpV<R>* __restrict__ samp, uint64_t nnz, int t,
                                                        Mat2 u, const uint64_t* __restrict__ off,
                                                        uint64_t* __restrict__ o0_idx, SpV<R>* __restrict__ o0_amp,
                                                        uint64_t* __restrict__ o1_idx, SpV<R>* __restrict__ o1_amp,
                                                        unsigned long long* __restrict__ zeros) {
  const R a0 = (R)u.v[0], b0 = (R)u.v[1], a1 = (R)u.v[2], b1 = (R)u.v[3];
  const R a2 = (R)u.v[4], b2 = (R)u.v[5], a3 = (R)u.v[6], b3 = (R)u.v[7];
  const uint64_t lo = (1ull << t) - 1;
  for (uint64_t i = (uint64_t)blockIdx.x * kSpBlock + threadIdx.x; i < nnz; i += (uint64_t)gridDim.x * kSpBlock) {
    const uint64_t pre = skey[i] >> 1;
    if (i > 0 && (skey[i - 1] >> 1) == pre) continue;
    SpV<R> p, q;
    p.x = p.y = q.x = q.y = 0;
    if (skey[i] & 1) q = samp[i];
    else p = samp[i];
    if (i + 1 < nnz && (skey[i + 1] >> 1) == pre) q = samp[i + 1];   // the bit-1 member follows the bit-0 one
    SpV<R> r0, r1;
    r0.x = a0 * p.x - b0 * p.y + a1 * q.x - b1 * q.y;
    r0.y = a0 * p.y + b0 * p.x + a1 * q.y + b1 * q.x;
    r1.x = a2 * p.x - b2 * p.y + a3 * q.x - b3 * q.y;
    r1.y = a2 * p.y + b2 * p.x + a3 * q.y + b3 * q.x;
    const uint64_t base = ((pre >> t) << (t + 1)) | (pre & lo);
    const uint64_t g = off[i];
    o0_idx[g] = base;
    o0_amp[g] = r0;
    o1_idx[g] = base | (1ull << t);
    o1_amp[g] = r1;
    const unsigned long long z = (r0.x == (R)0 && r0.y == (R)0 ? 1ull : 0ull) + (r1.x == (R)0 && r1.y == (R)0 ? 1ull : 0ull);
    if (z) atomicAdd(zeros, z);
  }
}

template <typename R>
__global__ __launch_bounds__(kSpBlock) void k_sp_nonzero_flags(const SpV<R>* __restrict__ amp, uint64_t n,
                                                               uint32_t* __restrict__ cnt) {
  for (uint64_t i = (uint64_t)blockIdx.x * kSpBlock + threadIdx.x; i < n; i += (uint64_t)gridDim.x * kSpBlock) {
    const SpV<R> a = amp[i];
    cnt[i] = (a.x != (R)0 || a.y != (R)0) ? 1u : 0u;
  }
}

template <typename R>
__global__ __launch_bounds__(kSpBlock) void k_sp_gather_kept(const uint64_t* __restrict__ idx,
                                                             const SpV<R>* __restrict__ amp, uint64_t n,
                                                             const uint32_t* __restrict__ cnt,
                                                             const uint64_t* __restrict__ off,
                                                             uint64_t* __restrict__ out_idx,
                                                             SpV<R>* __restrict__ out_amp) {
  for (uint64_t i = (uint64_t)blockIdx.x * kSpBlock + threadIdx.x; i < n; i += (uint64_t)gridDim.x * kSpBlock) {
    if (!cnt[i]) continue;
    out_idx[off[i]] = idx[i];
    out_amp[off[i]] = amp[i];
  }
}

// ---- diagonal and phase gates --------------------------------------------------------

template <typename R>
__global__ __launch_bounds__(kSpBlock) void k_sp_diag(const uint64_t* __restrict__ idx, SpV<R>* __restrict__ amp,
                                                      uint64_t nnz, SpTargets t, uint64_t cmask, Diag64 d) {
  for (uint64_t i = (uint64_t)blockIdx.x * kSpBlock + threadIdx.x; i < nnz; i += (uint64_t)gridDim.x * kSpBlock) {
    const uint64_t x = idx[i];
    if ((x & cmask) != cmask) continue;
    const uint64_t m = sp_ext(x, t);
    const R dr = (R)d.v[2 * m], di = (R)d.v[2 * m + 1];
    const SpV<R> a = amp[i];
    SpV<R> b;
    b.x = a.x * dr - a.y * di;
    b.y = a.x * di + a.y * dr;
    amp[i] = b;
  }
}

// A run of diagonal gates in one pass: for each entry, in gate order, every
// term whose control bits are all 1 multiplies the amplitude by its table
// entry at the entry's target bits.
template <typename R>
__global__ __launch_bounds__(kSpBlock) void k_sp_diag_run(const uint64_t* __restrict__ idx, SpV<R>* __restrict__ amp,
                                                          uint64_t nnz, SpDiagRun run) {
  for (uint64_t i = (uint64_t)blockIdx.x * kSpBlock + threadIdx.x; i < nnz; i += (uint64_t)gridDim.x * kSpBlock) {
    const uint64_t x = idx[i];
    SpV<R> a = amp[i];
    for (int j = 0; j < run.n; ++j) {
      const SpDiagTerm& tm = run.t[j];
      if ((x & tm.cmask) != tm.cmask) continue;
      int m = 0;
      for (int b = 0; b < tm.k; ++b) m |= (int)((x >> tm.pos[b]) & 1ull) << b;
      const R dr = (R)tm.d[2 * m], di = (R)tm.d[2 * m + 1];
      SpV<R> r;
      r.x = a.x * dr - a.y * di;
      r.y = a.x * di + a.y * dr;
      a = r;
    }
    amp[i] = a;
  }
}

// ---- permutations ---------------------------------------------------------------------

__global__ __launch_bounds__(kSpBlock) void k_sp_perm_keys(const uint64_t* __restrict__ idx, uint64_t nnz,
                                                           SpTargets t, uint64_t cmask, int mode,
                                                           const uint32_t* __restrict__ ftab, uint64_t A, uint64_t B,
                                                           uint64_t N, uint64_t* __restrict__ key) {
  const uint64_t tmask = sp_dep((1ull << t.k) - 1, t);
  const uint64_t kmask = (t.k >= 64) ? ~0ull : ((1ull << t.k) - 1);
  // targets on consecutive bits in gate order (a register): plain shifts instead of bit loops
  bool contig = true;
  for (int j = 1; j < t.k; ++j) contig = contig && t.pos[j] == t.pos[0] + j;
  const int t0 = t.pos[0];
  for (uint64_t i = (uint64_t)blockIdx.x * kSpBlock + threadIdx.x; i < nnz; i += (uint64_t)gridDim.x * kSpBlock) {
    const uint64_t x = idx[i];
    if ((x & cmask) != cmask) {
      key[i] = x;
      continue;
    }
    const uint64_t m = contig ? ((x >> t0) & kmask) : sp_ext(x, t);
    uint64_t y;
    if (mode == SP_PERM_TABLE) y = ftab[m];
    else if (mode == SP_PERM_AFFINE) y = (A * m + B) & kmask;
    else if (mode == SP_PERM_MODMUL) {
      // (A m) mod N with A, m < N < 2^32: Barrett reduction with mu = floor((2^64 - 1) / N)
      // (the estimate q is at most 2 below the true quotient)
      if (m < N) {
        const uint64_t P = A * m;
        uint64_t r = P - __umul64hi(P, B) * N;
        while (r >= N) r -= N;
        y = r;
      } else {
        y = m;
      }
    }
    else y = ((m & 1ull) << 1) | ((m >> 1) & 1ull);       // swap of the two targets
    key[i] = (x & ~tmask) | (contig ? (y << t0) : sp_dep(y, t));
  }
}

// Physical index -> logical index: bit j of the result is bit phys.pos[j].
__global__ __launch_bounds__(kSpBlock) void k_sp_relabel(const uint64_t* __restrict__ idx, uint64_t nnz, SpTargets phys,
                                                         uint64_t* __restrict__ key) {
  for (uint64_t i = (uint64_t)blockIdx.x * kSpBlock + threadIdx.x; i < nnz; i += (uint64_t)gridDim.x * kSpBlock)
    key[i] = sp_ext(idx[i], phys);
}

// ---- measurement ------------------------------------------------------------------------

template <typename R>
__global__ __launch_bounds__(kSpBlock) void k_sp_prob_partial(const uint64_t* __restrict__ idx,
                                                              const SpV<R>* __restrict__ amp, uint64_t nnz,
                                                              uint64_t per_block, uint64_t qbit,
                                                              double* __restrict__ partials) {
  __shared__ double sh[2][4];
  const uint64_t start = (uint64_t)blockIdx.x * per_block;
  const uint64_t end = (start + per_block < nnz) ? start + per_block : nnz;
  double s0 = 0, s1 = 0;
  for (uint64_t i = start + threadIdx.x; i < end; i += kSpBlock) {
    const SpV<R> a = amp[i];
    const double p = (double)a.x * (double)a.x + (double)a.y * (double)a.y;
    if (idx[i] & qbit) s1 += p;
    else s0 += p;
  }
  s0 = sp_wave_sum(s0);
  s1 = sp_wave_sum(s1);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) {
    sh[0][w] = s0;
    sh[1][w] = s1;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    partials[2 * blockIdx.x] = ((sh[0][0] + sh[0][1]) + sh[0][2]) + sh[0][3];
    partials[2 * blockIdx.x + 1] = ((sh[1][0] + sh[1][1]) + sh[1][2]) + sh[1][3];
  }
}

// One thread: block sums in order, then the draw (or the forced outcome), the
// cbit, 1/sqrt(p_outcome) and a log entry.
__global__ void k_sp_meas_finalize(const double* __restrict__ partials, int nblocks, double u,
                                   const double* __restrict__ d_u, int forced, int cbit, double* __restrict__ result,
                                   uint8_t* __restrict__ cbits, double* __restrict__ log,
                                   uint32_t* __restrict__ log_count) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double p0 = 0, p1 = 0;
  for (int b = 0; b < nblocks; ++b) {
    p0 += partials[2 * b];
    p1 += partials[2 * b + 1];
  }
  const double P0 = p0 / (p0 + p1);
  const double uu = meas_draw(d_u ? *d_u : u);
  const int oc = forced >= 0 ? forced : ((uu < P0) ? 0 : 1);
  const double po = oc ? p1 : p0;
  const double scale = (po > 0.0) ? 1.0 / sqrt(po) : 0.0;
  result[0] = p0;
  result[1] = p1;
  result[2] = scale;
  result[3] = (double)oc;
  if (cbit >= 0 && po > 0.0) cbits[cbit] = (uint8_t)oc;
  const uint32_t c = *log_count;
  const uint32_t slot = c % (uint32_t)kMeasLog;
  log[3 * slot] = p0;
  log[3 * slot + 1] = p1;
  log[3 * slot + 2] = (double)oc;
  *log_count = c + 1;
}

__global__ __launch_bounds__(kSpBlock) void k_sp_keep_flags(const uint64_t* __restrict__ idx, uint64_t nnz, int q,
                                                            const double* __restrict__ result,
                                                            uint32_t* __restrict__ cnt) {
  const bool keep_all = result[2] == 0.0;     // impossible forced outcome: state left as it is
  const uint64_t oc = (uint64_t)result[3];
  for (uint64_t i = (uint64_t)blockIdx.x * kSpBlock + threadIdx.x; i < nnz; i += (uint64_t)gridDim.x * kSpBlock)
    cnt[i] = (keep_all || ((idx[i] >> q) & 1ull) == oc) ? 1u : 0u;
}

template <typename R>
__global__ __launch_bounds__(kSpBlock) void k_sp_compact(const uint64_t* __restrict__ idx,
                                                         const SpV<R>* __restrict__ amp, uint64_t nnz,
                                                         const uint32_t* __restrict__ cnt,
                                                         const uint64_t* __restrict__ off,
                                                         const double* __restrict__ result,
                                                         uint64_t* __restrict__ out_idx, SpV<R>* __restrict__ out_amp) {
  const double sd = result[2];
  const R s = sd == 0.0 ? (R)1 : (R)sd;
  for (uint64_t i = (uint64_t)blockIdx.x * kSpBlock + threadIdx.x; i < nnz; i += (uint64_t)gridDim.x * kSpBlock) {
    if (!cnt[i]) continue;
    const uint64_t o = off[i];
    out_idx[o] = idx[i];
    SpV<R> a = amp[i];
    a.x *= s;
    a.y *= s;
    out_amp[o] = a;
  }
}

// ---- norm and readout helpers -----------------------------------------------------------

template <typename R>
__global__ __launch_bounds__(kSpBlock) void k_sp_norm_partial(const SpV<R>* __restrict__ amp, uint64_t nnz,
                                                              uint64_t per_block, double* __restrict__ partials) {
  __shared__ double sh[4];
  const uint64_t start = (uint64_t)blockIdx.x * per_block;
  const uint64_t end = (start + per_block < nnz) ? start + per_block : nnz;
  double s = 0;
  for (uint64_t i = start + threadIdx.x; i < end; i += kSpBlock) {
    const SpV<R> a = amp[i];
    s += (double)a.x * (double)a.x + (double)a.y * (double)a.y;
  }
  s = sp_wave_sum(s);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) partials[blockIdx.x] = ((sh[0] + sh[1]) + sh[2]) + sh[3];
}

__global__ __launch_bounds__(kSpBlock) void k_sp_project(const uint64_t* __restrict__ idx,
                                                         const uint64_t* __restrict__ pos, uint64_t nshots,
                                                         SpTargets ql, uint64_t* __restrict__ out) {
  for (uint64_t s = (uint64_t)blockIdx.x * kSpBlock + threadIdx.x; s < nshots; s += (uint64_t)gridDim.x * kSpBlock) {
    const uint64_t p = pos[s];
    if (p == ~0ull) {                     // zero-norm state
      out[s] = ~0ull;
      continue;
    }
    const uint64_t i = idx[p];
    out[s] = ql.k ? sp_ext(i, ql) : i;
  }
}

template <typename R>
__global__ __launch_bounds__(kSpBlock) void k_sp_init(uint64_t* idx, SpV<R>* amp) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    idx[0] = 0;
    SpV<R> one;
    one.x = 1;
    one.y = 0;
    amp[0] = one;
  }
}

// ---- orchestration -------------------------------------------------------------------------

namespace {

template <typename R>
hipError_t sort_pairs(SpBufs& b, const uint64_t* kin, uint64_t* kout, const void* vin, void* vout, uint64_t n,
                      int bits, hipStream_t st) {
  if (n == 0) return hipSuccess;
  size_t bytes = b.temp_bytes;
  return rocprim::radix_sort_pairs(b.temp, bytes, kin, kout, (const SpV<R>*)vin, (SpV<R>*)vout, n, 0u,
                                   (unsigned)bits, st);
}

hipError_t scan_counts(SpBufs& b, uint64_t n, hipStream_t st) {
  if (n == 0) return hipSuccess;
  size_t bytes = b.temp_bytes;
  hipError_t e = rocprim::exclusive_scan(b.temp, bytes, b.cnt, b.off, (uint64_t)0, (size_t)n,
                                         rocprim::plus<uint64_t>(), st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_sp_total, dim3(1), dim3(64), 0, st, (const uint32_t*)b.cnt, (const uint64_t*)b.off, n, b.scal);
  return hipGetLastError();
}

// Below this many entries a sort costs about as much as the round trip that
// would tell whether it can be skipped.
constexpr uint64_t kCheckOrderMin = 1u << 15;

hipError_t check_order(SpBufs& b, const uint64_t* key, uint64_t n, bool* unsorted, hipStream_t st) {
  *unsorted = true;
  if (n < kCheckOrderMin) return hipSuccess;
  hipLaunchKernelGGL(k_sp_clear, dim3(1), dim3(64), 0, st, b.scal + 2, 1);
  hipLaunchKernelGGL(k_sp_check_order, dim3(sp_grid(n)), dim3(kSpBlock), 0, st, key, n, b.scal + 2);
  uint64_t flag = 1;
  hipError_t e = hipMemcpyAsync(&flag, b.scal + 2, sizeof flag, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  *unsorted = flag != 0;
  return e;
}

hipError_t read_scalars(SpBufs& b, uint64_t* host2, hipStream_t st) {
  hipError_t e = hipMemcpyAsync(host2, b.scal, 2 * sizeof(uint64_t), hipMemcpyDeviceToHost, st);
  if (e != hipSuccess) return e;
  return hipStreamSynchronize(st);
}

Special sorted_special(const SpTargets& t) {
  Special s{};
  s.n = t.k;
  for (int j = 0; j < t.k; ++j) s.pos[j] = t.pos[j];
  std::sort(s.pos, s.pos + s.n);
  return s;
}

template <typename R>
hipError_t dense_gate(SpBufs& b, int n, const SpTargets& t, uint64_t cmask, const void* d_mat, hipStream_t st) {
  const Special ts = sorted_special(t);
  const uint64_t nnz = b.nnz;
  hipLaunchKernelGGL(k_sp_keys, dim3(sp_grid(nnz)), dim3(kSpBlock), 0, st, (const uint64_t*)b.idx, nnz, ts, t, b.key);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  bool unsorted;
  if ((e = check_order(b, b.key, nnz, &unsorted, st)) != hipSuccess) return e;
  if (unsorted) {
    if ((e = sort_pairs<R>(b, b.key, b.idx_b, b.amp, b.amp_b, nnz, n, st)) != hipSuccess) return e;
  } else {   // already in key order: the keys and amplitudes move over as they are
    std::swap(b.key, b.idx_b);
    std::swap(b.amp, b.amp_b);
  }
  hipLaunchKernelGGL(k_sp_group_count, dim3(sp_grid(nnz)), dim3(kSpBlock), 0, st, (const uint64_t*)b.idx_b, nnz, ts,
                     t.k, cmask, b.cnt);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if ((e = scan_counts(b, nnz, st)) != hipSuccess) return e;
  uint64_t sc[2];
  if ((e = read_scalars(b, sc, st)) != hipSuccess) return e;
  const uint64_t total = sc[0];
  if (total > b.cap) return hipErrorOutOfMemory;
  const uint64_t sentinel = 1ull << n;
  hipLaunchKernelGGL((k_sp_group_apply<R>), dim3(sp_grid(nnz)), dim3(kSpBlock), 0, st, (const uint64_t*)b.idx_b,
                     (const SpV<R>*)b.amp_b, nnz, ts, t, cmask, (const SpV<R>*)d_mat, (const uint64_t*)b.off, sentinel,
                     b.key, (SpV<R>*)b.amp, (unsigned long long*)(b.scal + 1));
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if ((e = read_scalars(b, sc, st)) != hipSuccess) return e;
  const uint64_t zeros = sc[1];
  unsorted = true;
  if (zeros == 0 && (e = check_order(b, b.key, total, &unsorted, st)) != hipSuccess) return e;
  if (unsorted) {
    // ascending index order; exact zeros (sentinel index 2^n) sort to the end
    if ((e = sort_pairs<R>(b, b.key, b.idx, b.amp, b.amp_b, total, n + 1, st)) != hipSuccess) return e;
    std::swap(b.amp, b.amp_b);
  } else {
    std::swap(b.idx, b.key);
  }
  b.nnz = total - zeros;
  return hipSuccess;
}

template <typename R>
hipError_t merge_pairs(SpBufs& b, const uint64_t* k1, const uint64_t* k2, uint64_t* kout, const void* v1,
                       const void* v2, void* vout, uint64_t n1, uint64_t n2, hipStream_t st) {
  if (n1 + n2 == 0) return hipSuccess;
  size_t bytes = b.temp_bytes;
  return rocprim::merge(b.temp, bytes, k1, k2, kout, (const SpV<R>*)v1, (const SpV<R>*)v2, (SpV<R>*)vout,
                        (size_t)n1, (size_t)n2, rocprim::less<uint64_t>(), st);
}

// Uncontrolled one-qubit gate on target t by split, merge, apply, merge.
template <typename R>
hipError_t one_qubit(SpBufs& b, int n, int t, const Mat2& u, hipStream_t st) {
  const uint64_t nnz = b.nnz;
  SpTargets tt{};
  tt.k = 1;
  tt.pos[0] = t;
  const Special ts = sorted_special(tt);
  hipLaunchKernelGGL(k_sp_keys, dim3(sp_grid(nnz)), dim3(kSpBlock), 0, st, (const uint64_t*)b.idx, nnz, ts, tt, b.key);
  hipLaunchKernelGGL(k_sp_bit_flags, dim3(sp_grid(nnz)), dim3(kSpBlock), 0, st, (const uint64_t*)b.idx, nnz, t, b.cnt);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if ((e = scan_counts(b, nnz, st)) != hipSuccess) return e;
  hipLaunchKernelGGL((k_sp_split<R>), dim3(sp_grid(nnz)), dim3(kSpBlock), 0, st, (const uint64_t*)b.key,
                     (const SpV<R>*)b.amp, (const uint32_t*)b.cnt, (const uint64_t*)b.off, nnz, b.idx_b,
                     (SpV<R>*)b.amp_b);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  uint64_t sc[2];
  if ((e = read_scalars(b, sc, st)) != hipSuccess) return e;
  const uint64_t nB = sc[0], nA = nnz - nB;
  // entries in key order: keys into b.key, amplitudes into b.amp
  if ((e = merge_pairs<R>(b, b.idx_b, b.idx_b + nA, b.key, b.amp_b, (const SpV<R>*)b.amp_b + nA, b.amp, nA, nB,
                          st)) != hipSuccess)
    return e;
  hipLaunchKernelGGL(k_sp_head_flags, dim3(sp_grid(nnz)), dim3(kSpBlock), 0, st, (const uint64_t*)b.key, nnz, b.cnt);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if ((e = scan_counts(b, nnz, st)) != hipSuccess) return e;
  if ((e = read_scalars(b, sc, st)) != hipSuccess) return e;
  const uint64_t G = sc[0];
  if (2 * G > b.cap) return hipErrorOutOfMemory;
  hipLaunchKernelGGL((k_sp_apply1<R>), dim3(sp_grid(nnz)), dim3(kSpBlock), 0, st, (const uint64_t*)b.key,
                     (const SpV<R>*)b.amp, nnz, t, u, (const uint64_t*)b.off, b.idx_b, (SpV<R>*)b.amp_b, b.idx_b + G,
                     (SpV<R>*)b.amp_b + G, (unsigned long long*)(b.scal + 1));
  if ((e = hipGetLastError()) != hipSuccess) return e;
  // ascending index order again
  if ((e = merge_pairs<R>(b, b.idx_b, b.idx_b + G, b.idx, b.amp_b, (const SpV<R>*)b.amp_b + G, b.amp, G, G, st)) !=
      hipSuccess)
    return e;
  if ((e = read_scalars(b, sc, st)) != hipSuccess) return e;
  const uint64_t zeros = sc[1];
  b.nnz = 2 * G;
  if (zeros) {   // drop the exact zeros, keeping the order
    hipLaunchKernelGGL((k_sp_nonzero_flags<R>), dim3(sp_grid(b.nnz)), dim3(kSpBlock), 0, st, (const SpV<R>*)b.amp,
                       b.nnz, b.cnt);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if ((e = scan_counts(b, b.nnz, st)) != hipSuccess) return e;
    hipLaunchKernelGGL((k_sp_gather_kept<R>), dim3(sp_grid(b.nnz)), dim3(kSpBlock), 0, st, (const uint64_t*)b.idx,
                       (const SpV<R>*)b.amp, b.nnz, (const uint32_t*)b.cnt, (const uint64_t*)b.off, b.idx_b,
                       (SpV<R>*)b.amp_b);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    std::swap(b.idx, b.idx_b);
    std::swap(b.amp, b.amp_b);
    b.nnz -= zeros;
  }
  (void)n;
  return hipSuccess;
}

template <typename R>
hipError_t permute(SpBufs& b, int n, const SpTargets& t, uint64_t cmask, int mode, const uint32_t* ftab, uint64_t A,
                   uint64_t B, uint64_t N, hipStream_t st) {
  const uint64_t nnz = b.nnz;
  hipLaunchKernelGGL(k_sp_perm_keys, dim3(sp_grid(nnz)), dim3(kSpBlock), 0, st, (const uint64_t*)b.idx, nnz, t, cmask,
                     mode, ftab, A, B, N, b.key);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  bool unsorted;
  if ((e = check_order(b, b.key, nnz, &unsorted, st)) != hipSuccess) return e;
  if (unsorted) {
    if ((e = sort_pairs<R>(b, b.key, b.idx, b.amp, b.amp_b, nnz, n, st)) != hipSuccess) return e;
    std::swap(b.amp, b.amp_b);
  } else {   // the mapped indices are already ascending
    std::swap(b.idx, b.key);
  }
  return hipSuccess;
}

template <typename R>
hipError_t relabel(SpBufs& b, int n, const SpTargets& phys, hipStream_t st) {
  const uint64_t nnz = b.nnz;
  hipLaunchKernelGGL(k_sp_relabel, dim3(sp_grid(nnz)), dim3(kSpBlock), 0, st, (const uint64_t*)b.idx, nnz, phys, b.key);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if ((e = sort_pairs<R>(b, b.key, b.idx, b.amp, b.amp_b, nnz, n, st)) != hipSuccess) return e;
  std::swap(b.amp, b.amp_b);
  return hipSuccess;
}

template <typename R>
hipError_t measure(SpBufs& b, int q, int cbit, double u, const double* d_u, int forced, const MeasBuffers& mb,
                   hipStream_t st) {
  const uint64_t nnz = b.nnz;
  uint64_t nb = std::min<uint64_t>((uint64_t)kReduceBlocks, std::max<uint64_t>(1, nnz / 4096));
  const uint64_t per = (nnz + nb - 1) / nb;
  hipLaunchKernelGGL((k_sp_prob_partial<R>), dim3((unsigned)nb), dim3(kSpBlock), 0, st, (const uint64_t*)b.idx,
                     (const SpV<R>*)b.amp, nnz, per, 1ull << q, mb.partials);
  hipLaunchKernelGGL(k_sp_meas_finalize, dim3(1), dim3(64), 0, st, (const double*)mb.partials, (int)nb, u, d_u, forced,
                     cbit, mb.result, mb.cbits, mb.log, mb.log_count);
  hipLaunchKernelGGL(k_sp_keep_flags, dim3(sp_grid(nnz)), dim3(kSpBlock), 0, st, (const uint64_t*)b.idx, nnz, q,
                     (const double*)mb.result, b.cnt);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if ((e = scan_counts(b, nnz, st)) != hipSuccess) return e;
  hipLaunchKernelGGL((k_sp_compact<R>), dim3(sp_grid(nnz)), dim3(kSpBlock), 0, st, (const uint64_t*)b.idx,
                     (const SpV<R>*)b.amp, nnz, (const uint32_t*)b.cnt, (const uint64_t*)b.off,
                     (const double*)mb.result, b.idx_b, (SpV<R>*)b.amp_b);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  uint64_t sc[2];
  if ((e = read_scalars(b, sc, st)) != hipSuccess) return e;
  std::swap(b.idx, b.idx_b);
  std::swap(b.amp, b.amp_b);
  b.nnz = sc[0];
  return hipSuccess;
}

}  // namespace

size_t sp_temp_bytes(uint64_t cap, bool c64) {
  size_t a = 0, s = 0;
  uint64_t* kp = nullptr;
  if (c64)
    (void)rocprim::radix_sort_pairs(nullptr, a, kp, kp, (const float2*)nullptr, (float2*)nullptr, cap, 0u, 64u);
  else
    (void)rocprim::radix_sort_pairs(nullptr, a, kp, kp, (const double2*)nullptr, (double2*)nullptr, cap, 0u, 64u);
  (void)rocprim::exclusive_scan(nullptr, s, (const uint32_t*)nullptr, (uint64_t*)nullptr, (uint64_t)0, (size_t)cap,
                                rocprim::plus<uint64_t>());
  size_t m = 0;
  if (c64)
    (void)rocprim::merge(nullptr, m, kp, kp, kp, (const float2*)nullptr, (const float2*)nullptr, (float2*)nullptr,
                         (size_t)cap, (size_t)cap, rocprim::less<uint64_t>());
  else
    (void)rocprim::merge(nullptr, m, kp, kp, kp, (const double2*)nullptr, (const double2*)nullptr, (double2*)nullptr,
                         (size_t)cap, (size_t)cap, rocprim::less<uint64_t>());
  return std::max(std::max(a, s), m);
}

hipError_t sp_init(SpBufs& b, bool c64, hipStream_t st) {
  if (c64) hipLaunchKernelGGL(k_sp_init<float>, dim3(1), dim3(64), 0, st, b.idx, (float2*)b.amp);
  else hipLaunchKernelGGL(k_sp_init<double>, dim3(1), dim3(64), 0, st, b.idx, (double2*)b.amp);
  b.nnz = 1;
  return hipGetLastError();
}

hipError_t sp_one_qubit(SpBufs& b, int n, bool c64, int t, const Mat2& u, hipStream_t st) {
  return c64 ? one_qubit<float>(b, n, t, u, st) : one_qubit<double>(b, n, t, u, st);
}

hipError_t sp_dense_gate(SpBufs& b, int n, bool c64, const SpTargets& t, uint64_t cmask, const void* d_mat,
                         hipStream_t st) {
  return c64 ? dense_gate<float>(b, n, t, cmask, d_mat, st) : dense_gate<double>(b, n, t, cmask, d_mat, st);
}

hipError_t sp_diag(SpBufs& b, bool c64, const SpTargets& t, uint64_t cmask, const Diag64& d, hipStream_t st) {
  if (b.nnz == 0) return hipSuccess;
  if (c64)
    hipLaunchKernelGGL(k_sp_diag<float>, dim3(sp_grid(b.nnz)), dim3(kSpBlock), 0, st, (const uint64_t*)b.idx,
                       (float2*)b.amp, b.nnz, t, cmask, d);
  else
    hipLaunchKernelGGL(k_sp_diag<double>, dim3(sp_grid(b.nnz)), dim3(kSpBlock), 0, st, (const uint64_t*)b.idx,
                       (double2*)b.amp, b.nnz, t, cmask, d);
  return hipGetLastError();
}

hipError_t sp_diag_run(SpBufs& b, bool c64, const SpDiagRun& run, hipStream_t st) {
  if (b.nnz == 0 || run.n == 0) return hipSuccess;
  if (c64)
    hipLaunchKernelGGL(k_sp_diag_run<float>, dim3(sp_grid(b.nnz)), dim3(kSpBlock), 0, st, (const uint64_t*)b.idx,
                       (float2*)b.amp, b.nnz, run);
  else
    hipLaunchKernelGGL(k_sp_diag_run<double>, dim3(sp_grid(b.nnz)), dim3(kSpBlock), 0, st, (const uint64_t*)b.idx,
                       (double2*)b.amp, b.nnz, run);
  return hipGetLastError();
}

hipError_t sp_permute(SpBufs& b, int n, bool c64, const SpTargets& t, uint64_t cmask, int mode, const uint32_t* ftab,
                      uint64_t A, uint64_t B, uint64_t N, hipStream_t st) {
  return c64 ? permute<float>(b, n, t, cmask, mode, ftab, A, B, N, st)
             : permute<double>(b, n, t, cmask, mode, ftab, A, B, N, st);
}

hipError_t sp_relabel(SpBufs& b, int n, bool c64, const SpTargets& phys, hipStream_t st) {
  return c64 ? relabel<float>(b, n, phys, st) : relabel<double>(b, n, phys, st);
}

hipError_t sp_measure(SpBufs& b, bool c64, int q, int cbit, double u, const double* d_u, int forced,
                      const MeasBuffers& mb, hipStream_t st) {
  return c64 ? measure<float>(b, q, cbit, u, d_u, forced, mb, st) : measure<double>(b, q, cbit, u, d_u, forced, mb, st);
}

hipError_t sp_norm_partials(const SpBufs& b, bool c64, double* partials, int nblocks, hipStream_t st) {
  const uint64_t per = (b.nnz + nblocks - 1) / nblocks;
  if (c64)
    hipLaunchKernelGGL(k_sp_norm_partial<float>, dim3(nblocks), dim3(kSpBlock), 0, st, (const float2*)b.amp, b.nnz,
                       per, partials);
  else
    hipLaunchKernelGGL(k_sp_norm_partial<double>, dim3(nblocks), dim3(kSpBlock), 0, st, (const double2*)b.amp, b.nnz,
                       per, partials);
  return hipGetLastError();
}

hipError_t sp_project(const SpBufs& b, const uint64_t* pos, uint64_t nshots, const SpTargets& ql, uint64_t* d_out,
                      hipStream_t st) {
  if (nshots == 0) return hipSuccess;
  hipLaunchKernelGGL(k_sp_project, dim3(sp_grid(nshots)), dim3(kSpBlock), 0, st, (const uint64_t*)b.idx, pos, nshots,
                     ql, d_out);
  return hipGetLastError();
}

}  // namespace qk
