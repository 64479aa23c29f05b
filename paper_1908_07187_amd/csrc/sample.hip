// Deferred measurement on gfx950: shots drawn from the state without
// collapsing it (the paper lets qubits be measured in place or at the end,
// section "Q-Kit."), via a cumulative distribution of |psi_i|^2 in FP64.
//
// The index space is cut into segments of 256 amplitudes (4 rows of 64, one
// amplitude per lane per row, so every load instruction of a wave is one
// contiguous 1 KiB / 512 B run) and chunks of 64 segments (16384 amplitudes).
//
//   k_cdf_segments  one read sweep: each wave sums one chunk; lane l adds its
//                   4 row weights in row order, a fixed xor tree adds lanes ->
//                   segment sum; the chunk sum is the same tree over its 64
//                   segment sums.  Writes 1/256 (c64: 1/128) of the state's
//                   bytes.
//   k_cdf_scan      one block: exclusive prefix of the chunk sums.  Thread t
//                   owns a contiguous run of chunks; prefix[c] = E_t + I_c,
//                   with E_t the sequential sum of the earlier runs' totals
//                   and I_c the sequential sum of the run before c.  The run
//                   total is the same sequence of additions as I, so a chunk
//                   of zero weight gets an interval of length exactly zero
//                   and a draw can never land in it.
//   k_sample        one wave per shot: binary search of the chunk prefix,
//                   then an inclusive lane scan over the chunk's 64 segment
//                   sums, then over the segment's rows and lanes.  Each level
//                   takes the first element whose running sum exceeds the
//                   residual and whose weight is positive; when rounding leaves
//                   the residual past the level's own total it takes the last
//                   element of positive weight.  The drawn index is therefore
//                   always one of positive weight, and equals the exact
//                   inverse-CDF index unless the draw lies within rounding of
//                   an interval boundary.
//
// The marginal distribution over a qubit list is a gather: row m of the
// (2^nq x 2^(n-nq)) table of weights, the complement bits enumerated in
// ascending index order, is summed by one block per (m, slab) tile with a
// fixed thread mapping and tree, then the slabs are added in order.
#include <algorithm>

#include "qk_internal.h"

namespace qk {
namespace {

template <typename R> struct AmpT;
template <> struct AmpT<float> { using T = float2; };
template <> struct AmpT<double> { using T = double2; };
template <typename R> using Amp = typename AmpT<R>::T;

constexpr int kRows = 4;
constexpr int kSeg = 64 * kRows;
constexpr int kChunkSegs = 64;
constexpr uint64_t kChunk = (uint64_t)kSeg * kChunkSegs;
constexpr int kScanThreads = 1024;

template <typename R>
__device__ __forceinline__ double weight(const Amp<R>* __restrict__ psi, uint64_t i, uint64_t dim) {
  if (i >= dim) return 0.0;
  const Amp<R> a = psi[i];
  const double re = a.x, im = a.y;
  return re * re + im * im;
}

// Fixed xor tree over the 64 lanes; every lane gets the sum.
__device__ __forceinline__ double wave_total(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Inclusive scan in lane order (fixed Hillis-Steele steps).
__device__ __forceinline__ double wave_scan(double v, int lane) {
  for (int off = 1; off < 64; off <<= 1) {
    const double o = __shfl_up(v, off, 64);
    if (lane >= off) v += o;
  }
  return v;
}

__device__ __forceinline__ int first_lane(uint64_t m) { return __ffsll((unsigned long long)m) - 1; }
__device__ __forceinline__ int last_lane(uint64_t m) { return 63 - __clzll((unsigned long long)m); }

struct QubitList {
  int n;
  int q[QK_MAX_GATE_QUBITS];
};

__device__ __forceinline__ uint64_t project(uint64_t i, const QubitList& ql) {
  if (ql.n == 0) return i;
  uint64_t o = 0;
  for (int j = 0; j < ql.n; ++j) o |= ((i >> ql.q[j]) & 1ull) << j;
  return o;
}

struct Positions {
  int n;
  int p[QK_MAX_GATE_QUBITS];
};

constexpr uint64_t kMaxGrid = 1u << 20;   // blocks per launch; the kernels loop past it

inline unsigned blocks_for(uint64_t items, uint64_t per) {
  return (unsigned)std::min<uint64_t>(kMaxGrid, std::max<uint64_t>(1, (items + per - 1) / per));
}

}  // namespace

template <typename R>
__global__ __launch_bounds__(256) void k_cdf_segments(const Amp<R>* __restrict__ psi, uint64_t dim, uint64_t nseg,
                                                      uint64_t nchunk, double* __restrict__ seg_sum,
                                                      double* __restrict__ chunk_sum) {
  const int lane = threadIdx.x & 63;
  const uint64_t chunk = (uint64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (chunk >= nchunk) return;   // whole wave
  const uint64_t g0 = chunk * kChunkSegs;
  double mine = 0.0;
#pragma unroll 4
  for (int r = 0; r < kChunkSegs; ++r) {
    const uint64_t base = (g0 + r) * kSeg + lane;
    double acc = 0.0;
#pragma unroll
    for (int j = 0; j < kRows; ++j) acc += weight<R>(psi, base + 64 * j, dim);
    const double s = wave_total(acc);
    if (lane == r) mine = s;
  }
  if (g0 + lane < nseg) seg_sum[g0 + lane] = mine;
  const double t = wave_total(mine);
  if (lane == 0) chunk_sum[chunk] = t;
}

__global__ __launch_bounds__(kScanThreads) void k_cdf_scan(const double* __restrict__ chunk_sum, uint64_t nchunk,
                                                           double* __restrict__ prefix) {
  __shared__ double run_start[kScanThreads];
  const int t = threadIdx.x;
  const uint64_t per = (nchunk + kScanThreads - 1) / kScanThreads;
  const uint64_t a = std::min<uint64_t>(nchunk, (uint64_t)t * per);
  const uint64_t b = std::min<uint64_t>(nchunk, a + per);
  double local = 0.0;
#pragma unroll 8
  for (uint64_t c = a; c < b; ++c) local += chunk_sum[c];
  run_start[t] = local;
  __syncthreads();
  if (t == 0) {
    double e = 0.0;
#pragma unroll 16
    for (int i = 0; i < kScanThreads; ++i) {
      const double v = run_start[i];
      run_start[i] = e;
      e += v;
    }
    prefix[nchunk] = e;
  }
  __syncthreads();
  const double base = run_start[t];
  double inner = 0.0;
#pragma unroll 8
  for (uint64_t c = a; c < b; ++c) {
    prefix[c] = base + inner;
    inner += chunk_sum[c];
  }
}

template <typename R>
__global__ __launch_bounds__(256) void k_sample(const Amp<R>* __restrict__ psi, uint64_t dim, uint64_t nseg,
                                                uint64_t nchunk, const double* __restrict__ seg_sum,
                                                const double* __restrict__ prefix, const double* __restrict__ u,
                                                uint64_t nshots, QubitList ql, uint64_t* __restrict__ out) {
  const int lane = threadIdx.x & 63;
  const double T = prefix[nchunk];
  const uint64_t waves = (uint64_t)gridDim.x * 4;
  for (uint64_t s = (uint64_t)blockIdx.x * 4 + (threadIdx.x >> 6); s < nshots; s += waves) {   // whole waves
    if (!(T > 0.0)) {
      if (lane == 0) out[s] = ~0ull;
      continue;
    }
    double target = u[s] * T;
    if (!(target >= 0.0)) target = 0.0;            // negative or NaN draw
    if (!(target < T)) target = nextafter(T, 0.0);  // a draw that rounded onto the total

    // chunk: the largest c with prefix[c] <= target (prefix[0] = 0)
    uint64_t lo = 0, hi = nchunk - 1;
    while (lo < hi) {
      const uint64_t mid = lo + (hi - lo + 1) / 2;
      if (prefix[mid] <= target) lo = mid;
      else hi = mid - 1;
    }
    const uint64_t g0 = lo * kChunkSegs;
    const double r = target - prefix[lo];

    // segment within the chunk
    const double v = (g0 + lane < nseg) ? seg_sum[g0 + lane] : 0.0;
    const double q = wave_scan(v, lane);
    double ex = __shfl_up(q, 1, 64);
    if (lane == 0) ex = 0.0;
    const uint64_t hit = __ballot(q > r && v > 0.0);
    const int k = hit ? first_lane(hit) : last_lane(__ballot(v > 0.0));
    double rr = r - __shfl(ex, k, 64);
    if (!(rr >= 0.0)) rr = 0.0;

    // row, then lane, within the segment
    const uint64_t base = (g0 + k) * kSeg;
    double p[kRows], rows[kRows];
#pragma unroll
    for (int j = 0; j < kRows; ++j) p[j] = weight<R>(psi, base + 64 * j + lane, dim);
#pragma unroll
    for (int j = 0; j < kRows; ++j) rows[j] = wave_total(p[j]);
    int J = -1;
    double cum = 0.0;
#pragma unroll
    for (int j = 0; j < kRows; ++j) {
      if (J < 0) {
        if (rows[j] > 0.0 && cum + rows[j] > rr) J = j;
        else cum += rows[j];
      }
    }
    double rrr = rr - cum;
    if (J < 0) {                    // residual past the segment's total: its last weighted amplitude
#pragma unroll
      for (int j = 0; j < kRows; ++j)
        if (rows[j] > 0.0) J = j;
      rrr = __builtin_inf();
    }
    if (!(rrr >= 0.0)) rrr = 0.0;
    double pj = p[0];
#pragma unroll
    for (int j = 1; j < kRows; ++j)
      if (j == J) pj = p[j];
    const double Q = wave_scan(pj, lane);
    const uint64_t hit2 = __ballot(Q > rrr && pj > 0.0);
    const int L = hit2 ? first_lane(hit2) : last_lane(__ballot(pj > 0.0));
    if (lane == 0) out[s] = project(base + 64 * (uint64_t)J + (uint64_t)L, ql);
  }
}

// ---- marginal distribution ----------------------------------------------------

// Tile = (row m, slab of 2^slab_bits complement indices).  The complement
// index c maps to the amplitude index by inserting zeros at the listed
// qubits' positions (ascending) and or-ing in the row's bits.  Thread t sums
// c = t, t + 256, ... of its slab in order; a fixed tree adds the threads.
template <typename R>
__global__ __launch_bounds__(256) void k_marginal_tiles(const Amp<R>* __restrict__ psi, Positions rows,
                                                        Positions sorted, int slab_bits, uint64_t nslabs,
                                                        uint64_t ntiles, double* __restrict__ partial) {
  __shared__ double sh[4];
  const uint64_t per = 1ull << slab_bits;
  for (uint64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const uint64_t m = tile / nslabs, slab = tile % nslabs;
    uint64_t rowbase = 0;
    for (int j = 0; j < rows.n; ++j) rowbase |= ((m >> j) & 1ull) << rows.p[j];
    double acc = 0.0;
    for (uint64_t c = threadIdx.x; c < per; c += 256) {
      uint64_t i = slab * per + c;
      for (int j = 0; j < sorted.n; ++j) {
        const int b = sorted.p[j];
        i = ((i >> b) << (b + 1)) | (i & ((1ull << b) - 1));
      }
      const Amp<R> a = psi[i | rowbase];
      const double re = a.x, im = a.y;
      acc += re * re + im * im;
    }
    acc = wave_total(acc);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) sh[w] = acc;
    __syncthreads();
    if (threadIdx.x == 0) partial[tile] = ((sh[0] + sh[1]) + sh[2]) + sh[3];
    __syncthreads();
  }
}

__global__ __launch_bounds__(256) void k_marginal_rows(const double* __restrict__ partial, uint64_t nslabs,
                                                       uint64_t nrows, double* __restrict__ out) {
  for (uint64_t m = (uint64_t)blockIdx.x * 256 + threadIdx.x; m < nrows; m += (uint64_t)gridDim.x * 256) {
    double s = 0.0;
    for (uint64_t k = 0; k < nslabs; ++k) s += partial[m * nslabs + k];
    out[m] = s;
  }
}

SampleLayout sample_layout_dim(uint64_t dim) {
  SampleLayout s;
  s.nseg = (dim + kSeg - 1) / kSeg;
  s.nchunk = (s.nseg + kChunkSegs - 1) / kChunkSegs;
  s.doubles = s.nseg + s.nchunk + (s.nchunk + 1);
  return s;
}

SampleLayout sample_layout(int n) { return sample_layout_dim(1ull << n); }

hipError_t launch_cdf_dim(const void* psi, uint64_t dim, bool c64, hipStream_t st, double* work) {
  const SampleLayout sl = sample_layout_dim(dim);
  double* seg = work;
  double* chunk = seg + sl.nseg;
  double* prefix = chunk + sl.nchunk;
  const unsigned g = blocks_for(sl.nchunk, 4);
  if (c64)
    hipLaunchKernelGGL(k_cdf_segments<float>, dim3(g), dim3(256), 0, st, (const float2*)psi, dim, sl.nseg, sl.nchunk,
                       seg, chunk);
  else
    hipLaunchKernelGGL(k_cdf_segments<double>, dim3(g), dim3(256), 0, st, (const double2*)psi, dim, sl.nseg,
                       sl.nchunk, seg, chunk);
  hipLaunchKernelGGL(k_cdf_scan, dim3(1), dim3(kScanThreads), 0, st, (const double*)chunk, sl.nchunk, prefix);
  return hipGetLastError();
}

static hipError_t draw(const void* psi, uint64_t dim, bool c64, hipStream_t st, const double* work, const int* qubits,
                       int nq, const double* d_u, uint64_t nshots, uint64_t* d_out) {
  if (nshots == 0) return hipSuccess;
  const SampleLayout sl = sample_layout_dim(dim);
  const double* seg = work;
  const double* prefix = work + sl.nseg + sl.nchunk;
  QubitList ql{};
  ql.n = nq;
  for (int j = 0; j < nq; ++j) ql.q[j] = qubits[j];
  const unsigned g = blocks_for(nshots, 4);
  if (c64)
    hipLaunchKernelGGL(k_sample<float>, dim3(g), dim3(256), 0, st, (const float2*)psi, dim, sl.nseg, sl.nchunk, seg,
                       prefix, d_u, nshots, ql, d_out);
  else
    hipLaunchKernelGGL(k_sample<double>, dim3(g), dim3(256), 0, st, (const double2*)psi, dim, sl.nseg, sl.nchunk, seg,
                       prefix, d_u, nshots, ql, d_out);
  return hipGetLastError();
}

hipError_t launch_draw_dim(const void* psi, uint64_t dim, bool c64, hipStream_t st, const double* work,
                           const double* d_u, uint64_t nshots, uint64_t* d_out) {
  return draw(psi, dim, c64, st, work, nullptr, 0, d_u, nshots, d_out);
}

hipError_t launch_cdf(const Launch& L, double* work) { return launch_cdf_dim(L.psi, 1ull << L.n, L.c64, L.stream, work); }

hipError_t launch_draw(const Launch& L, const double* work, const int* qubits, int nq, const double* d_u,
                       uint64_t nshots, uint64_t* d_out) {
  return draw(L.psi, 1ull << L.n, L.c64, L.stream, work, qubits, nq, d_u, nshots, d_out);
}

MarginalLayout marginal_layout(int n, int nq) {
  MarginalLayout m;
  const int cbits = n - nq;
  m.nrows = 1ull << nq;
  m.slab_bits = std::min(cbits, 14);
  m.nslabs = 1ull << (cbits - m.slab_bits);
  m.partial_doubles = m.nrows * m.nslabs;
  return m;
}

hipError_t launch_marginal(const Launch& L, const int* qubits, int nq, double* partial, double* d_out) {
  const MarginalLayout ml = marginal_layout(L.n, nq);
  Positions rows{}, sorted{};
  rows.n = sorted.n = nq;
  for (int j = 0; j < nq; ++j) rows.p[j] = sorted.p[j] = qubits[j];
  std::sort(sorted.p, sorted.p + nq);
  const uint64_t tiles = ml.nrows * ml.nslabs;
  const unsigned g = blocks_for(tiles, 1);
  if (L.c64)
    hipLaunchKernelGGL(k_marginal_tiles<float>, dim3(g), dim3(256), 0, L.stream, (const float2*)L.psi, rows, sorted,
                       ml.slab_bits, ml.nslabs, tiles, partial);
  else
    hipLaunchKernelGGL(k_marginal_tiles<double>, dim3(g), dim3(256), 0, L.stream, (const double2*)L.psi, rows,
                       sorted, ml.slab_bits, ml.nslabs, tiles, partial);
  hipLaunchKernelGGL(k_marginal_rows, dim3(blocks_for(ml.nrows, 256)), dim3(256), 0, L.stream, (const double*)partial,
                     ml.nslabs, ml.nrows, d_out);
  return hipGetLastError();
}

}  // namespace qk
