// Per-gate state sweeps for gfx950: one pass over the amplitudes a gate may
// change, in place, coalesced.  Every kernel evaluates the gate's classical
// conditions on the device first and exits uniformly when one fails, so
// measurement outcomes steer later gates without a host round trip.
#include <algorithm>
#include <mutex>
#include <type_traits>

#include "qk_internal.h"

namespace qk {

template <typename R> struct V2T;
template <> struct V2T<float> { using T = float2; };
template <> struct V2T<double> { using T = double2; };
template <typename R> using V2 = typename V2T<R>::T;

struct Pos32 {
  int p[32];
};

__device__ __forceinline__ bool conds_ok(const CondArgs& c) {
  for (int i = 0; i < c.n; ++i)
    if (c.cbits[c.cbit[i]] != (uint8_t)c.val[i]) return false;
  return true;
}

// Insert a zero bit at each (ascending) special position of the compact counter x.
__device__ __forceinline__ uint64_t insert_zeros(uint64_t x, const Special& s) {
  for (int i = 0; i < s.n; ++i) {
    const int p = s.pos[i];
    const uint64_t lo = x & ((1ull << p) - 1);
    x = ((x >> p) << (p + 1)) | lo;
  }
  return x;
}

// Gate index m of amplitude i: bit j of m = bit pos[j] of i.
__device__ __forceinline__ uint64_t extract(uint64_t i, const int* pos, int k) {
  uint64_t m = 0;
  for (int j = 0; j < k; ++j) m |= ((i >> pos[j]) & 1ull) << j;
  return m;
}
__device__ __forceinline__ uint64_t deposit(uint64_t m, const int* pos, int k) {
  uint64_t i = 0;
  for (int j = 0; j < k; ++j) i |= ((m >> j) & 1ull) << pos[j];
  return i;
}

// Workgroups are dealt to the 8 XCDs round-robin.  Renumbering them so that
// each XCD sweeps one contiguous eighth of the launch measured 2-8 % faster
// for in-place sweeps of a 16 GiB state; grids whose size is not a multiple of
// 8 keep the plain order.
// One grid dimension holds fewer than 2^32 work-items, and a one-shot sweep of
// 32 or more qubits needs more, so a grid of more than kGridRow workgroups is
// laid out as rows of kGridRow (a multiple of 8, so every row starts on XCD 0)
// and the kernels read their position in launch order with flat_block().
constexpr uint64_t kGridRow = 1ull << 22;

__device__ __forceinline__ uint64_t flat_block() { return (uint64_t)blockIdx.y * gridDim.x + blockIdx.x; }
__device__ __forceinline__ uint64_t flat_grid() { return (uint64_t)gridDim.y * gridDim.x; }

__device__ __forceinline__ uint64_t sweep_block(bool xcd) {
  const uint64_t b = flat_block(), g = flat_grid();
  if (!xcd || (g & 7)) return b;
  return (b & 7) * (g >> 3) + (b >> 3);
}

// Workgroups for `items` work items at `per_block` per workgroup, as rows of
// kGridRow when there are more than that.  Workgroups past the end (at most
// kGridRow - 1 in the last row) find no item in range and exit; every kernel
// launched this way checks its items against the count.
static inline dim3 grid_for(uint64_t items, int per_block) {
  const uint64_t g = std::max<uint64_t>(1, (items + per_block - 1) / per_block);
  if (g <= kGridRow) return dim3((unsigned)g);
  return dim3((unsigned)kGridRow, (unsigned)((g + kGridRow - 1) / kGridRow));
}

Special make_special(const int* a, int na, const int* b, int nb, const int* c, int nc) {
  std::vector<int> v;
  for (int i = 0; i < na; ++i) v.push_back(a[i]);
  for (int i = 0; i < nb; ++i) v.push_back(b[i]);
  for (int i = 0; i < nc; ++i) v.push_back(c[i]);
  std::sort(v.begin(), v.end());
  v.erase(std::unique(v.begin(), v.end()), v.end());
  Special s{};
  s.n = (int)std::min<size_t>(v.size(), kMaxSpecial);   // callers pass at most 46 (40 gate qubits + 6 tile bits)
  for (int i = 0; i < s.n; ++i) s.pos[i] = v[i];
  return s;
}

static uint64_t mask_of(const int* q, int nq) {
  uint64_t m = 0;
  for (int i = 0; i < nq; ++i) m |= 1ull << q[i];
  return m;
}

// ---------------------------------------------------------------- fill / copy

template <typename R>
__global__ __launch_bounds__(kBlock) void k_fill_zero(V2<R>* p, uint64_t from, uint64_t to) {
  const uint64_t stride = (uint64_t)gridDim.x * kBlock;
  for (uint64_t i = from + (uint64_t)blockIdx.x * kBlock + threadIdx.x; i < to; i += stride) p[i] = V2<R>{0, 0};
}

template <typename R>
__global__ void k_set_one(V2<R>* p, uint64_t idx) {
  if (threadIdx.x == 0 && blockIdx.x == 0) p[idx] = V2<R>{1, 0};
}

template <typename R>
__global__ __launch_bounds__(kBlock) void k_copy(V2<R>* __restrict__ dst, const V2<R>* __restrict__ src, uint64_t n) {
  const uint64_t stride = (uint64_t)gridDim.x * kBlock;
  for (uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += stride) dst[i] = src[i];
}

hipError_t launch_fill_zero(void* p, uint64_t from, uint64_t to, bool c64, hipStream_t s) {
  if (to <= from) return hipSuccess;
  const unsigned g = (unsigned)std::min<uint64_t>((to - from + kBlock * 4 - 1) / (kBlock * 4), 65536);
  if (c64) hipLaunchKernelGGL(k_fill_zero<float>, dim3(g), dim3(kBlock), 0, s, (float2*)p, from, to);
  else hipLaunchKernelGGL(k_fill_zero<double>, dim3(g), dim3(kBlock), 0, s, (double2*)p, from, to);
  return hipGetLastError();
}

hipError_t launch_set_one(void* p, uint64_t idx, bool c64, hipStream_t s) {
  if (c64) hipLaunchKernelGGL(k_set_one<float>, dim3(1), dim3(64), 0, s, (float2*)p, idx);
  else hipLaunchKernelGGL(k_set_one<double>, dim3(1), dim3(64), 0, s, (double2*)p, idx);
  return hipGetLastError();
}

hipError_t launch_copy(void* dst, const void* src, uint64_t count, bool c64, hipStream_t s) {
  if (!count) return hipSuccess;
  const unsigned g = (unsigned)std::min<uint64_t>((count + kBlock * 4 - 1) / (kBlock * 4), 65536);
  if (c64) hipLaunchKernelGGL(k_copy<float>, dim3(g), dim3(kBlock), 0, s, (float2*)dst, (const float2*)src, count);
  else hipLaunchKernelGGL(k_copy<double>, dim3(g), dim3(kBlock), 0, s, (double2*)dst, (const double2*)src, count);
  return hipGetLastError();
}

// ---------------------------------------------------------------- load / store policy
// A gate sweep touches each byte once.  When a wave's accesses cover whole
// cache lines, loads and stores are issued non-temporal (streaming) so the
// sweep does not churn the caches; when the two halves of a line are read by
// different instructions (target or control on a low bit), the regular policy
// lets the second read hit in cache.

template <typename R> struct EV;
template <> struct EV<float> { typedef float T __attribute__((ext_vector_type(2))); };
template <> struct EV<double> { typedef double T __attribute__((ext_vector_type(2))); };
template <typename R> using CV = typename EV<R>::T;

template <bool NT, typename T>
__device__ __forceinline__ T ld(const T* p) {
  if constexpr (NT) return __builtin_nontemporal_load(p);
  else return *p;
}
template <bool NT, typename T>
__device__ __forceinline__ void st(T* p, T v) {
  if constexpr (NT) __builtin_nontemporal_store(v, p);
  else *p = v;
}

// Non-temporal only for a state larger than the Infinity Cache, and when
// every run of consecutive amplitudes an instruction touches is at least 256
// bytes long (the lowest zero-inserted bit sets it).
static bool use_nt(const Launch& L, int lowest_special) {
  if (L.tune.nt == 0) return false;
  if (L.tune.nt == 2) return true;
  if (!state_streams(L)) return false;
  return lowest_special >= (L.c64 ? 5 : 4);
}
static int lowest(const int* a, int na, const int* b, int nb, int dflt) {
  int m = dflt;
  for (int i = 0; i < na; ++i) m = std::min(m, a[i]);
  for (int i = 0; i < nb; ++i) m = std::min(m, b[i]);
  return m;
}

// ---------------------------------------------------------------- 2x2 butterfly
// For every index pair (i, i | 2^t) with bit t of i = 0 and all control bits
// 1: [a_i, a_{i+2^t}] <- U [a_i, a_{i+2^t}].
//
// k_butterfly: each wave owns 32 pairs per item; lanes 0-31 load the lower
// amplitudes (bit t = 0) and lanes 32-63 the upper ones, so every thread moves
// one amplitude each way and the partner arrives by a cross-lane exchange
// between the two half-waves.  Measured on a 30-qubit complex128 state this is
// 6 % faster on average over targets 6-29 than a thread loading both halves
// of its pair (two loads in flight per thread run slower than one, as in a
// plain read-modify-write sweep).  Items are strided by the block's pair
// count, so each load instruction covers two runs of 32 amplitudes.
// Controls at or above bit 4 (complex128) / 5 (complex64) are skipped in the
// enumeration (only the controlled subspace is touched); lower controls would
// leave partial cache lines, so they are evaluated as a per-pair predicate of
// a full sweep instead.  (The CTRL flag only separates controlled launches,
// e.g. CNOT, into their own kernel symbol for profiling.)

constexpr int kPairsPerBlock = kBlock / 2;

template <typename R, int ITEMS, bool NT, bool CTRL>
__global__ __launch_bounds__(kBlock) void k_butterfly(CV<R>* __restrict__ psi, uint64_t npairs, Special sp,
                                                      uint64_t cmask, uint64_t pmask, uint64_t tbit, Mat2 u,
                                                      CondArgs cond, bool xcd) {
  if (!conds_ok(cond)) return;
  const int lane = threadIdx.x & 63;
  const bool up = lane >= 32;
  // lower half: u00 a + u01 b; upper half: u11 a + u10 b (b = the partner)
  const R sr = (R)(up ? u.v[6] : u.v[0]), si = (R)(up ? u.v[7] : u.v[1]);
  const R orr = (R)(up ? u.v[4] : u.v[2]), oi = (R)(up ? u.v[5] : u.v[3]);
  const uint64_t half = up ? tbit : 0;
  const uint64_t j0 = sweep_block(xcd) * (kPairsPerBlock * ITEMS) + (threadIdx.x >> 6) * 32 + (lane & 31);
  CV<R> a[ITEMS];
  uint64_t idx[ITEMS];
#pragma unroll
  for (int k = 0; k < ITEMS; ++k) {
    const uint64_t j = j0 + (uint64_t)k * kPairsPerBlock;
    idx[k] = insert_zeros(j, sp) | cmask | half;
    a[k] = CV<R>{0, 0};
    if (j < npairs) a[k] = ld<NT>(psi + idx[k]);
  }
#pragma unroll
  for (int k = 0; k < ITEMS; ++k) {
    // both halves of a pair share j, so a lane and its partner are in or out
    // of range together; the exchange itself runs on every lane
    const R bx = __shfl_xor(a[k].x, 32, 64);
    const R by = __shfl_xor(a[k].y, 32, 64);
    CV<R> r;
    r.x = sr * a[k].x - si * a[k].y + orr * bx - oi * by;
    r.y = sr * a[k].y + si * a[k].x + orr * by + oi * bx;
    const uint64_t j = j0 + (uint64_t)k * kPairsPerBlock;
    // controls on low bits are a predicate: pairs outside the controlled
    // subspace are written back unchanged, so every line is written whole
    const bool act = (idx[k] & pmask) == pmask;
    if (j < npairs) st<NT>(psi + idx[k], act ? r : a[k]);
  }
}

// k_butterfly_lane: target bit t < 6.  Lane l of a wave holds amplitude
// 64 s + l of segment s, so every load and store is one fully coalesced,
// contiguous run; the pair partner (lane l ^ 2^t) arrives by a cross-lane
// exchange.  Controls at bits >= 6 select the segments; controls below 6
// become a per-lane predicate on the store.

template <typename R, int ITEMS, bool NT>
__global__ __launch_bounds__(kBlock) void k_butterfly_lane(CV<R>* __restrict__ psi, uint64_t nseg, Special sp,
                                                           uint64_t cmask_hi, uint32_t cmask_lo, uint32_t cmask_fine,
                                                           int t, Mat2 u, CondArgs cond, bool xcd) {
  if (!conds_ok(cond)) return;
  const int lane = threadIdx.x & 63;
  const uint64_t s0 = (sweep_block(xcd) * (kBlock / 64) + (threadIdx.x >> 6)) * ITEMS;
  if (s0 >= nseg) return;   // uniform per wave
  const bool up = (lane >> t) & 1;
  // Controls below 6 are per-lane predicates.  `touch`: the lane's
  // amplitude is read and written at all; it fails only on controls whose
  // runs are a 64-byte sector or more, so untouched lanes leave whole sectors
  // alone.  Controls with shorter runs (cmask_fine) would leave sectors
  // partly written, which costs more than writing them whole: there the lane
  // is touched and writes its own value back.
  const uint32_t coarse = cmask_lo & ~cmask_fine;
  const bool touch = ((uint32_t)lane & coarse) == coarse;
  const bool act = ((uint32_t)lane & cmask_lo) == cmask_lo;
  // lower lane: u00 a + u01 b; upper lane: u11 a + u10 b (b = partner)
  const R sr = (R)(up ? u.v[6] : u.v[0]), si = (R)(up ? u.v[7] : u.v[1]);
  const R orr = (R)(up ? u.v[4] : u.v[2]), oi = (R)(up ? u.v[5] : u.v[3]);
  const int mask = 1 << t;
  CV<R> a[ITEMS];
  uint64_t addr[ITEMS];
#pragma unroll
  for (int k = 0; k < ITEMS; ++k) {
    addr[k] = ((insert_zeros(s0 + k, sp) << 6) | cmask_hi) + (uint64_t)lane;
    // a lane and its partner share the control bits, so the exchange below
    // only ever reads loaded values into lanes that act
    a[k] = CV<R>{0, 0};
    if (touch) a[k] = ld<NT>(psi + addr[k]);
  }
#pragma unroll
  for (int k = 0; k < ITEMS; ++k) {
    const R bx = __shfl_xor(a[k].x, mask, 64);
    const R by = __shfl_xor(a[k].y, mask, 64);
    CV<R> r;
    r.x = sr * a[k].x - si * a[k].y + orr * bx - oi * by;
    r.y = sr * a[k].y + si * a[k].x + orr * by + oi * bx;
    if (touch) st<NT>(psi + addr[k], act ? r : a[k]);
  }
}

template <typename R, int IT, bool NT, bool CTRL>
static void launch_bfly_generic(const Launch& L, uint64_t npairs, const Special& sp, uint64_t cmask, uint64_t pmask,
                                uint64_t tbit, const Mat2& u) {
  const dim3 g = grid_for(npairs, kPairsPerBlock * IT);
  hipLaunchKernelGGL((k_butterfly<R, IT, NT, CTRL>), g, dim3(kBlock), 0, L.stream, (CV<R>*)L.psi, npairs, sp,
                     cmask, pmask, tbit, u, L.cond, L.tune.xcd != 0);
}

template <typename R, bool NT, bool CTRL>
static void launch_bfly_items(const Launch& L, uint64_t npairs, const Special& sp, uint64_t cmask, uint64_t pmask,
                              uint64_t tbit, const Mat2& u) {
  switch (L.tune.sweep_items) {
    case 2: launch_bfly_generic<R, 2, NT, CTRL>(L, npairs, sp, cmask, pmask, tbit, u); break;
    case 4: launch_bfly_generic<R, 4, NT, CTRL>(L, npairs, sp, cmask, pmask, tbit, u); break;
    default: launch_bfly_generic<R, 1, NT, CTRL>(L, npairs, sp, cmask, pmask, tbit, u); break;
  }
}

template <typename R, int IT, bool NT>
static void launch_lane(const Launch& L, uint64_t nseg, const Special& sp, uint64_t cmask_hi, uint32_t cmask_lo, int t,
                        const Mat2& u) {
  const dim3 g = grid_for(nseg / IT, kBlock / 64);
  // controls whose runs are shorter than a 64-byte sector: bits 0-1 of
  // complex128 amplitudes, 0-2 of complex64
  const uint32_t fine = cmask_lo & (L.c64 ? 7u : 3u);
  hipLaunchKernelGGL((k_butterfly_lane<R, IT, NT>), g, dim3(kBlock), 0, L.stream, (CV<R>*)L.psi, nseg, sp,
                     cmask_hi, cmask_lo, fine, t, u, L.cond, L.tune.xcd != 0);
}

template <typename R>
static void launch_bfly_typed(const Launch& L, int t, const int* controls, int nc, const Mat2& u) {
  if (L.tune.lane_bfly && t < 6 && L.n >= 6) {
    std::vector<int> hi;
    uint64_t cmask_hi = 0;
    uint32_t cmask_lo = 0;
    for (int i = 0; i < nc; ++i) {
      if (controls[i] >= 6) {
        hi.push_back(controls[i] - 6);
        cmask_hi |= 1ull << controls[i];
      } else {
        cmask_lo |= 1u << controls[i];
      }
    }
    Special sp = make_special(hi.data(), (int)hi.size(), nullptr, 0);
    const uint64_t nseg = 1ull << (L.n - 6 - (int)hi.size());
    const bool nt = L.tune.nt == 2 || (L.tune.nt == 1 && state_streams(L));
    const int it = (int)std::min<uint64_t>((uint64_t)L.tune.lane_items, nseg);
    if (it >= 4) { if (nt) launch_lane<R, 4, true>(L, nseg, sp, cmask_hi, cmask_lo, t, u); else launch_lane<R, 4, false>(L, nseg, sp, cmask_hi, cmask_lo, t, u); }
    else if (it == 2) { if (nt) launch_lane<R, 2, true>(L, nseg, sp, cmask_hi, cmask_lo, t, u); else launch_lane<R, 2, false>(L, nseg, sp, cmask_hi, cmask_lo, t, u); }
    else { if (nt) launch_lane<R, 1, true>(L, nseg, sp, cmask_hi, cmask_lo, t, u); else launch_lane<R, 1, false>(L, nseg, sp, cmask_hi, cmask_lo, t, u); }
    return;
  }
  // controls below the whole-line threshold become a predicate (when sweeps are non-temporal)
  // Controls below the bit whose runs are one 128-byte line (bit 3 for
  // complex128, 4 for complex64) become a predicate of a full sweep: skipping
  // their complement would leave lines half written.  From that bit up they
  // are skipped in the enumeration, whole lines at a time.
  const int thr = L.c64 ? 5 : 4;
  const int pthr = L.c64 ? 4 : 3;
  std::vector<int> en;
  uint64_t pmask = 0;
  for (int i = 0; i < nc; ++i) {
    if (L.tune.nt != 0 && controls[i] < pthr && t >= thr) pmask |= 1ull << controls[i];
    else en.push_back(controls[i]);
  }
  const int ne = (int)en.size();
  Special sp = make_special(&t, 1, en.data(), ne);
  const uint64_t npairs = 1ull << (L.n - 1 - ne);
  const uint64_t cmask = mask_of(en.data(), ne), tbit = 1ull << t;
  const bool nt = use_nt(L, lowest(&t, 1, en.data(), ne, 64));
  if (nc == 0) {
    if (nt) launch_bfly_items<R, true, false>(L, npairs, sp, cmask, pmask, tbit, u);
    else launch_bfly_items<R, false, false>(L, npairs, sp, cmask, pmask, tbit, u);
  } else {
    if (nt) launch_bfly_items<R, true, true>(L, npairs, sp, cmask, pmask, tbit, u);
    else launch_bfly_items<R, false, true>(L, npairs, sp, cmask, pmask, tbit, u);
  }
}

hipError_t launch_butterfly(const Launch& L, int t, const int* controls, int nc, const Mat2& u) {
  if (L.c64) launch_bfly_typed<float>(L, t, controls, nc, u);
  else launch_bfly_typed<double>(L, t, controls, nc, u);
  return hipGetLastError();
}

// ---------------------------------------------------------------- diagonal
// a_i <- d[m(i)] a_i with m(i) the bits of i on the targets, over the subspace
// where every control bit is 1.

struct Pos8 {
  int p[8];
};

template <typename R, int ITEMS, bool NT>
__global__ __launch_bounds__(kBlock) void k_diag(CV<R>* __restrict__ psi, uint64_t nitems, Special sp, uint64_t cmask,
                                                 int k, Pos8 tp, Diag64 d, CondArgs cond, bool xcd) {
  if (!conds_ok(cond)) return;
  const uint64_t j0 = sweep_block(xcd) * (kBlock * ITEMS) + threadIdx.x;
  CV<R> x[ITEMS];
  uint64_t idx[ITEMS];
#pragma unroll
  for (int it = 0; it < ITEMS; ++it) {
    const uint64_t j = j0 + (uint64_t)it * kBlock;
    idx[it] = insert_zeros(j, sp) | cmask;
    if (j < nitems) x[it] = ld<NT>(psi + idx[it]);
  }
  if (k <= 2) {
    // at most four factors: kept in registers and picked by selects, so no
    // amplitude waits on a per-lane load of its factor
    const R d0r = (R)d.v[0], d0i = (R)d.v[1], d1r = (R)d.v[2], d1i = (R)d.v[3];
    const R d2r = (R)d.v[4], d2i = (R)d.v[5], d3r = (R)d.v[6], d3i = (R)d.v[7];
    const int p0 = tp.p[0], p1 = k > 1 ? tp.p[1] : 63;   // bit 63 of an index is 0
#pragma unroll
    for (int it = 0; it < ITEMS; ++it) {
      const uint64_t j = j0 + (uint64_t)it * kBlock;
      if (j < nitems) {
        const bool b0 = (idx[it] >> p0) & 1ull, b1 = (idx[it] >> p1) & 1ull;
        const R dr = b1 ? (b0 ? d3r : d2r) : (b0 ? d1r : d0r);
        const R di = b1 ? (b0 ? d3i : d2i) : (b0 ? d1i : d0i);
        const CV<R> p = x[it];
        CV<R> r;
        r.x = dr * p.x - di * p.y;
        r.y = dr * p.y + di * p.x;
        st<NT>(psi + idx[it], r);
      }
    }
    return;
  }
#pragma unroll
  for (int it = 0; it < ITEMS; ++it) {
    const uint64_t j = j0 + (uint64_t)it * kBlock;
    if (j < nitems) {
      const int m = (int)extract(idx[it], tp.p, k);
      const R dr = (R)d.v[2 * m], di = (R)d.v[2 * m + 1];
      const CV<R> p = x[it];
      CV<R> r;
      r.x = dr * p.x - di * p.y;
      r.y = dr * p.y + di * p.x;
      st<NT>(psi + idx[it], r);
    }
  }
}

template <typename R, bool NT>
static void launch_diag_items(const Launch& L, unsigned items, uint64_t nitems, const Special& sp, uint64_t cmask,
                              int k, const Pos8& tp, const Diag64& d) {
  switch (items) {
    case 2: hipLaunchKernelGGL((k_diag<R, 2, NT>), grid_for(nitems, kBlock * 2), dim3(kBlock), 0, L.stream,
                               (CV<R>*)L.psi, nitems, sp, cmask, k, tp, d, L.cond, L.tune.xcd != 0); break;
    case 4: hipLaunchKernelGGL((k_diag<R, 4, NT>), grid_for(nitems, kBlock * 4), dim3(kBlock), 0, L.stream,
                               (CV<R>*)L.psi, nitems, sp, cmask, k, tp, d, L.cond, L.tune.xcd != 0); break;
    default: hipLaunchKernelGGL((k_diag<R, 1, NT>), grid_for(nitems, kBlock), dim3(kBlock), 0, L.stream,
                                (CV<R>*)L.psi, nitems, sp, cmask, k, tp, d, L.cond, L.tune.xcd != 0); break;
  }
}

hipError_t launch_diag(const Launch& L, const int* targets, int k, const int* controls, int nc, const Diag64& d_in) {
  if (k > 6) return hipErrorInvalidValue;
  // Controls whose runs are shorter than a 128-byte line (below bit 3 for
  // complex128, 4 for complex64) join the diagonal (entry 1 where such a
  // control is 0), so the sweep covers whole lines; from that bit up they are
  // skipped in the enumeration, whole lines at a time.
  const int thr = L.c64 ? 4 : 3;
  std::vector<int> tg(targets, targets + k), en, low;
  for (int i = 0; i < nc; ++i) {
    if (L.tune.nt != 0 && controls[i] < thr && k + (int)low.size() < 6) low.push_back(controls[i]);
    else en.push_back(controls[i]);
  }
  Diag64 d = d_in;
  if (!low.empty()) {
    const int kk = k + (int)low.size();
    const int lowall = (1 << low.size()) - 1;
    for (int m = 0; m < (1 << kk); ++m) {
      const int mt = m & ((1 << k) - 1), ml = m >> k;
      d.v[2 * m] = ml == lowall ? d_in.v[2 * mt] : 1.0;
      d.v[2 * m + 1] = ml == lowall ? d_in.v[2 * mt + 1] : 0.0;
    }
    for (int c : low) tg.push_back(c);
  }
  const int kk = (int)tg.size(), ne = (int)en.size();
  Special sp = make_special(en.data(), ne, nullptr, 0);
  const uint64_t nitems = 1ull << (L.n - ne);
  Pos8 tp{};
  for (int j = 0; j < kk; ++j) tp.p[j] = tg[j];
  const uint64_t cmask = mask_of(en.data(), ne);
  const bool nt = use_nt(L, lowest(en.data(), ne, nullptr, 0, 64));
  const unsigned items = (unsigned)L.tune.diag_items;
  if (L.c64) { if (nt) launch_diag_items<float, true>(L, items, nitems, sp, cmask, kk, tp, d); else launch_diag_items<float, false>(L, items, nitems, sp, cmask, kk, tp, d); }
  else { if (nt) launch_diag_items<double, true>(L, items, nitems, sp, cmask, kk, tp, d); else launch_diag_items<double, false>(L, items, nitems, sp, cmask, kk, tp, d); }
  return hipGetLastError();
}

// ---------------------------------------------------------------- phase on the all-ones subspace
// a_i <- z a_i where every bit of `bits` is 1 (PHASE, CPHASE, S, T, Z and
// their controlled forms touch only this 2^(n - |bits|) subspace).

template <typename R, int ITEMS, bool NT>
__global__ __launch_bounds__(kBlock) void k_phase_all1(CV<R>* __restrict__ psi, uint64_t nitems, Special sp,
                                                       uint64_t mask, double zr_, double zi_, CondArgs cond,
                                                       bool xcd) {
  if (!conds_ok(cond)) return;
  const R zr = (R)zr_, zi = (R)zi_;
  const uint64_t j0 = sweep_block(xcd) * (kBlock * ITEMS) + threadIdx.x;
  CV<R> x[ITEMS];
  uint64_t idx[ITEMS];
#pragma unroll
  for (int it = 0; it < ITEMS; ++it) {
    const uint64_t j = j0 + (uint64_t)it * kBlock;
    idx[it] = insert_zeros(j, sp) | mask;
    if (j < nitems) x[it] = ld<NT>(psi + idx[it]);
  }
#pragma unroll
  for (int it = 0; it < ITEMS; ++it) {
    const uint64_t j = j0 + (uint64_t)it * kBlock;
    if (j < nitems) {
      const CV<R> p = x[it];
      CV<R> r;
      r.x = zr * p.x - zi * p.y;
      r.y = zr * p.y + zi * p.x;
      st<NT>(psi + idx[it], r);
    }
  }
}

hipError_t launch_phase_all1(const Launch& L, const int* bits, int nb, double zr, double zi) {
  Special sp = make_special(bits, nb, nullptr, 0);
  const uint64_t nitems = 1ull << (L.n - nb);
  const uint64_t mask = mask_of(bits, nb);
  const bool nt = use_nt(L, lowest(bits, nb, nullptr, 0, 64));
  const int it = L.tune.diag_items;
#define QK_PH(R, IT, NT)                                                                                             \
  hipLaunchKernelGGL((k_phase_all1<R, IT, NT>), grid_for(nitems, kBlock * IT), dim3(kBlock), 0, L.stream,   \
                     (CV<R>*)L.psi, nitems, sp, mask, zr, zi, L.cond, L.tune.xcd != 0)
#define QK_PH_IT(R, NT) \
  do { if (it == 2) QK_PH(R, 2, NT); else if (it == 4) QK_PH(R, 4, NT); else QK_PH(R, 1, NT); } while (0)
  if (L.c64) { if (nt) QK_PH_IT(float, true); else QK_PH_IT(float, false); }
  else { if (nt) QK_PH_IT(double, true); else QK_PH_IT(double, false); }
#undef QK_PH_IT
#undef QK_PH
  return hipGetLastError();
}

// ---------------------------------------------------------------- diagonal runs
// Several diagonal gates in one pass, in two launches.  k_diag_run_tables
// (one workgroup) finds which terms are active (lane c of a wave reads
// condition c, a ballot gathers the failures) and tabulates every group's
// combined factor over the group's bits (FP64 products, rounded once to the
// state's precision) into a small device table, with a word that says whether
// any term is active.  k_diag_run then sweeps the subspace like the other
// diagonal sweeps, each workgroup with its own LDS copy of the tables:
// a_i <- a_i * prod_g tab_g[bits of i on group g].

template <typename R>
__global__ __launch_bounds__(512) void k_diag_run_tables(CV<R>* __restrict__ tab, uint32_t* __restrict__ any,
                                                         DiagRunArgs run) {
  constexpr int TW = 1 << kDiagRunGroupBits;
  const int lane = threadIdx.x & 63;
  bool bad = false;
  if (lane < run.ncond) bad = run.cbits[run.cb[lane]] != run.cv[lane];
  const uint64_t fail = __ballot(bad);
  uint32_t active = 0;
  for (int t = 0; t < run.n; ++t) {
    const uint64_t cm = ((1ull << run.t[t].c1) - 1) & ~((1ull << run.t[t].c0) - 1);
    if (!(fail & cm)) active |= 1u << t;
  }
  if (threadIdx.x == 0) *any = active;
  for (int e = threadIdx.x; e < run.ng * TW; e += blockDim.x) {
    const int g = e / TW, m = e % TW;
    double fr = 1, fi = 0;
    for (int t = 0; t < run.n; ++t) {
      const DiagRunTerm& T = run.t[t];
      if (T.g != g || !((active >> t) & 1u) || (m & T.lmask) != T.lmask) continue;
      // entries picked by selects, not by an index (no scratch copy of the terms)
      const bool b0 = T.k > 0 && ((m >> T.l0) & 1), b1 = T.k > 1 && ((m >> T.l1) & 1);
      const double dr = b1 ? (b0 ? T.d[6] : T.d[4]) : (b0 ? T.d[2] : T.d[0]);
      const double di = b1 ? (b0 ? T.d[7] : T.d[5]) : (b0 ? T.d[3] : T.d[1]);
      const double nr = fr * dr - fi * di;
      fi = fr * di + fi * dr;
      fr = nr;
    }
    CV<R> v;
    v.x = (R)fr;
    v.y = (R)fi;
    tab[e] = v;
  }
}

constexpr int kDiagRunItems = 4;   // amplitudes per thread of the run sweep

struct DiagRunGroups {
  int ng;
  DiagRunGroup grp[kDiagRunGroups];
  uint8_t item[kDiagRunGroups][kDiagRunItems];   // table-index bits contributed by the item offset
};

// Table index of a group for amplitude index (lo, hi words): bit b of the
// index is bit pos[b] of the amplitude index.  The host pads unused positions
// with bit 63, which is 0 in every amplitude index, so the loop has a fixed
// trip count and compiles to one bit-field extract and one shift-or per bit.
__device__ __forceinline__ uint32_t group_index(uint32_t lo, uint32_t hi, const DiagRunGroup& gr) {
  uint32_t m = 0;
#pragma unroll
  for (int b = 0; b < kDiagRunGroupBits; ++b) {
    const int p = gr.pos[b];
    m |= (((p < 32 ? lo : hi) >> (p & 31)) & 1u) << b;
  }
  return m;
}

// The same on the host, for the item offsets.
static uint32_t group_index_host(uint64_t x, const DiagRunGroup& gr) {
  uint32_t m = 0;
  for (int b = 0; b < gr.nb; ++b) m |= (uint32_t)((x >> gr.pos[b]) & 1ull) << b;
  return m;
}

static uint64_t insert_zeros_host(uint64_t x, const Special& s) {
  for (int i = 0; i < s.n; ++i) {
    const int p = s.pos[i];
    x = ((x >> p) << (p + 1)) | (x & ((1ull << p) - 1));
  }
  return x;
}

template <typename R, int ITEMS, bool NT, int NG>
__global__ __launch_bounds__(kBlock) void k_diag_run(CV<R>* __restrict__ psi, uint64_t nitems, Special sp,
                                                     uint64_t common, const CV<R>* __restrict__ gtab,
                                                     const uint32_t* __restrict__ any, DiagRunGroups gs, bool xcd) {
  constexpr int TW = 1 << kDiagRunGroupBits;
  constexpr int CH = kBlock * ITEMS;   // amplitudes per workgroup (a power of two)
  __shared__ CV<R> tab[kDiagRunGroups * TW];
  if (*any == 0) return;               // every term's conditions failed
  for (int e = threadIdx.x; e < NG * TW; e += kBlock) tab[e] = gtab[e];
  __syncthreads();
  // The counter j of an amplitude splits into disjoint bit fields: the
  // workgroup base plus thread id, and the item offset (it * kBlock); zero
  // insertion maps each field onto its own index bits.  So a group's table
  // index is the OR of a per-thread part and a per-item part, the latter
  // computed on the host.
  const uint64_t base = sweep_block(xcd) * CH;
  const uint64_t i0 = insert_zeros(base + threadIdx.x, sp) | common;
  const uint32_t lo = (uint32_t)i0, hi = (uint32_t)(i0 >> 32);
  uint32_t mt[NG];
#pragma unroll
  for (int g = 0; g < NG; ++g) mt[g] = group_index(lo, hi, gs.grp[g]);
  CV<R> x[ITEMS];
  uint64_t idx[ITEMS];
#pragma unroll
  for (int it = 0; it < ITEMS; ++it) {
    const uint64_t j = base + (uint64_t)it * kBlock + threadIdx.x;
    idx[it] = insert_zeros(j, sp) | common;
    if (j < nitems) x[it] = ld<NT>(psi + idx[it]);
  }
#pragma unroll
  for (int it = 0; it < ITEMS; ++it) {
    const uint64_t j = base + (uint64_t)it * kBlock + threadIdx.x;
    if (j < nitems) {
      R fr = 1, fi = 0;
#pragma unroll
      for (int g = 0; g < NG; ++g) {
        const CV<R> f = tab[g * TW + (mt[g] | gs.item[g][it])];
        const R nr = fr * f.x - fi * f.y;
        fi = fr * f.y + fi * f.x;
        fr = nr;
      }
      const CV<R> p = x[it];
      CV<R> r;
      r.x = fr * p.x - fi * p.y;
      r.y = fr * p.y + fi * p.x;
      st<NT>(psi + idx[it], r);
    }
  }
}

hipError_t launch_diag_run(const Launch& L, const DiagRunArgs& run, const int* common, int nc, void* table) {
  if (run.n < 1 || run.n > kDiagRunTerms || run.ng < 1 || run.ng > kDiagRunGroups || run.ncond > kDiagRunConds)
    return hipErrorInvalidValue;
  Special sp = make_special(common, nc, nullptr, 0);
  const uint64_t nitems = 1ull << (L.n - nc);
  const uint64_t cm = mask_of(common, nc);
  const bool nt = use_nt(L, lowest(common, nc, nullptr, 0, 64));
  DiagRunGroups gs{};
  gs.ng = run.ng;
  for (int g = 0; g < run.ng; ++g) {
    gs.grp[g] = run.grp[g];
    for (int b = run.grp[g].nb; b < kDiagRunGroupBits; ++b) gs.grp[g].pos[b] = 63;
    for (int it = 0; it < kDiagRunItems; ++it)
      gs.item[g][it] = (uint8_t)group_index_host(insert_zeros_host((uint64_t)it * kBlock, sp), run.grp[g]);
  }
  uint32_t* any = (uint32_t*)((char*)table + kDiagRunTableBytes - 16);
  // four amplitudes per thread: the workgroup's copy of the tables into LDS
  // (at most 8 KiB, from L2) is shared by 1024 amplitudes
  const dim3 grid = grid_for(nitems, kBlock * kDiagRunItems);
  auto sweep = [&](auto tag_r, auto tag_nt, auto tag_ng) {
    using R = decltype(tag_r);
    constexpr bool NT = decltype(tag_nt)::value;
    constexpr int NG = decltype(tag_ng)::value;
    hipLaunchKernelGGL((k_diag_run<R, kDiagRunItems, NT, NG>), grid, dim3(kBlock), 0, L.stream, (CV<R>*)L.psi,
                       nitems, sp, cm, (const CV<R>*)table, any, gs, L.tune.xcd != 0);
  };
  auto by_groups = [&](auto tag_r, auto tag_nt) {
    switch (run.ng) {
      case 1: sweep(tag_r, tag_nt, std::integral_constant<int, 1>{}); break;
      case 2: sweep(tag_r, tag_nt, std::integral_constant<int, 2>{}); break;
      case 3: sweep(tag_r, tag_nt, std::integral_constant<int, 3>{}); break;
      case 4: sweep(tag_r, tag_nt, std::integral_constant<int, 4>{}); break;
      case 5: sweep(tag_r, tag_nt, std::integral_constant<int, 5>{}); break;
      case 6: sweep(tag_r, tag_nt, std::integral_constant<int, 6>{}); break;
      case 7: sweep(tag_r, tag_nt, std::integral_constant<int, 7>{}); break;
      default: sweep(tag_r, tag_nt, std::integral_constant<int, 8>{}); break;
    }
  };
  if (L.c64) {
    hipLaunchKernelGGL(k_diag_run_tables<float>, dim3(1), dim3(512), 0, L.stream, (CV<float>*)table, any, run);
    if (nt) by_groups(float{}, std::true_type{}); else by_groups(float{}, std::false_type{});
  } else {
    hipLaunchKernelGGL(k_diag_run_tables<double>, dim3(1), dim3(512), 0, L.stream, (CV<double>*)table, any, run);
    if (nt) by_groups(double{}, std::true_type{}); else by_groups(double{}, std::false_type{});
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------- swap
// Exchanges a_{base|2^a} and a_{base|2^b} for every base with both bits 0 and
// all control bits 1 (touches 2^(n-1-c) amplitudes).

template <typename R, int ITEMS, bool NT>
__global__ __launch_bounds__(kBlock) void k_swap(CV<R>* __restrict__ psi, uint64_t nitems, Special sp, uint64_t cmask,
                                                 uint64_t abit, uint64_t bbit, CondArgs cond, bool xcd) {
  if (!conds_ok(cond)) return;
  const uint64_t j0 = sweep_block(xcd) * (kBlock * ITEMS) + threadIdx.x;
  CV<R> x[ITEMS], y[ITEMS];
  uint64_t idx[ITEMS];
#pragma unroll
  for (int it = 0; it < ITEMS; ++it) {
    const uint64_t j = j0 + (uint64_t)it * kBlock;
    idx[it] = insert_zeros(j, sp) | cmask;
    if (j < nitems) {
      x[it] = ld<NT>(psi + (idx[it] | abit));
      y[it] = ld<NT>(psi + (idx[it] | bbit));
    }
  }
#pragma unroll
  for (int it = 0; it < ITEMS; ++it) {
    const uint64_t j = j0 + (uint64_t)it * kBlock;
    if (j < nitems) {
      st<NT>(psi + (idx[it] | abit), y[it]);
      st<NT>(psi + (idx[it] | bbit), x[it]);
    }
  }
}

// Uncontrolled swap with a low bit a (runs of 2^a amplitudes shorter than a
// 128-byte line): the touched half of the state would be scattered pieces of
// lines, so instead every amplitude is read and written once, whole lines at
// a time, and the partners meet by a cross-lane exchange.
// k_swap_lane_hi (b >= 6): lane l of a wave holds x = a_i and y = a_{i | 2^b}
// for i = 64 s + l in the half where bit b is 0; the amplitude for (bit a, bit
// b) = (1, 0) comes from the partner's y, the one for (0, 1) from its x.
template <typename R, bool NT>
__global__ __launch_bounds__(kBlock) void k_swap_lane_hi(CV<R>* __restrict__ psi, uint64_t nseg, Special sp, int a,
                                                         uint64_t bbit, CondArgs cond, bool xcd) {
  if (!conds_ok(cond)) return;
  const int lane = threadIdx.x & 63;
  const uint64_t s0 = sweep_block(xcd) * (kBlock / 64) + (threadIdx.x >> 6);
  if (s0 >= nseg) return;   // uniform per wave
  const uint64_t i = (insert_zeros(s0, sp) << 6) + (uint64_t)lane;
  const CV<R> x = ld<NT>(psi + i), y = ld<NT>(psi + (i | bbit));
  const int m = 1 << a;
  CV<R> px, py;
  px.x = __shfl_xor(x.x, m, 64);
  px.y = __shfl_xor(x.y, m, 64);
  py.x = __shfl_xor(y.x, m, 64);
  py.y = __shfl_xor(y.y, m, 64);
  const bool one = (lane >> a) & 1;
  st<NT>(psi + i, one ? py : x);
  st<NT>(psi + (i | bbit), one ? y : px);
}

// k_swap_lane_lo (a < b < 6): every amplitude of a 64-amplitude segment comes
// from the lane with bits a and b exchanged.
template <typename R, bool NT>
__global__ __launch_bounds__(kBlock) void k_swap_lane_lo(CV<R>* __restrict__ psi, uint64_t nseg, int a, int b,
                                                         CondArgs cond, bool xcd) {
  if (!conds_ok(cond)) return;
  const int lane = threadIdx.x & 63;
  const uint64_t s0 = sweep_block(xcd) * (kBlock / 64) + (threadIdx.x >> 6);
  if (s0 >= nseg) return;   // uniform per wave
  const uint64_t i = (s0 << 6) + (uint64_t)lane;
  const CV<R> x = ld<NT>(psi + i);
  const int ba = (lane >> a) & 1, bb = (lane >> b) & 1;
  const int src = ba == bb ? lane : lane ^ ((1 << a) | (1 << b));
  CV<R> v;
  v.x = __shfl(x.x, src, 64);
  v.y = __shfl(x.y, src, 64);
  st<NT>(psi + i, v);
}

hipError_t launch_swap(const Launch& L, int a, int b, const int* controls, int nc) {
  if (a > b) std::swap(a, b);
  if (nc == 0 && L.n >= 6 && a < (L.c64 ? 4 : 3)) {
    const bool nt = L.tune.nt == 2 || (L.tune.nt == 1 && state_streams(L));
    if (b >= 6) {
      const int hb = b - 6;
      Special sp = make_special(&hb, 1, nullptr, 0);
      const uint64_t nseg = 1ull << (L.n - 7);
      const dim3 g = grid_for(nseg, kBlock / 64);
      if (L.c64) {
        if (nt) hipLaunchKernelGGL((k_swap_lane_hi<float, true>), g, dim3(kBlock), 0, L.stream, (CV<float>*)L.psi, nseg, sp, a, 1ull << b, L.cond, L.tune.xcd != 0);
        else hipLaunchKernelGGL((k_swap_lane_hi<float, false>), g, dim3(kBlock), 0, L.stream, (CV<float>*)L.psi, nseg, sp, a, 1ull << b, L.cond, L.tune.xcd != 0);
      } else {
        if (nt) hipLaunchKernelGGL((k_swap_lane_hi<double, true>), g, dim3(kBlock), 0, L.stream, (CV<double>*)L.psi, nseg, sp, a, 1ull << b, L.cond, L.tune.xcd != 0);
        else hipLaunchKernelGGL((k_swap_lane_hi<double, false>), g, dim3(kBlock), 0, L.stream, (CV<double>*)L.psi, nseg, sp, a, 1ull << b, L.cond, L.tune.xcd != 0);
      }
    } else {
      const uint64_t nseg = 1ull << (L.n - 6);
      const dim3 g = grid_for(nseg, kBlock / 64);
      if (L.c64) {
        if (nt) hipLaunchKernelGGL((k_swap_lane_lo<float, true>), g, dim3(kBlock), 0, L.stream, (CV<float>*)L.psi, nseg, a, b, L.cond, L.tune.xcd != 0);
        else hipLaunchKernelGGL((k_swap_lane_lo<float, false>), g, dim3(kBlock), 0, L.stream, (CV<float>*)L.psi, nseg, a, b, L.cond, L.tune.xcd != 0);
      } else {
        if (nt) hipLaunchKernelGGL((k_swap_lane_lo<double, true>), g, dim3(kBlock), 0, L.stream, (CV<double>*)L.psi, nseg, a, b, L.cond, L.tune.xcd != 0);
        else hipLaunchKernelGGL((k_swap_lane_lo<double, false>), g, dim3(kBlock), 0, L.stream, (CV<double>*)L.psi, nseg, a, b, L.cond, L.tune.xcd != 0);
      }
    }
    return hipGetLastError();
  }
  int ab[2] = {a, b};
  Special sp = make_special(ab, 2, controls, nc);
  const uint64_t nitems = 1ull << (L.n - 2 - nc);
  const uint64_t cmask = mask_of(controls, nc);
  const bool nt = use_nt(L, lowest(ab, 2, controls, nc, 64));
  const int it = L.tune.sweep_items;
#define QK_SW(R, IT, NT)                                                                                           \
  hipLaunchKernelGGL((k_swap<R, IT, NT>), grid_for(nitems, kBlock * IT), dim3(kBlock), 0, L.stream,       \
                     (CV<R>*)L.psi, nitems, sp, cmask, 1ull << a, 1ull << b, L.cond, L.tune.xcd != 0)
#define QK_SW_IT(R, NT) \
  do { if (it == 2) QK_SW(R, 2, NT); else if (it == 4) QK_SW(R, 4, NT); else QK_SW(R, 1, NT); } while (0)
  if (L.c64) { if (nt) QK_SW_IT(float, true); else QK_SW_IT(float, false); }
  else { if (nt) QK_SW_IT(double, true); else QK_SW_IT(double, false); }
#undef QK_SW_IT
#undef QK_SW
  return hipGetLastError();
}

// ---------------------------------------------------------------- dense k-target (vector ALU)
// Each block stages G groups of 2^k amplitudes in LDS (G = max(1, 256 / 2^k)),
// then every thread writes rows r of M v for its groups.  Used for k > 6, for
// states too small for the matrix-core tile, and as the general fallback.

template <typename R>
__global__ __launch_bounds__(kBlock) void k_dense_generic(V2<R>* __restrict__ psi, const V2<R>* __restrict__ mat,
                                                          int k, uint64_t ngroups, Special sp, uint64_t cmask, Pos32 tp,
                                                          CondArgs cond) {
  if (!conds_ok(cond)) return;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  V2<R>* buf = reinterpret_cast<V2<R>*>(smem_raw);
  const int dimK = 1 << k;
  const int G = dimK >= kBlock ? 1 : kBlock / dimK;
  const uint64_t g0 = flat_block() * G;
  for (int e = threadIdx.x; e < G * dimK; e += kBlock) {
    const uint64_t gid = g0 + (uint64_t)(e >> k);
    if (gid < ngroups) {
      const uint64_t base = insert_zeros(gid, sp) | cmask;
      buf[e] = psi[base | deposit((uint64_t)(e & (dimK - 1)), tp.p, k)];
    }
  }
  __syncthreads();
  for (int e = threadIdx.x; e < G * dimK; e += kBlock) {
    const int g = e >> k, r = e & (dimK - 1);
    const uint64_t gid = g0 + (uint64_t)g;
    if (gid >= ngroups) continue;
    const V2<R>* row = mat + (size_t)r * dimK;
    const V2<R>* v = buf + (size_t)g * dimK;
    R sr = 0, si = 0;
    for (int m = 0; m < dimK; ++m) {
      const V2<R> a = row[m], b = v[m];
      sr += a.x * b.x - a.y * b.y;
      si += a.x * b.y + a.y * b.x;
    }
    const uint64_t base = insert_zeros(gid, sp) | cmask;
    psi[base | deposit((uint64_t)r, tp.p, k)] = V2<R>{sr, si};
  }
}

hipError_t launch_dense_generic(const Launch& L, const int* targets, int k, const int* controls, int nc,
                                const void* d_matrix) {
  if (k < 1 || k > QK_MAX_MATRIX_K) return hipErrorInvalidValue;
  Special sp = make_special(targets, k, controls, nc);
  const uint64_t ngroups = 1ull << (L.n - k - nc);
  Pos32 tp{};
  for (int j = 0; j < k; ++j) tp.p[j] = targets[j];
  const int dimK = 1 << k;
  const int G = dimK >= kBlock ? 1 : kBlock / dimK;
  const dim3 g = grid_for(ngroups, G);
  const uint64_t cmask = mask_of(controls, nc);
  const size_t shm = (size_t)G * dimK * (L.c64 ? sizeof(float2) : sizeof(double2));
  if (L.c64)
    hipLaunchKernelGGL(k_dense_generic<float>, g, dim3(kBlock), shm, L.stream, (float2*)L.psi,
                       (const float2*)d_matrix, k, ngroups, sp, cmask, tp, L.cond);
  else
    hipLaunchKernelGGL(k_dense_generic<double>, g, dim3(kBlock), shm, L.stream, (double2*)L.psi,
                       (const double2*)d_matrix, k, ngroups, sp, cmask, tp, L.cond);
  return hipGetLastError();
}

// ---------------------------------------------------------------- permutation (oracle) gate
// U|x> = |f(x)> on the targets: the amplitude at gate index x moves to f(x).
// Done as a gather out[y] = in[f^-1(y)] (coalesced writes, gathered reads).
// Without controls the gather writes the whole permuted state into the second
// state buffer, which then becomes the state (one read and one write of every
// amplitude); when its classical condition fails it copies the state instead,
// so the second buffer always holds the result.  With controls it gathers the
// controlled subspace into a compact scratch buffer and copies that back.
// f^-1 is a device table (uint32) or a closed form: for the affine family
// x = A^-1 (y - B) mod 2^k; for modular multiplication (y -> A y mod N for
// y < N, y itself above) x = A^-1 y mod N for y < N, reduced by Barrett's
// method with mu = floor((2^64 - 1) / N): for p = A^-1 y < N^2 < 2^64 the
// quotient estimate hi64(p mu) is floor(p / N) or one less, so one
// conditional subtraction finishes the reduction.

__device__ __forceinline__ uint64_t mod_barrett(uint64_t p, uint64_t N, uint64_t mu) {
  const uint64_t q = __umul64hi(p, mu);
  uint64_t r = p - q * N;
  if (r >= N) r -= N;
  return r;
}

template <typename R>
__global__ __launch_bounds__(kBlock) void k_perm_gather(const V2<R>* __restrict__ in, V2<R>* __restrict__ out,
                                                        uint64_t nitems, Special sp, uint64_t cmask, Pos32 tp, int k,
                                                        int contiguous, uint64_t tmask,
                                                        const uint32_t* __restrict__ finv, int mode, uint64_t B,
                                                        uint64_t Ainv, uint64_t N, uint64_t mu, int whole,
                                                        CondArgs cond) {
  const bool run = conds_ok(cond);
  if (!run && !whole) return;
  const uint64_t kmask = (k >= 64) ? ~0ull : ((1ull << k) - 1);
  const uint64_t stride = (uint64_t)gridDim.x * kBlock;
  for (uint64_t e = (uint64_t)blockIdx.x * kBlock + threadIdx.x; e < nitems; e += stride) {
    const uint64_t i = insert_zeros(e, sp) | cmask;
    uint64_t src = i;
    if (run) {
      const uint64_t y = contiguous ? ((i >> tp.p[0]) & kmask) : extract(i, tp.p, k);
      uint64_t x;
      if (mode == 1) x = (Ainv * (y - B)) & kmask;
      else if (mode == 2) x = (y < N) ? mod_barrett(Ainv * y, N, mu) : y;   // Ainv, y < N < 2^32
      else x = (uint64_t)finv[y];
      src = (i & ~tmask) | (contiguous ? (x << tp.p[0]) : deposit(x, tp.p, k));
    }
    out[e] = in[src];
  }
}

template <typename R>
__global__ __launch_bounds__(kBlock) void k_perm_scatter(V2<R>* __restrict__ psi, const V2<R>* __restrict__ scratch,
                                                         uint64_t nitems, Special sp, uint64_t cmask, CondArgs cond) {
  if (!conds_ok(cond)) return;
  const uint64_t stride = (uint64_t)gridDim.x * kBlock;
  for (uint64_t e = (uint64_t)blockIdx.x * kBlock + threadIdx.x; e < nitems; e += stride)
    psi[insert_zeros(e, sp) | cmask] = scratch[e];
}

hipError_t launch_perm(const Launch& L, void* scratch, const int* targets, int k, const int* controls, int nc,
                       const uint32_t* d_finv, int mode, uint64_t A, uint64_t B, uint64_t Ainv, uint64_t N,
                       bool out_of_place) {
  (void)A;
  if (k < 1 || k > 32) return hipErrorInvalidValue;
  if (out_of_place && nc != 0) return hipErrorInvalidValue;
  if (mode == 2 && (N < 2 || N > 0xffffffffull)) return hipErrorInvalidValue;
  // the gather enumerates the controlled subspace; targets are part of it
  Special sp = make_special(controls, nc, nullptr, 0);
  const uint64_t nitems = 1ull << (L.n - nc);
  Pos32 tp{};
  int contiguous = 1;
  for (int j = 0; j < k; ++j) {
    tp.p[j] = targets[j];
    if (targets[j] != targets[0] + j) contiguous = 0;
  }
  const uint64_t tmask = mask_of(targets, k), cmask = mask_of(controls, nc);
  const uint64_t mu = (mode == 2) ? ~0ull / N : 0;
  const int whole = out_of_place ? 1 : 0;
  const unsigned g = (unsigned)std::min<uint64_t>((nitems + kBlock * 4 - 1) / (kBlock * 4), 1u << 20);
  if (L.c64) {
    hipLaunchKernelGGL(k_perm_gather<float>, dim3(g), dim3(kBlock), 0, L.stream, (const float2*)L.psi,
                       (float2*)scratch, nitems, sp, cmask, tp, k, contiguous, tmask, d_finv, mode, B, Ainv, N, mu,
                       whole, L.cond);
    if (!out_of_place)
      hipLaunchKernelGGL(k_perm_scatter<float>, dim3(g), dim3(kBlock), 0, L.stream, (float2*)L.psi,
                         (const float2*)scratch, nitems, sp, cmask, L.cond);
  } else {
    hipLaunchKernelGGL(k_perm_gather<double>, dim3(g), dim3(kBlock), 0, L.stream, (const double2*)L.psi,
                       (double2*)scratch, nitems, sp, cmask, tp, k, contiguous, tmask, d_finv, mode, B, Ainv, N, mu,
                       whole, L.cond);
    if (!out_of_place)
      hipLaunchKernelGGL(k_perm_scatter<double>, dim3(g), dim3(kBlock), 0, L.stream, (double2*)L.psi,
                         (const double2*)scratch, nitems, sp, cmask, L.cond);
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------- measurement
// (1) every block sums |a_i|^2 of a fixed contiguous range in FP64, split by
// bit q, with a fixed thread->element mapping and a fixed reduction tree;
// (2) one block adds the block sums in index order, draws the outcome
// (u < P0 ? 0 : 1), writes the cbit, 1/sqrt(p_outcome) and a log entry;
// (3) the collapse reads the outcome from device memory, scales the kept half
// and zeroes the other.  The result depends only on the state, never on what
// else runs on the device.

__device__ __forceinline__ double wave_sum(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Fixed-order sum over a 256-thread block; result valid in thread 0.
__device__ __forceinline__ double block_sum(double v, double* sh) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) sh[w] = v;
  __syncthreads();
  double s = 0;
  if (threadIdx.x == 0) s = ((sh[0] + sh[1]) + sh[2]) + sh[3];
  return s;
}

// Workgroups of a fixed-order reduction: one per 2048 elements, at most
// kReduceBlocks (so at 21 qubits the pass already spreads over 1024
// workgroups; from 2^21 elements up the count is fixed and the order with it).
int reduce_blocks_for(uint64_t count) {
  uint64_t b = count / 2048;
  if (b < 1) b = 1;
  if (b > (uint64_t)kReduceBlocks) b = kReduceBlocks;
  return (int)b;
}

// Each block sums a fixed contiguous range with 16-byte loads (one complex128
// or two complex64 amplitudes), eight loads in flight per thread, and a
// fixed thread -> element mapping and reduction tree.
template <typename R>
__global__ __launch_bounds__(kBlock) void k_prob_partial(const V2<R>* __restrict__ psi, uint64_t dim,
                                                         uint64_t per_block, uint64_t qbit, double* partials) {
  constexpr int VEC = 16 / (int)sizeof(V2<R>);   // amplitudes per load
  constexpr int U = 8;                            // loads in flight per thread
  using L = typename std::conditional<VEC == 1, double2, float4>::type;
  __shared__ double sh[4];
  const L* p = reinterpret_cast<const L*>(psi);
  const uint64_t start = (uint64_t)blockIdx.x * per_block / VEC;
  const uint64_t end = ((uint64_t)blockIdx.x * per_block + per_block < dim ? (uint64_t)blockIdx.x * per_block + per_block
                                                                            : dim) / VEC;
  double s0[U], s1[U];
#pragma unroll
  for (int u = 0; u < U; ++u) s0[u] = s1[u] = 0.0;
  for (uint64_t i = start + threadIdx.x; i < end; i += (uint64_t)U * kBlock) {
    L a[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const uint64_t ii = i + (uint64_t)u * kBlock;
      if (ii < end) a[u] = p[ii];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const uint64_t ii = i + (uint64_t)u * kBlock;
      if (ii < end) {
        if constexpr (VEC == 1) {
          const double w = a[u].x * a[u].x + a[u].y * a[u].y;
          if (ii & qbit) s1[u] += w; else s0[u] += w;
        } else {
          const double w0 = (double)a[u].x * (double)a[u].x + (double)a[u].y * (double)a[u].y;
          const double w1 = (double)a[u].z * (double)a[u].z + (double)a[u].w * (double)a[u].w;
          if (qbit == 1) {
            s0[u] += w0;
            s1[u] += w1;
          } else if ((2 * ii) & qbit) {
            s1[u] += w0 + w1;
          } else {
            s0[u] += w0 + w1;
          }
        }
      }
    }
  }
  double t0 = 0, t1 = 0;
#pragma unroll
  for (int u = 0; u < U; ++u) {
    t0 += s0[u];
    t1 += s1[u];
  }
  t0 = block_sum(t0, sh);
  t1 = block_sum(t1, sh);
  if (threadIdx.x == 0) {
    partials[2 * blockIdx.x] = t0;
    partials[2 * blockIdx.x + 1] = t1;
  }
}

__global__ __launch_bounds__(kBlock) void k_meas_finalize(const double* __restrict__ partials, int nblocks, double u,
                                                          const double* d_u, int forced, int cbit, double* result,
                                                          uint8_t* cbits, double* log, uint32_t* log_count,
                                                          double* out) {
  __shared__ double sh[4];
  double a0 = 0, a1 = 0;
  for (int b = threadIdx.x; b < nblocks; b += kBlock) {
    a0 += partials[2 * b];
    a1 += partials[2 * b + 1];
  }
  const double p0 = block_sum(a0, sh);
  const double p1 = block_sum(a1, sh);
  if (threadIdx.x == 0) {
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
    if (log) {
      const uint32_t c = *log_count;
      const uint32_t slot = c % (uint32_t)kMeasLog;
      log[3 * slot] = p0;
      log[3 * slot + 1] = p1;
      log[3 * slot + 2] = (double)oc;
      *log_count = c + 1;
    }
    if (out) {
      out[0] = p0;
      out[1] = p1;
      out[2] = (double)oc;
    }
  }
}

template <typename R, int ITEMS>
__global__ __launch_bounds__(kBlock) void k_collapse(V2<R>* __restrict__ psi, uint64_t npairs, int q,
                                                     const double* __restrict__ result, bool xcd) {
  const double scale_d = result[2];
  if (scale_d == 0.0) return;
  const R scale = (R)scale_d;
  const int oc = (int)result[3];
  const uint64_t qb = 1ull << q, lo = qb - 1;
  const uint64_t j0 = sweep_block(xcd) * (kBlock * ITEMS) + threadIdx.x;
  V2<R> x[ITEMS];
  uint64_t keep[ITEMS];
#pragma unroll
  for (int it = 0; it < ITEMS; ++it) {
    const uint64_t j = j0 + (uint64_t)it * kBlock;
    const uint64_t i0 = ((j & ~lo) << 1) | (j & lo);
    keep[it] = oc ? (i0 | qb) : i0;
    if (j < npairs) x[it] = psi[keep[it]];
  }
#pragma unroll
  for (int it = 0; it < ITEMS; ++it) {
    const uint64_t j = j0 + (uint64_t)it * kBlock;
    if (j < npairs) {
      psi[keep[it]] = V2<R>{x[it].x * scale, x[it].y * scale};
      psi[keep[it] ^ qb] = V2<R>{0, 0};
    }
  }
}

hipError_t launch_measure(const Launch& L, int qubit, int cbit, double u, const double* d_u, int forced,
                          const MeasBuffers& mb) {
  const uint64_t dim = 1ull << L.n;
  const int nb = reduce_blocks_for(dim);
  const uint64_t per_block = (dim + nb - 1) / nb;
  if (L.c64)
    hipLaunchKernelGGL(k_prob_partial<float>, dim3(nb), dim3(kBlock), 0, L.stream, (const float2*)L.psi, dim,
                       per_block, 1ull << qubit, mb.partials);
  else
    hipLaunchKernelGGL(k_prob_partial<double>, dim3(nb), dim3(kBlock), 0, L.stream, (const double2*)L.psi, dim,
                       per_block, 1ull << qubit, mb.partials);
  hipLaunchKernelGGL(k_meas_finalize, dim3(1), dim3(kBlock), 0, L.stream, (const double*)mb.partials, nb, u, d_u,
                     forced, cbit, mb.result, mb.cbits, mb.log, mb.log_count, mb.out);
  const uint64_t npairs = dim >> 1;
  // four pairs per thread on large states; one on small ones, where the
  // launch would otherwise have too few workgroups to cover the latency
  auto collapse = [&](auto tag_it) {
    constexpr int IT = decltype(tag_it)::value;
    const dim3 g = grid_for(npairs, kBlock * IT);
    if (L.c64)
      hipLaunchKernelGGL((k_collapse<float, IT>), g, dim3(kBlock), 0, L.stream, (float2*)L.psi, npairs, qubit,
                         (const double*)mb.result, L.tune.xcd != 0);
    else
      hipLaunchKernelGGL((k_collapse<double, IT>), g, dim3(kBlock), 0, L.stream, (double2*)L.psi, npairs, qubit,
                         (const double*)mb.result, L.tune.xcd != 0);
  };
  if (npairs >= (1ull << 24)) collapse(std::integral_constant<int, 4>{});
  else collapse(std::integral_constant<int, 1>{});
  return hipGetLastError();
}

// ---------------------------------------------------------------- allocation-free measurement
// The measurement kernels need a scratch buffer for the partial sums of the
// reduction grid and the 4-double result.  For callers that cannot allocate,
// it is this file-scope device array (one copy per GPU, held until the process
// ends).  Host code never passes the array's name to a kernel: its device
// address is looked up once per device and kept.

constexpr size_t kNoAllocDoubles = 2 * kReduceBlocks + 8;   // 16,448 bytes
static __device__ __align__(256) double scratch[kNoAllocDoubles];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static double* g_scratch_ptr[kMaxDevices] = {};

static hipError_t noalloc_scratch(int device, double** out) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    int prev = -1;
    hipError_t e = hipGetDevice(&prev);
    if (e != hipSuccess) return e;
    if (prev != device && (e = hipSetDevice(device)) != hipSuccess) return e;
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (prev != device) (void)hipSetDevice(prev);
    if (e != hipSuccess) return e;
    g_scratch_ptr[device] = (double*)p;
  }
  *out = g_scratch_ptr[device];
  return hipSuccess;
}

hipError_t launch_measure_noalloc(int device, hipStream_t stream, void* psi, int n, bool c64, int qubit,
                                  const double* d_u, uint8_t* d_cbit, double* d_out) {
  double* sc = nullptr;
  hipError_t e = noalloc_scratch(device, &sc);
  if (e != hipSuccess) return e;
  MeasBuffers mb;
  mb.partials = sc;                       // 2 * kReduceBlocks doubles, every slot rewritten by each call
  mb.result = sc + 2 * kReduceBlocks;     // p0, p1, scale, outcome
  mb.cbits = d_cbit;
  mb.out = d_out;
  Launch L{};
  L.stream = stream;
  L.n = n;
  L.c64 = c64;
  L.psi = psi;
  return launch_measure(L, qubit, d_cbit ? 0 : -1, 0.0, d_u, -1, mb);
}

// ---------------------------------------------------------------- inner product
// Block partials of sum conj(a_i) b_i in FP64 over fixed ranges; the host adds
// them in index order.

template <typename RA, typename RB>
__global__ __launch_bounds__(kBlock) void k_inner_partials(const V2<RA>* __restrict__ a, const V2<RB>* __restrict__ b,
                                                           uint64_t dim, uint64_t per_block, double* partials) {
  __shared__ double sh[4];
  const uint64_t start = (uint64_t)blockIdx.x * per_block;
  const uint64_t end = (start + per_block < dim) ? start + per_block : dim;
  double re = 0, im = 0;
  for (uint64_t i = start + threadIdx.x; i < end; i += kBlock) {
    const double ar = a[i].x, ai = a[i].y, br = b[i].x, bi = b[i].y;
    re += ar * br + ai * bi;
    im += ar * bi - ai * br;
  }
  const double tr = block_sum(re, sh);
  const double ti = block_sum(im, sh);
  if (threadIdx.x == 0) {
    partials[2 * blockIdx.x] = tr;
    partials[2 * blockIdx.x + 1] = ti;
  }
}

hipError_t launch_inner_partials(const void* a, bool a64, const void* b, bool b64, uint64_t dim, double* partials,
                                 int nblocks, hipStream_t s) {
  const uint64_t per_block = (dim + nblocks - 1) / nblocks;
  if (a64 && b64)
    hipLaunchKernelGGL((k_inner_partials<float, float>), dim3(nblocks), dim3(kBlock), 0, s, (const float2*)a,
                       (const float2*)b, dim, per_block, partials);
  else if (a64)
    hipLaunchKernelGGL((k_inner_partials<float, double>), dim3(nblocks), dim3(kBlock), 0, s, (const float2*)a,
                       (const double2*)b, dim, per_block, partials);
  else if (b64)
    hipLaunchKernelGGL((k_inner_partials<double, float>), dim3(nblocks), dim3(kBlock), 0, s, (const double2*)a,
                       (const float2*)b, dim, per_block, partials);
  else
    hipLaunchKernelGGL((k_inner_partials<double, double>), dim3(nblocks), dim3(kBlock), 0, s, (const double2*)a,
                       (const double2*)b, dim, per_block, partials);
  return hipGetLastError();
}

}  // namespace qk
