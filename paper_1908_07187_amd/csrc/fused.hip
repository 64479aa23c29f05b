// Dense 2^K x 2^K gate (K = 2..6) on arbitrary target bits as a complex GEMM
// on gfx950 matrix cores.
//
// Tile: 2^K rows (the target combinations, gate index m) x 16 columns (the
// 16 combinations of the 4 lowest bits outside targets and controls, so a row
// of the tile is up to 16 consecutive amplitudes).  One wave owns one tile
// ("chunk") at a time; chunks are the remaining bits.  With the real
// embedding Y = [[Mr, -Mi], [Mi, Mr]] [Xr; Xi] the tile update is a
// (2^(K+1) x 2^(K+1)) x (2^(K+1) x 16) real GEMM, run as 16x16x4 MFMA steps:
//   B operand: lane (h = lane/16, c = lane%16) loads the amplitude at tile row
//     m = 4 ks + h, column c (one float2/double2); its real part feeds one MFMA
//     and its imaginary part a second one, so no lane loads anything twice;
//   A operand: the matching columns of the real-embedded matrix, staged once
//     per block in LDS in per-lane fragment order (conflict-free reads);
//   D: 16x16 accumulators per 16-row tile; the rows are arranged so that lane
//     (h, v) holds real row 4h + v, i.e. the (re, im) pairs of two complex
//     rows, stored straight back as float2/double2 (16 lanes = one contiguous
//     run of 16 amplitudes).
// Complex64 states use v_mfma_f32_16x16x4f32 (FP32 products and accumulation);
// complex128 states use v_mfma_f64_16x16x4f64.  The f32 and f64 instructions
// place D rows differently (row 4h+v vs 4v+h for lane h, register v), which the
// A staging absorbs by permuting the rows.
// Each wave prefetches the next chunk's 2^K/4 loads before the current MFMAs.
#include <algorithm>

#include "qk_internal.h"

namespace qk {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef double doublex4 __attribute__((ext_vector_type(4)));

template <typename R> struct MF;
template <> struct MF<float> {
  using V = float2;
  using Acc = floatx4;
  static constexpr bool kRowsByReg = false;   // D[i][j] at lane j + 16 (i / 4), register i % 4
  __device__ static Acc op(float a, float b, Acc c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
};
template <> struct MF<double> {
  using V = double2;
  using Acc = doublex4;
  static constexpr bool kRowsByReg = true;    // D[i][j] at lane j + 16 (i % 4), register i / 4
  __device__ static Acc op(double a, double b, Acc c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
};

struct MfmaArgs {
  int tpos[6];   // target bit of gate index bit j
  int lpos[4];   // column bits
};

__device__ __forceinline__ bool conds_ok_m(const CondArgs& c) {
  for (int i = 0; i < c.n; ++i)
    if (c.cbits[c.cbit[i]] != (uint8_t)c.val[i]) return false;
  return true;
}

__device__ __forceinline__ uint64_t insert_zeros_m(uint64_t x, const Special& s) {
  for (int i = 0; i < s.n; ++i) {
    const int p = s.pos[i];
    const uint64_t lo = x & ((1ull << p) - 1);
    x = ((x >> p) << (p + 1)) | lo;
  }
  return x;
}

template <int K>
__device__ __forceinline__ uint64_t dep_t(uint32_t m, const MfmaArgs& a) {
  uint64_t i = 0;
#pragma unroll
  for (int j = 0; j < K; ++j) i |= (uint64_t)((m >> j) & 1u) << a.tpos[j];
  return i;
}

template <typename R, int K>
__global__ __launch_bounds__(256) void k_dense_mfma(typename MF<R>::V* psi, const typename MF<R>::V* __restrict__ mat,
                                                    uint64_t nchunks, Special sp, uint64_t cmask, MfmaArgs ma,
                                                    CondArgs cond) {
  using V = typename MF<R>::V;
  using Acc = typename MF<R>::Acc;
  constexpr int DIM = 1 << K;
  constexpr int RT = (2 * DIM + 15) / 16;   // 16-row tiles of the real output
  constexpr int KS = DIM / 4;               // steps of 4 complex input rows
  constexpr int NF = RT * KS * 2;           // A fragments (one value per lane each)
  extern __shared__ unsigned char smem_raw[];
  R* afrag = reinterpret_cast<R*>(smem_raw);

  if (!conds_ok_m(cond)) return;

  // Stage the real-embedded matrix in fragment order: fragment f = (rt, ks, part).
  for (int e = threadIdx.x; e < NF * 64; e += 256) {
    const int l = e & 63, f = e >> 6;
    const int part = f & 1, ks = (f >> 1) % KS, rt = (f >> 1) / KS;
    const int i = l & 15, kk = l >> 4;
    const int rho = 16 * rt + (MF<R>::kRowsByReg ? (4 * (i & 3) + (i >> 2)) : i);
    const int r = rho >> 1, m = 4 * ks + kk;
    R val = 0;
    if (r < DIM) {
      const V z = mat[r * DIM + m];
      if ((rho & 1) == 0) val = part == 0 ? z.x : -z.y;   // Re-row: Mr * xr - Mi * xi
      else val = part == 0 ? z.y : z.x;                   // Im-row: Mi * xr + Mr * xi
    }
    afrag[e] = val;
  }
  __syncthreads();

  const int lane = threadIdx.x & 63;
  const int h = lane >> 4, c = lane & 15;
  uint64_t coloff = 0;
#pragma unroll
  for (int b = 0; b < 4; ++b) coloff |= (uint64_t)((c >> b) & 1) << ma.lpos[b];
  // input row m = 4 ks + h = (4 ks) | h: the ks part is uniform, the h part per lane
  const uint64_t lo_in = dep_t<K>((uint32_t)h, ma) | coloff;
  // output rows r = 8 rt + 2 h + s
  const bool wr0 = (2 * h) < DIM;          // false only for K = 2, h >= 2 (padding rows)
  const uint64_t lo_out0 = dep_t<K>((uint32_t)(2 * h) & (DIM - 1), ma) | coloff;
  const uint64_t lo_out1 = dep_t<K>((uint32_t)(2 * h + 1) & (DIM - 1), ma) | coloff;

  const uint64_t wid = (uint64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const uint64_t nw = (uint64_t)gridDim.x * 4;

  V xa[KS], xb[KS];
  auto load = [&](uint64_t base, V* x) {
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) x[ks] = psi[base + dep_t<K>((uint32_t)(4 * ks), ma) + lo_in];
  };
  auto compute_store = [&](uint64_t base, const V* x) {
    Acc acc[RT];
#pragma unroll
    for (int rt = 0; rt < RT; ++rt) acc[rt] = Acc{0, 0, 0, 0};
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
#pragma unroll
      for (int rt = 0; rt < RT; ++rt) {
        const int f = (rt * KS + ks) * 2;
        acc[rt] = MF<R>::op(afrag[f * 64 + lane], x[ks].x, acc[rt]);
        acc[rt] = MF<R>::op(afrag[(f + 1) * 64 + lane], x[ks].y, acc[rt]);
      }
    }
#pragma unroll
    for (int rt = 0; rt < RT; ++rt) {
      if (wr0) {
        const uint64_t hi = dep_t<K>((uint32_t)(8 * rt), ma);
        psi[base + hi + lo_out0] = V{acc[rt][0], acc[rt][1]};
        psi[base + hi + lo_out1] = V{acc[rt][2], acc[rt][3]};
      }
    }
  };

  uint64_t ch = wid;
  if (ch >= nchunks) return;
  uint64_t base = insert_zeros_m(ch, sp) | cmask;
  load(base, xa);
  for (;;) {
    uint64_t nx = ch + nw;
    uint64_t nbase = 0;
    if (nx < nchunks) {
      nbase = insert_zeros_m(nx, sp) | cmask;
      load(nbase, xb);
    }
    compute_store(base, xa);
    if (nx >= nchunks) break;
    ch = nx;
    base = nbase;
    nx = ch + nw;
    if (nx < nchunks) {
      nbase = insert_zeros_m(nx, sp) | cmask;
      load(nbase, xa);
    }
    compute_store(base, xb);
    if (nx >= nchunks) break;
    ch = nx;
    base = nbase;
  }
}

bool mfma_supported(int n, int k, int nc, bool c64) {
  (void)c64;
  return k >= 2 && k <= 6 && n - k - nc >= 4;
}

template <typename R, int K>
static hipError_t launch_k(const Launch& L, const void* mat, uint64_t nchunks, const Special& sp, uint64_t cmask,
                           const MfmaArgs& ma, int waves_per_cu) {
  constexpr int DIM = 1 << K;
  constexpr int RT = (2 * DIM + 15) / 16;
  constexpr int KS = DIM / 4;
  const size_t shm = (size_t)RT * KS * 2 * 64 * sizeof(R);
  static bool attr_set = false;
  if (!attr_set) {
    hipError_t e = hipFuncSetAttribute((const void*)k_dense_mfma<R, K>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)shm);
    if (e != hipSuccess) return e;
    attr_set = true;
  }
  int ncu = 256;
  {
    int dev = 0;
    if (hipGetDevice(&dev) == hipSuccess) {
      int v = 0;
      if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && v > 0) ncu = v;
    }
  }
  const uint64_t want = (nchunks + 3) / 4;
  uint64_t cap = (uint64_t)ncu * std::max(1, waves_per_cu / 4);
  const unsigned g = (unsigned)std::max<uint64_t>(1, std::min(want, cap));
  hipLaunchKernelGGL((k_dense_mfma<R, K>), dim3(g), dim3(256), shm, L.stream, (typename MF<R>::V*)L.psi,
                     (const typename MF<R>::V*)mat, nchunks, sp, cmask, ma, L.cond);
  return hipGetLastError();
}

hipError_t launch_dense_mfma(const Launch& L, const int* targets, int k, const int* controls, int nc,
                             const void* d_matrix, int waves_per_cu) {
  if (!mfma_supported(L.n, k, nc, L.c64)) return hipErrorInvalidValue;
  MfmaArgs ma{};
  uint64_t used = 0;
  for (int j = 0; j < k; ++j) {
    ma.tpos[j] = targets[j];
    used |= 1ull << targets[j];
  }
  for (int j = 0; j < nc; ++j) used |= 1ull << controls[j];
  int nl = 0;
  for (int b = 0; b < L.n && nl < 4; ++b)
    if (!((used >> b) & 1)) ma.lpos[nl++] = b;
  std::vector<int> sv(targets, targets + k);
  for (int j = 0; j < nc; ++j) sv.push_back(controls[j]);
  for (int j = 0; j < 4; ++j) sv.push_back(ma.lpos[j]);
  Special sp = make_special(sv.data(), (int)sv.size(), nullptr, 0);
  uint64_t cmask = 0;
  for (int j = 0; j < nc; ++j) cmask |= 1ull << controls[j];
  const uint64_t nchunks = 1ull << (L.n - k - nc - 4);
  if (waves_per_cu <= 0) waves_per_cu = 8;
  if (L.c64) {
    switch (k) {
      case 2: return launch_k<float, 2>(L, d_matrix, nchunks, sp, cmask, ma, waves_per_cu);
      case 3: return launch_k<float, 3>(L, d_matrix, nchunks, sp, cmask, ma, waves_per_cu);
      case 4: return launch_k<float, 4>(L, d_matrix, nchunks, sp, cmask, ma, waves_per_cu);
      case 5: return launch_k<float, 5>(L, d_matrix, nchunks, sp, cmask, ma, waves_per_cu);
      case 6: return launch_k<float, 6>(L, d_matrix, nchunks, sp, cmask, ma, waves_per_cu);
    }
  } else {
    switch (k) {
      case 2: return launch_k<double, 2>(L, d_matrix, nchunks, sp, cmask, ma, waves_per_cu);
      case 3: return launch_k<double, 3>(L, d_matrix, nchunks, sp, cmask, ma, waves_per_cu);
      case 4: return launch_k<double, 4>(L, d_matrix, nchunks, sp, cmask, ma, waves_per_cu);
      case 5: return launch_k<double, 5>(L, d_matrix, nchunks, sp, cmask, ma, waves_per_cu);
      case 6: return launch_k<double, 6>(L, d_matrix, nchunks, sp, cmask, ma, waves_per_cu);
    }
  }
  return hipErrorInvalidValue;
}

}  // namespace qk
