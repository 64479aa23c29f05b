// Dense 2^K x 2^K gate (K = 2..6) on arbitrary target bits as a complex GEMM
// on gfx950 matrix cores.
//
// Tile: 2^K rows (the target combinations, gate index m) x CW columns (the
// combinations of the log2(CW) lowest bits outside targets and controls, so a
// row of the tile is a run of CW consecutive amplitudes when those bits are
// the lowest ones).  One wave owns one tile ("chunk") at a time; chunks are
// the remaining bits.  With the real embedding Y = [[Mr, -Mi], [Mi, Mr]]
// [Xr; Xi] the tile update is a (2^(K+1) x 2^(K+1)) x (2^(K+1) x CW) real
// GEMM, run as 16x16x4 MFMA steps in CW/16 independent column groups:
//   B operand: lane (h = lane/16, c = lane%16) loads the amplitude at tile row
//     m = 4 ks + h, column c + 16 g (one float2/double2); its real part feeds
//     one MFMA and its imaginary part a second one, so nothing is loaded twice;
//   A operand: the matching columns of the real-embedded matrix, staged once
//     per block in LDS in per-lane fragment order (conflict-free reads); each
//     A read serves all CW/16 column groups;
//   D: 16x16 accumulators per 16-row tile and column group; the rows are
//     arranged so that lane (h, v) holds real row 4h + v, i.e. the (re, im)
//     pairs of two complex rows, stored straight back as float2/double2.
// Complex64 states use v_mfma_f32_16x16x4f32 (FP32 products and accumulation);
// complex128 states use v_mfma_f64_16x16x4f64.  The f32 and f64 instructions
// place D rows differently (row 4h+v vs 4v+h for lane h, register v), which the
// A staging absorbs by permuting the rows.
// Each wave prefetches the next chunk's loads before the current MFMAs; wider
// tiles (CW = 32, 64) keep more bytes in flight per wave.
#include <algorithm>
#include <type_traits>

#include "qk_internal.h"

namespace qk {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef double doublex4 __attribute__((ext_vector_type(4)));

template <typename R> struct MF;
template <> struct MF<float> {
  typedef float V __attribute__((ext_vector_type(2)));
  using Acc = floatx4;
  static constexpr bool kRowsByReg = false;   // D[i][j] at lane j + 16 (i / 4), register i % 4
  __device__ static Acc op(float a, float b, Acc c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
};
template <> struct MF<double> {
  typedef double V __attribute__((ext_vector_type(2)));
  using Acc = doublex4;
  static constexpr bool kRowsByReg = true;    // D[i][j] at lane j + 16 (i % 4), register i / 4
  __device__ static Acc op(double a, double b, Acc c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
};

struct MfmaArgs {
  int tpos[6];   // target bit of gate index bit j
  int lpos[6];   // column bits (log2(CW) of them)
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

template <bool NT, typename T>
__device__ __forceinline__ T mld(const T* p) {
  if constexpr (NT) return __builtin_nontemporal_load(p);
  else return *p;
}
template <bool NT, typename T>
__device__ __forceinline__ void mst(T* p, T v) {
  if constexpr (NT) __builtin_nontemporal_store(v, p);
  else *p = v;
}

template <typename R, int K, int CW, bool NT, bool AREG>
__global__ __launch_bounds__(256) void k_dense_mfma(typename MF<R>::V* psi, const typename MF<R>::V* __restrict__ mat,
                                                    uint64_t nchunks, Special sp, uint64_t cmask, MfmaArgs ma,
                                                    CondArgs cond, bool xcd) {
  using V = typename MF<R>::V;
  using Acc = typename MF<R>::Acc;
  constexpr int DIM = 1 << K;
  constexpr int RT = (2 * DIM + 15) / 16;   // 16-row tiles of the real output
  constexpr int KS = DIM / 4;               // steps of 4 complex input rows
  constexpr int NF = RT * KS * 2;           // A fragments (one value per lane each)
  constexpr int G = CW / 16;                // column groups per wave
  constexpr int LB = (CW == 16) ? 4 : (CW == 32 ? 5 : 6);
  extern __shared__ __align__(16) unsigned char smem_raw[];
  R* afrag = reinterpret_cast<R*>(smem_raw);
  // AREG = false: the A fragments are re-read from LDS for every tile.  The
  // offset `zoff` (always 0) passes through an empty asm statement per tile,
  // so the compiler cannot hoist the fragment reads into registers; this keeps
  // the register count (and so the waves per SIMD) of large blocks in check.
  // (A memory read of a zero would do the same but, issued through the
  // generic address space, it would also drain the prefetched global loads.)

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
  uint64_t lo_in[G], lo_out0[G], lo_out1[G];
  const uint64_t din = dep_t<K>((uint32_t)h, ma);
  const uint64_t dout0 = dep_t<K>((uint32_t)(2 * h) & (DIM - 1), ma);
  const uint64_t dout1 = dep_t<K>((uint32_t)(2 * h + 1) & (DIM - 1), ma);
#pragma unroll
  for (int g = 0; g < G; ++g) {
    uint64_t coloff = 0;
    const int col = c + 16 * g;
#pragma unroll
    for (int b = 0; b < LB; ++b) coloff |= (uint64_t)((col >> b) & 1) << ma.lpos[b];
    lo_in[g] = din | coloff;
    lo_out0[g] = dout0 | coloff;
    lo_out1[g] = dout1 | coloff;
  }
  const bool wr0 = (2 * h) < DIM;          // false only for K = 2, h >= 2 (padding rows)

  // xcd: workgroups are numbered so that the ones an XCD runs (every eighth
  // in launch order) take one contiguous range of chunks
  uint64_t blk = blockIdx.x;
  if (xcd && !(gridDim.x & 7)) blk = (blk & 7) * (gridDim.x >> 3) + (blk >> 3);
  const uint64_t wid = blk * 4 + (threadIdx.x >> 6);
  const uint64_t nw = (uint64_t)gridDim.x * 4;

  V xa[KS][G], xb[KS][G];
  auto load = [&](uint64_t base, V (*x)[G]) {
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
      const uint64_t row = base + dep_t<K>((uint32_t)(4 * ks), ma);
#pragma unroll
      for (int g = 0; g < G; ++g) x[ks][g] = mld<NT>(psi + row + lo_in[g]);
    }
  };
  auto compute_store = [&](uint64_t base, V (*x)[G]) {
    int zoff = 0;
    if constexpr (!AREG) asm volatile("" : "+s"(zoff));
    Acc acc[RT][G];
#pragma unroll
    for (int rt = 0; rt < RT; ++rt)
#pragma unroll
      for (int g = 0; g < G; ++g) acc[rt][g] = Acc{0, 0, 0, 0};
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
#pragma unroll
      for (int rt = 0; rt < RT; ++rt) {
        const int f = (rt * KS + ks) * 2;
        const R a0 = afrag[f * 64 + lane + zoff];
        const R a1 = afrag[(f + 1) * 64 + lane + zoff];
#pragma unroll
        for (int g = 0; g < G; ++g) {
          acc[rt][g] = MF<R>::op(a0, x[ks][g].x, acc[rt][g]);
          acc[rt][g] = MF<R>::op(a1, x[ks][g].y, acc[rt][g]);
        }
      }
    }
#pragma unroll
    for (int rt = 0; rt < RT; ++rt) {
      if (wr0) {
        const uint64_t hi = base + dep_t<K>((uint32_t)(8 * rt), ma);
#pragma unroll
        for (int g = 0; g < G; ++g) {
          V v0, v1;
          v0.x = acc[rt][g][0];
          v0.y = acc[rt][g][1];
          v1.x = acc[rt][g][2];
          v1.y = acc[rt][g][3];
          mst<NT>(psi + hi + lo_out0[g], v0);
          mst<NT>(psi + hi + lo_out1[g], v1);
        }
      }
    }
  };

  // The next chunk's loads are issued unconditionally (the last chunk loads
  // itself once more and drops the values): with the same number of loads in
  // flight on every path, the wait before a chunk's MFMAs covers only that
  // chunk's own loads instead of draining the prefetch as well.
  uint64_t ch = wid;
  if (ch >= nchunks) return;
  uint64_t base = insert_zeros_m(ch, sp) | cmask;
  load(base, xa);
  for (;;) {
    uint64_t nx = ch + nw;
    bool more = nx < nchunks;
    uint64_t nbase = more ? (insert_zeros_m(nx, sp) | cmask) : base;
    load(nbase, xb);
    compute_store(base, xa);
    if (!more) break;
    ch = nx;
    base = nbase;
    nx = ch + nw;
    more = nx < nchunks;
    nbase = more ? (insert_zeros_m(nx, sp) | cmask) : base;
    load(nbase, xa);
    compute_store(base, xb);
    if (!more) break;
    ch = nx;
    base = nbase;
  }
}

// ---------------------------------------------------------------- LDS-staged tiles
// The same GEMM with the tile staged through LDS by the whole workgroup, so
// that global memory is read and written in address order: every wave-wide
// access is 64 consecutive 16-byte pieces (1 KiB).
// Tile = 2^K rows (gate index m) x CW = 2^LB columns (the LB lowest bits
// outside targets and controls); since the column bits are the lowest free
// bits, the tile's amplitudes form runs of at least CW consecutive
// amplitudes.  The tile-local address index j has one bit per bit of U =
// targets + column bits (ascending); both its global offset and its LDS
// position (row m, column c) are sums of per-bit weights, so a thread's part
// and each access's part are added.
//   load:    global (address order) -> registers, prefetched one tile ahead;
//   stage:   registers -> LDS X[m][c] (row stride CW + 1);
//   compute: wave w takes column groups [w*GW, (w+1)*GW); MFMA as above with
//            the B operand from LDS and the A operand from the complex matrix
//            kept in LDS (row stride DIM + 1): one 16-byte read gives both
//            real-embedding values a lane needs for an MFMA pair;
//   store:   results written over the wave's own columns of X, then
//            LDS -> global in address order.
// Stand-alone variants of this kernel at 30 qubits showed its time is set by
// the memory side: with the MFMAs removed it runs 4-12 % faster than the full
// kernel, yet 15-50 % slower than a plain in-place sweep of the same state
// (more so when the tile's rows lie far apart in memory); with the global
// accesses removed, 5-qubit blocks still take 90-97 % of a plain sweep's
// time.  Storing straight from the accumulators (runs of 16 columns per row)
// was slower than the address-order stores, and more workgroups per compute
// unit or a second tile of prefetch did not help.
static int g_ncu = 0;

struct LdsTileArgs {
  int tpos[6];         // target bit of gate index bit j
  int lpos[8];         // column bit b
  int nu;              // bits of the tile index (K + LB)
  uint32_t lw[13];     // LDS offset (in amplitudes) of tile-index bit b
  uint64_t gw[13];     // global offset (in amplitudes) of tile-index bit b
};

template <int K>
__device__ __forceinline__ uint64_t lds_dep_rows(uint32_t m, const LdsTileArgs& a) {
  uint64_t i = 0;
#pragma unroll
  for (int j = 0; j < K; ++j) i |= (uint64_t)((m >> j) & 1u) << a.tpos[j];
  return i;
}

template <typename R, int K, int LB, bool NT>
__global__ __launch_bounds__(256) void k_dense_lds(typename MF<R>::V* psi, const typename MF<R>::V* __restrict__ mat,
                                                   uint64_t ntiles, Special sp, uint64_t cmask, LdsTileArgs ta,
                                                   CondArgs cond, bool xcd) {
  using V = typename MF<R>::V;
  using Acc = typename MF<R>::Acc;
  constexpr int DIM = 1 << K;
  constexpr int CW = 1 << LB;
  constexpr int S = CW + 1;                   // LDS row stride of the tile (amplitudes)
  constexpr int SA = DIM + 1;                 // LDS row stride of the matrix
  constexpr int RT = (2 * DIM + 15) / 16;
  constexpr int KS = DIM / 4;
  constexpr int GW = CW / 64;                 // 16-column groups per wave
  constexpr int VEC = 16 / (int)sizeof(V);    // amplitudes per 16-byte access (1 or 2)
  constexpr int E = DIM * CW;                 // amplitudes per tile
  constexpr int NA = E / (256 * VEC);         // accesses per thread per tile
  static_assert(K >= 3 && GW >= 1 && NA >= 1, "tile too small for a 256-thread workgroup");
  using Q = typename std::conditional<VEC == 1, V, floatx4>::type;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  V* Am = reinterpret_cast<V*>(smem_raw);
  V* X = Am + DIM * SA;

  if (!conds_ok_m(cond)) return;

  for (int e = threadIdx.x; e < DIM * DIM; e += 256) Am[(e / DIM) * SA + (e % DIM)] = mat[e];

  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int h = lane >> 4, c = lane & 15;
  // A operand of lane (i = lane % 16, kk = lane / 16) for 16-row tile rt and
  // step ks: real-embedding row rho = 16 rt + p(i) (p orders D rows the way
  // the instruction returns them), complex row rho / 2 = 8 rt + p(i) / 2,
  // column 4 ks + kk; an even rho takes (Re, -Im), an odd one (Im, Re)
  const int pi_ = MF<R>::kRowsByReg ? (4 * (c & 3) + (c >> 2)) : c;
  const bool odd = pi_ & 1;
  const int arow = (pi_ >> 1) * SA + h;

  // this thread's part of the tile index: bits of VEC * threadIdx.x; the
  // remaining bits come from the access number a (j = VEC * (tid + 256 a) + v)
  uint32_t lofs_t = 0;
  uint64_t gofs_t = 0;
  {
    const uint32_t jt = (uint32_t)(VEC * threadIdx.x);
    for (int b = 0; b < ta.nu; ++b)
      if ((jt >> b) & 1u) {
        lofs_t += ta.lw[b];
        gofs_t += ta.gw[b];
      }
  }
  uint32_t lofs_a[NA];
  uint64_t gofs_a[NA];
#pragma unroll
  for (int a = 0; a < NA; ++a) {
    const uint32_t ja = (uint32_t)(VEC * 256 * a);
    uint32_t lo = 0;
    uint64_t go = 0;
    for (int b = 0; b < ta.nu; ++b)
      if ((ja >> b) & 1u) {
        lo += ta.lw[b];
        go += ta.gw[b];
      }
    lofs_a[a] = lo + lofs_t;
    gofs_a[a] = go + gofs_t;
  }
  const uint32_t lw0 = ta.lw[0];   // LDS offset of the second amplitude of a pair (VEC = 2)
  uint64_t blk = blockIdx.x;
  if (xcd && !(gridDim.x & 7)) blk = (blk & 7) * (gridDim.x >> 3) + (blk >> 3);
  const uint64_t nwg = gridDim.x;

  Q rg[NA];
  auto gload = [&](uint64_t base) {
#pragma unroll
    for (int a = 0; a < NA; ++a) rg[a] = mld<NT>(reinterpret_cast<const Q*>(psi + base + gofs_a[a]));
  };
  uint64_t t = blk;
  if (t >= ntiles) return;
  uint64_t base = insert_zeros_m(t, sp) | cmask;
  gload(base);
  for (;;) {
    // registers -> LDS
#pragma unroll
    for (int a = 0; a < NA; ++a) {
      if constexpr (VEC == 1) {
        X[lofs_a[a]] = rg[a];
      } else {
        V v0, v1;
        v0.x = rg[a].x;
        v0.y = rg[a].y;
        v1.x = rg[a].z;
        v1.y = rg[a].w;
        X[lofs_a[a]] = v0;
        X[lofs_a[a] + lw0] = v1;
      }
    }
    __syncthreads();   // (first pass: the matrix is staged too)
    const uint64_t tn = t + nwg;
    const bool more = tn < ntiles;
    const uint64_t nbase = more ? (insert_zeros_m(tn, sp) | cmask) : base;
    if (more) gload(nbase);
    // compute this wave's columns
    Acc acc[RT][GW];
#pragma unroll
    for (int rt = 0; rt < RT; ++rt)
#pragma unroll
      for (int g = 0; g < GW; ++g) acc[rt][g] = Acc{0, 0, 0, 0};
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
      V xb[GW];
#pragma unroll
      for (int g = 0; g < GW; ++g) xb[g] = X[(4 * ks + h) * S + 16 * (wv * GW + g) + c];
#pragma unroll
      for (int rt = 0; rt < RT; ++rt) {
        const V z = Am[arow + 8 * rt * SA + 4 * ks];
        const R a0 = odd ? z.y : z.x;
        const R a1 = odd ? z.x : -z.y;
#pragma unroll
        for (int g = 0; g < GW; ++g) {
          acc[rt][g] = MF<R>::op(a0, xb[g].x, acc[rt][g]);
          acc[rt][g] = MF<R>::op(a1, xb[g].y, acc[rt][g]);
        }
      }
    }
    {
#pragma unroll
      for (int rt = 0; rt < RT; ++rt) {
        const int r0 = 8 * rt + 2 * h;
        if (r0 < DIM) {
#pragma unroll
          for (int g = 0; g < GW; ++g) {
            const int col = 16 * (wv * GW + g) + c;
            V v0, v1;
            v0.x = acc[rt][g][0];
            v0.y = acc[rt][g][1];
            v1.x = acc[rt][g][2];
            v1.y = acc[rt][g][3];
            X[r0 * S + col] = v0;
            X[(r0 + 1) * S + col] = v1;
          }
        }
      }
      __syncthreads();
      // LDS -> global, address order
#pragma unroll
      for (int a = 0; a < NA; ++a) {
        Q q;
        if constexpr (VEC == 1) {
          q = X[lofs_a[a]];
        } else {
          const V v0 = X[lofs_a[a]], v1 = X[lofs_a[a] + lw0];
          q = floatx4{v0.x, v0.y, v1.x, v1.y};
        }
        mst<NT>(reinterpret_cast<Q*>(psi + base + gofs_a[a]), q);
      }
      if (!more) break;
      __syncthreads();   // every store has read X before the next tile overwrites it
    }
    t = tn;
    base = nbase;
  }
}

template <typename R, int K, int LB, bool NT>
static hipError_t launch_lds_k(const Launch& L, const void* mat, uint64_t ntiles, const Special& sp, uint64_t cmask,
                               const LdsTileArgs& ta, int wg_per_cu) {
  constexpr int DIM = 1 << K;
  constexpr size_t shm = ((size_t)DIM * (DIM + 1) + (size_t)DIM * ((1 << LB) + 1)) * 2 * sizeof(R);
  static bool attr_set = false;
  if (!attr_set) {
    hipError_t e = hipFuncSetAttribute((const void*)k_dense_lds<R, K, LB, NT>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
    if (e != hipSuccess) return e;
    attr_set = true;
  }
  if (g_ncu <= 0) {
    int dev = 0, v = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && v > 0)
      g_ncu = v;
    else
      g_ncu = 256;
  }
  const uint64_t cap = (uint64_t)g_ncu * (uint64_t)std::max(1, wg_per_cu);
  const unsigned g = (unsigned)std::max<uint64_t>(1, std::min<uint64_t>(ntiles, cap));
  hipLaunchKernelGGL((k_dense_lds<R, K, LB, NT>), dim3(g), dim3(256), shm, L.stream, (typename MF<R>::V*)L.psi,
                     (const typename MF<R>::V*)mat, ntiles, sp, cmask, ta, L.cond, L.tune.xcd != 0);
  return hipGetLastError();
}

template <typename R, int K, int LB>
static hipError_t launch_lds_kn(const Launch& L, const void* mat, uint64_t ntiles, const Special& sp, uint64_t cmask,
                                const LdsTileArgs& ta, int wg_per_cu, bool nt) {
  return nt ? launch_lds_k<R, K, LB, true>(L, mat, ntiles, sp, cmask, ta, wg_per_cu)
            : launch_lds_k<R, K, LB, false>(L, mat, ntiles, sp, cmask, ta, wg_per_cu);
}

// Tile widths of the LDS-staged kernel: 64 columns (complex128) and 128
// (complex64), so that a tile is 2^K x 1 KiB.
static int lds_lb(bool c64) { return c64 ? 7 : 6; }

// Blocks of 4 or 5 qubits whose tile starts at bit 0 (no control on bit 0),
// with enough free bits for a tile row.
bool mfma_lds_supported(int n, int k, const int* controls, int nc, bool c64) {
  for (int j = 0; j < nc; ++j)
    if (controls[j] == 0) return false;
  return (k == 4 || k == 5) && n - k - nc >= lds_lb(c64);
}

// The automatic choice (tuning value 2), from 30-qubit timings of both
// kernels over low, scattered and high target sets: 4-qubit blocks gain
// 2-33 % from LDS tiles (most where targets sit on the lowest bits, whose
// register tiles then load short pieces); 5-qubit blocks gain only for
// complex64 blocks with three or more targets below bit 5 (4.4 -> 3.5 ms on
// bits 0-4) and are otherwise 0-10 % slower, so they keep register tiles.
bool mfma_lds_auto(int k, const int* targets, bool c64) {
  if (k == 4) return true;
  int low = 0;
  for (int j = 0; j < k; ++j) low += targets[j] < 5;
  return k == 5 && c64 && low >= 3;
}

hipError_t launch_dense_lds(const Launch& L, const int* targets, int k, const int* controls, int nc,
                            const void* d_matrix, int wg_per_cu) {
  if (!mfma_lds_supported(L.n, k, controls, nc, L.c64)) return hipErrorInvalidValue;
  const int lb = lds_lb(L.c64);
  const int CW = 1 << lb;
  uint64_t used = 0;
  for (int j = 0; j < k; ++j) used |= 1ull << targets[j];
  for (int j = 0; j < nc; ++j) used |= 1ull << controls[j];
  LdsTileArgs ta{};
  int nl = 0;
  for (int b = 0; b < L.n && nl < lb; ++b)
    if (!((used >> b) & 1)) ta.lpos[nl++] = b;
  // tile index bits: targets and column bits in ascending bit order
  std::vector<int> ubits(targets, targets + k);
  for (int j = 0; j < lb; ++j) ubits.push_back(ta.lpos[j]);
  std::sort(ubits.begin(), ubits.end());
  ta.nu = (int)ubits.size();
  for (int j = 0; j < k; ++j) ta.tpos[j] = targets[j];
  for (int b = 0; b < ta.nu; ++b) {
    const int bit = ubits[b];
    ta.gw[b] = 1ull << bit;
    uint32_t w = 0;
    for (int j = 0; j < k; ++j)
      if (targets[j] == bit) w = (uint32_t)(1u << j) * (uint32_t)(CW + 1);   // row m bit j
    for (int j = 0; j < lb; ++j)
      if (ta.lpos[j] == bit) w = 1u << j;                                     // column bit j
    ta.lw[b] = w;
  }
  // runs of the tile start at bit 0 (a 16-byte access covers two complex64 amplitudes)
  if (ubits[0] != 0) return hipErrorInvalidValue;
  std::vector<int> sv(targets, targets + k);
  for (int j = 0; j < nc; ++j) sv.push_back(controls[j]);
  for (int j = 0; j < lb; ++j) sv.push_back(ta.lpos[j]);
  Special sp = make_special(sv.data(), (int)sv.size(), nullptr, 0);
  uint64_t cmask = 0;
  for (int j = 0; j < nc; ++j) cmask |= 1ull << controls[j];
  const uint64_t ntiles = 1ull << (L.n - k - nc - lb);
  if (wg_per_cu <= 0) wg_per_cu = 2;
  const bool nt = L.tune.nt == 2 || (L.tune.nt == 1 && state_streams(L));
  if (L.c64) {
    if (k == 4) return launch_lds_kn<float, 4, 7>(L, d_matrix, ntiles, sp, cmask, ta, wg_per_cu, nt);
    return launch_lds_kn<float, 5, 7>(L, d_matrix, ntiles, sp, cmask, ta, wg_per_cu, nt);
  }
  if (k == 4) return launch_lds_kn<double, 4, 6>(L, d_matrix, ntiles, sp, cmask, ta, wg_per_cu, nt);
  return launch_lds_kn<double, 5, 6>(L, d_matrix, ntiles, sp, cmask, ta, wg_per_cu, nt);
}

// Widest tile (columns per wave) that is instantiated for this block size
// and keeps the double-buffered B registers of a lane at or below 64 VGPRs:
// 64 columns up to k = 4; 32 up to k = 5, and at k = 6 for complex64; else 16.
// launch_kwa dispatches exactly these widths.
static int max_cols(int k, bool c64) {
  if (k <= 4) return 64;
  if (k == 5 || c64) return 32;
  return 16;
}

bool mfma_supported(int n, int k, int nc, bool c64) {
  (void)c64;
  return k >= 2 && k <= 6 && n - k - nc >= 4;
}

template <typename R, int K, int CW, bool NT, bool AREG>
static hipError_t launch_k(const Launch& L, const void* mat, uint64_t nchunks, const Special& sp, uint64_t cmask,
                           const MfmaArgs& ma, int waves_per_cu) {
  constexpr int DIM = 1 << K;
  constexpr int RT = (2 * DIM + 15) / 16;
  constexpr int KS = DIM / 4;
  const size_t shm = (size_t)RT * KS * 2 * 64 * sizeof(R);
  static bool attr_set = false;
  if (!attr_set) {
    hipError_t e = hipFuncSetAttribute((const void*)k_dense_mfma<R, K, CW, NT, AREG>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
    if (e != hipSuccess) return e;
    attr_set = true;
  }
  if (g_ncu <= 0) {
    int dev = 0, v = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && v > 0)
      g_ncu = v;
    else
      g_ncu = 256;
  }
  const uint64_t want = (nchunks + 3) / 4;
  const uint64_t cap = (uint64_t)g_ncu * std::max(1, waves_per_cu / 4);
  const unsigned g = (unsigned)std::max<uint64_t>(1, std::min(want, cap));
  hipLaunchKernelGGL((k_dense_mfma<R, K, CW, NT, AREG>), dim3(g), dim3(256), shm, L.stream, (typename MF<R>::V*)L.psi,
                     (const typename MF<R>::V*)mat, nchunks, sp, cmask, ma, L.cond, L.tune.xcd != 0);
  return hipGetLastError();
}

template <typename R, int K, bool AREG>
static hipError_t launch_kwa(const Launch& L, const void* mat, int cw, bool nt, uint64_t nchunks, const Special& sp,
                             uint64_t cmask, const MfmaArgs& ma, int waves) {
  if (cw == 64) {
    if constexpr (K <= 4) {
      return nt ? launch_k<R, K, 64, true, AREG>(L, mat, nchunks, sp, cmask, ma, waves)
                : launch_k<R, K, 64, false, AREG>(L, mat, nchunks, sp, cmask, ma, waves);
    }
    return hipErrorInvalidValue;   // the host laid out chunks for a width this block size does not have
  }
  if (cw == 32) {
    if constexpr (K <= 5 || std::is_same<R, float>::value) {
      return nt ? launch_k<R, K, 32, true, AREG>(L, mat, nchunks, sp, cmask, ma, waves)
                : launch_k<R, K, 32, false, AREG>(L, mat, nchunks, sp, cmask, ma, waves);
    }
    return hipErrorInvalidValue;
  }
  if (cw != 16) return hipErrorInvalidValue;
  return nt ? launch_k<R, K, 16, true, AREG>(L, mat, nchunks, sp, cmask, ma, waves)
            : launch_k<R, K, 16, false, AREG>(L, mat, nchunks, sp, cmask, ma, waves);
}

// Blocks up to k = 4 keep their (at most 16) A values in registers; larger
// blocks choose by the "mfma_areg" knob, except complex128 k = 6, whose 256
// A values would not fit beside the tile (the registers would spill to
// scratch memory), so it always re-reads them from LDS.
template <typename R, int K>
static hipError_t launch_kw(const Launch& L, const void* mat, int cw, bool nt, uint64_t nchunks, const Special& sp,
                            uint64_t cmask, const MfmaArgs& ma, int waves) {
  if constexpr (K <= 4) {
    return launch_kwa<R, K, true>(L, mat, cw, nt, nchunks, sp, cmask, ma, waves);
  } else if constexpr (K == 6 && std::is_same<R, double>::value) {
    return launch_kwa<R, K, false>(L, mat, cw, nt, nchunks, sp, cmask, ma, waves);
  } else {
    if (L.tune.mfma_areg) return launch_kwa<R, K, true>(L, mat, cw, nt, nchunks, sp, cmask, ma, waves);
    return launch_kwa<R, K, false>(L, mat, cw, nt, nchunks, sp, cmask, ma, waves);
  }
}

hipError_t launch_dense_mfma(const Launch& L, const int* targets, int k, const int* controls, int nc,
                             const void* d_matrix, int waves_per_cu) {
  if (!mfma_supported(L.n, k, nc, L.c64)) return hipErrorInvalidValue;
  // tile width: the tuned one, capped by registers and by the bits available
  int cw = std::max(16, std::min(L.tune.mfma_cols, max_cols(k, L.c64)));
  while (cw > 16 && (1ull << (L.n - k - nc)) < (uint64_t)cw) cw >>= 1;
  const int lb = cw == 16 ? 4 : (cw == 32 ? 5 : 6);
  MfmaArgs ma{};
  uint64_t used = 0;
  for (int j = 0; j < k; ++j) {
    ma.tpos[j] = targets[j];
    used |= 1ull << targets[j];
  }
  for (int j = 0; j < nc; ++j) used |= 1ull << controls[j];
  int nl = 0;
  for (int b = 0; b < L.n && nl < lb; ++b)
    if (!((used >> b) & 1)) ma.lpos[nl++] = b;
  std::vector<int> sv(targets, targets + k);
  for (int j = 0; j < nc; ++j) sv.push_back(controls[j]);
  for (int j = 0; j < lb; ++j) sv.push_back(ma.lpos[j]);
  Special sp = make_special(sv.data(), (int)sv.size(), nullptr, 0);
  uint64_t cmask = 0;
  for (int j = 0; j < nc; ++j) cmask |= 1ull << controls[j];
  const uint64_t nchunks = 1ull << (L.n - k - nc - lb);
  if (waves_per_cu <= 0) waves_per_cu = 8;
  // non-temporal when every row run of the tile is at least 256 bytes: the
  // column bits are then the lowest ones and the run is CW amplitudes long
  bool contiguous = true;
  for (int j = 0; j < lb; ++j) contiguous = contiguous && ma.lpos[j] == j;
  const size_t run = (contiguous ? (size_t)cw : 1) * (L.c64 ? 8 : 16);
  const bool nt = L.tune.nt == 2 || (L.tune.nt == 1 && run >= 256 && state_streams(L));
  if (L.c64) {
    switch (k) {
      case 2: return launch_kw<float, 2>(L, d_matrix, cw, nt, nchunks, sp, cmask, ma, waves_per_cu);
      case 3: return launch_kw<float, 3>(L, d_matrix, cw, nt, nchunks, sp, cmask, ma, waves_per_cu);
      case 4: return launch_kw<float, 4>(L, d_matrix, cw, nt, nchunks, sp, cmask, ma, waves_per_cu);
      case 5: return launch_kw<float, 5>(L, d_matrix, cw, nt, nchunks, sp, cmask, ma, waves_per_cu);
      case 6: return launch_kw<float, 6>(L, d_matrix, cw, nt, nchunks, sp, cmask, ma, waves_per_cu);
    }
  } else {
    switch (k) {
      case 2: return launch_kw<double, 2>(L, d_matrix, cw, nt, nchunks, sp, cmask, ma, waves_per_cu);
      case 3: return launch_kw<double, 3>(L, d_matrix, cw, nt, nchunks, sp, cmask, ma, waves_per_cu);
      case 4: return launch_kw<double, 4>(L, d_matrix, cw, nt, nchunks, sp, cmask, ma, waves_per_cu);
      case 5: return launch_kw<double, 5>(L, d_matrix, cw, nt, nchunks, sp, cmask, ma, waves_per_cu);
      case 6: return launch_kw<double, 6>(L, d_matrix, cw, nt, nchunks, sp, cmask, ma, waves_per_cu);
    }
  }
  return hipErrorInvalidValue;
}

}  // namespace qk
