// Host runtime behind the C ABI (qk.h): simulator registry, classical bits,
// gate table and validation, per-gate dispatch to the sweep kernels, fusion,
// measurement and readout.  Host-side checks run before any HIP call, so
// argument errors are reported even where no GPU is present.
#include <algorithm>
#include <cctype>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "qk_internal.h"

using namespace qk;

namespace {

struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
};

enum UKind { U_MATRIX = 0, U_TABLE = 1, U_AFFINE = 2, U_MODMUL = 3 };

struct UserGate {
  int kind = U_MATRIX;
  int k = 1;
  std::string name;
  std::vector<cd> m;       // FP64 matrix (U_MATRIX)
  bool diag = false;
  DevBuf dmat;             // matrix in the state's precision (uploaded at define time)
  DevBuf finv;             // inverse table, uint32 (U_TABLE)
  DevBuf ftab;             // forward table, uint32 (U_TABLE; the sparse engine maps indices forward)
  uint64_t a = 1, b = 0;   // U_AFFINE; U_MODMUL: multiplier a, modulus b
};

// Gate description after classification.
enum DKind { D_BUTTERFLY, D_DIAG, D_PHASE1, D_SWAP, D_DENSE, D_PERM };

struct GateDesc {
  int kind = D_DENSE;
  std::vector<int> targets, controls;
  std::vector<qk_cond> conds;
  std::vector<cd> m;         // dense matrix (2^k x 2^k) for D_BUTTERFLY / D_DENSE, or diagonal for D_DIAG
  cd z = 1.0;                // D_PHASE1 factor
  const UserGate* ug = nullptr;
  uint64_t A = 1, B = 0, Ainv = 1, N = 0;   // D_PERM closed forms (affine power; modular multiplier)
  bool fusable = false;      // matrix gate without conditions
};

// Append-only constant arena (device + pinned host staging).  Reset only after
// the stream has drained, so staged host bytes are never overwritten while a
// copy from them may still be pending.
struct Arena {
  void* dev = nullptr;
  void* host = nullptr;
  size_t cap = 0;
  size_t used = 0;
};

std::string g_last_error;

}  // namespace

struct qk_sim_s {
  qk_dtype dtype = QK_C128;
  bool c64 = false;
  size_t amp = 16;
  qk_allocator alloc{};
  bool has_alloc = false;
  hipStream_t stream = nullptr;
  int n = 0;
  DevBuf state, scratch, cbits, meas;
  DevBuf samp, shots;               // deferred-measurement work space; host-call staging of uniforms and shots
  bool sparse = false;              // state kept as sorted (index, amplitude) entries
  SpBufs sp;
  SpDiagRun sp_run{};               // diagonal gates held back to be applied in one pass
  std::vector<int> sp_phys;         // logical qubit -> index bit (a SWAP exchanges two entries, no data moves)
  std::vector<int> dphys;           // the same for a dense state (identity until an uncontrolled SWAP relabels)
  int ncbits = 0;
  std::vector<Arena> arenas;        // constant chunks in use (the last one is being filled)
  std::vector<Arena> saved_arenas;  // chunks set aside while a capture owns `arenas`
  bool capturing = false;
  std::vector<UserGate*> ugates;
  int fuse_k = 0;
  std::vector<GateDesc> pending;
  std::vector<qk_op> stage_q;       // builtin gates held back for the LDS-tile mode (physical qubits; never beside
                                    // `pending` or `drun`)
  std::vector<GateDesc> drun;       // diagonal gates held back for one combined pass (never beside `pending`)
  std::vector<uint64_t> drun_groups;  // their factor-table groups in gate order (the fit check when adding)
  int drun_conds = 0;               // classical conditions they carry
  Tuning tune;
  int64_t sweeps = 0, fused_blocks = 0, fused_gates = 0;
  std::string err;
  qk_status latched = QK_OK;
};

namespace {

constexpr int kUserBase = 0x100;
constexpr size_t kArenaBytes = 32u << 20;
constexpr int kMaxQubits = 40;
constexpr int kMaxSparseQubits = 62;    // indices and the sort's sentinel bit fit 64 bits
constexpr uint64_t kSpMergeMin = 1u << 12;   // entries from which one-qubit gates merge instead of sorting
constexpr size_t kStageQueueMax = 8192;      // held-back gates of the LDS-tile mode (about 0.7 MB of records)

qk_status fail(qk_sim s, qk_status st, const std::string& msg) {
  if (s) s->err = msg;
  else g_last_error = msg;
  return st;
}

qk_status hip_fail(qk_sim s, hipError_t e, const char* what) {
  return fail(s, QK_E_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

void* dev_alloc(qk_sim s, size_t bytes) {
  if (bytes == 0) bytes = 256;
  if (s->has_alloc) return s->alloc.alloc(bytes, (void*)s->stream, s->alloc.ctx);
  void* p = nullptr;
  if (hipMalloc(&p, bytes) != hipSuccess) {
    (void)hipGetLastError();
    return nullptr;
  }
  return p;
}

void dev_free(qk_sim s, DevBuf& b) {
  if (!b.p) return;
  if (s->has_alloc) s->alloc.free(b.p, b.bytes, (void*)s->stream, s->alloc.ctx);
  else (void)hipFree(b.p);
  b.p = nullptr;
  b.bytes = 0;
}

qk_status ensure(qk_sim s, DevBuf& b, size_t bytes, const char* what) {
  if (b.p && b.bytes >= bytes) return QK_OK;
  dev_free(s, b);
  b.p = dev_alloc(s, bytes);
  if (!b.p) return fail(s, QK_E_OOM, std::string("device allocation failed: ") + what);
  b.bytes = bytes;
  return QK_OK;
}

// ---- small device helpers (graph-safe: kernels, never memset) -----------------

__global__ void k_u8_fill(uint8_t* p, size_t from, size_t to, uint8_t v) {
  for (size_t i = from + (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < to; i += (size_t)gridDim.x * blockDim.x)
    p[i] = v;
}
__global__ void k_u8_copy(uint8_t* dst, const uint8_t* src, size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    dst[i] = src[i];
}
__global__ void k_u32_zero(uint32_t* p) {
  if (threadIdx.x == 0) *p = 0;
}

// Measurement buffer layout (doubles): partials[2*kReduceBlocks] | result[4] |
// log[3*kMeasLog] | log_count (uint32, in the last 8 bytes).
constexpr size_t kMeasDoubles = 2 * kReduceBlocks + 4 + 3 * kMeasLog + 1;
// The diagonal-run tables follow, 16-byte aligned.
constexpr size_t kRunTableOffset = ((kMeasDoubles * sizeof(double) + 15) / 16) * 16;

MeasBuffers meas_buffers(qk_sim s) {
  double* d = (double*)s->meas.p;
  MeasBuffers mb;
  mb.partials = d;
  mb.result = d + 2 * kReduceBlocks;
  mb.log = mb.result + 4;
  mb.log_count = (uint32_t*)(mb.log + 3 * kMeasLog);
  mb.cbits = (uint8_t*)s->cbits.p;
  return mb;
}

qk_status ensure_meas(qk_sim s) {
  if (s->meas.p) return QK_OK;
  qk_status st = ensure(s, s->meas, kRunTableOffset + kDiagRunTableBytes, "measurement buffers");
  if (st) return st;
  MeasBuffers mb = meas_buffers(s);
  hipLaunchKernelGGL(k_u32_zero, dim3(1), dim3(64), 0, s->stream, mb.log_count);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? QK_OK : hip_fail(s, e, "measurement buffer init");
}

// ---- constant arena ----------------------------------------------------------

// Pinned staging chunks are pooled for the life of the process and shared by
// every simulator: pinning and unpinning 32 MiB per simulator cost
// milliseconds each (up to 100 ms to unpin; 5 s of host time over 2000
// short-lived simulators in a serving loop that creates one per job).  A chunk
// goes back to the pool only once no copy from it can be pending (its
// simulator's stream has drained, or the capture that staged into it never
// ran), so the next owner may overwrite it at once.
constexpr size_t kPinnedPoolMax = 16;
std::mutex g_pinned_mu;
std::vector<void*> g_pinned_free;

void* pinned_take() {
  {
    std::lock_guard<std::mutex> lk(g_pinned_mu);
    if (!g_pinned_free.empty()) {
      void* p = g_pinned_free.back();
      g_pinned_free.pop_back();
      return p;
    }
  }
  void* p = nullptr;
  if (hipHostMalloc(&p, kArenaBytes, hipHostMallocDefault) != hipSuccess) {
    (void)hipGetLastError();
    return nullptr;
  }
  return p;
}

void pinned_give(void* p) {
  {
    std::lock_guard<std::mutex> lk(g_pinned_mu);
    if (g_pinned_free.size() < kPinnedPoolMax) {
      g_pinned_free.push_back(p);
      return;
    }
  }
  (void)hipHostFree(p);
}

qk_status arena_new_chunk(qk_sim s) {
  Arena a;
  a.dev = dev_alloc(s, kArenaBytes);
  if (!a.dev) return fail(s, QK_E_OOM, "device allocation failed: constant arena");
  a.host = pinned_take();
  if (!a.host) {
    DevBuf b{a.dev, kArenaBytes};
    dev_free(s, b);
    return fail(s, QK_E_OOM, "pinned host allocation failed: constant arena");
  }
  a.cap = kArenaBytes;
  a.used = 0;
  s->arenas.push_back(a);
  return QK_OK;
}

void arena_free_chunk(qk_sim s, Arena& a) {
  if (a.dev) {
    DevBuf b{a.dev, a.cap};
    dev_free(s, b);
  }
  if (a.host) pinned_give(a.host);
  a = Arena{};
}

// Outside a capture a full arena is recycled after the stream drains (so no
// pending copy still reads the staged bytes); inside a capture the graph will
// replay the copies, so every staged byte must survive: a new chunk is added.
qk_status arena_put(qk_sim s, const void* data, size_t bytes, const void** dptr) {
  const size_t need = (bytes + 255) & ~(size_t)255;
  if (need > kArenaBytes) return fail(s, QK_E_ARG, "constant block larger than the arena");
  qk_status st;
  if (s->arenas.empty() && (st = arena_new_chunk(s))) return st;
  if (s->arenas.back().used + need > s->arenas.back().cap) {
    if (s->capturing) {
      if ((st = arena_new_chunk(s))) return st;
    } else {
      hipError_t e = hipStreamSynchronize(s->stream);
      if (e != hipSuccess) return hip_fail(s, e, "arena recycle");
      while (s->arenas.size() > 1) {
        arena_free_chunk(s, s->arenas.back());
        s->arenas.pop_back();
      }
      s->arenas[0].used = 0;
    }
  }
  Arena& a = s->arenas.back();
  std::memcpy((char*)a.host + a.used, data, bytes);
  hipError_t e = hipMemcpyAsync((char*)a.dev + a.used, (char*)a.host + a.used, bytes, hipMemcpyHostToDevice, s->stream);
  if (e != hipSuccess) return hip_fail(s, e, "constant upload");
  *dptr = (char*)a.dev + a.used;
  a.used += need;
  return QK_OK;
}

// Matrix in the state's precision, row-major interleaved.
std::vector<unsigned char> pack_matrix(const std::vector<cd>& m, bool c64) {
  std::vector<unsigned char> out(m.size() * (c64 ? 8 : 16));
  if (c64) {
    float* f = (float*)out.data();
    for (size_t i = 0; i < m.size(); ++i) {
      f[2 * i] = (float)m[i].real();
      f[2 * i + 1] = (float)m[i].imag();
    }
  } else {
    double* f = (double*)out.data();
    for (size_t i = 0; i < m.size(); ++i) {
      f[2 * i] = m[i].real();
      f[2 * i + 1] = m[i].imag();
    }
  }
  return out;
}

// ---- builtin gates (FP64 definitions) -------------------------------------------

struct BuiltinInfo {
  const char* name;
  int id;
  int arity;
  int nparams;
};
const BuiltinInfo kBuiltins[] = {
    {"H", QK_H, 1, 0},         {"HADAMARD", QK_H, 1, 0}, {"X", QK_X, 1, 0},       {"SIGMAX", QK_X, 1, 0},
    {"NOT", QK_X, 1, 0},       {"CNOT", QK_X, 1, 0},     {"Y", QK_Y, 1, 0},       {"SIGMAY", QK_Y, 1, 0},
    {"Z", QK_Z, 1, 0},         {"SIGMAZ", QK_Z, 1, 0},   {"S", QK_S, 1, 0},       {"T", QK_T, 1, 0},
    {"SDG", QK_SDG, 1, 0},     {"TDG", QK_TDG, 1, 0},    {"RX", QK_RX, 1, 1},     {"RY", QK_RY, 1, 1},
    {"RZ", QK_RZ, 1, 1},       {"PHASE", QK_PHASE, 1, 1}, {"RPHASE", QK_PHASE, 1, 1}, {"CPHASE", QK_CPHASE, 2, 1},
    {"SWAP", QK_SWAP, 2, 0},   {"RZZ", QK_RZZ, 2, 1},
};

const BuiltinInfo* builtin_by_id(int id) {
  for (const auto& b : kBuiltins)
    if (b.id == id) return &b;
  return nullptr;
}

}  // namespace

namespace qk {

bool builtin_info(int id, int* arity, int* nparams) {
  const BuiltinInfo* b = builtin_by_id(id);
  if (!b) return false;
  if (arity) *arity = b->arity;
  if (nparams) *nparams = b->nparams;
  return true;
}

// Builtin gate data in FP64, following the definitions in qk.h.
BuiltinGate builtin_gate(int id, double p) {
  const double s2 = 1.0 / std::sqrt(2.0);
  const cd i1(0, 1);
  const double c = std::cos(p / 2), sn = std::sin(p / 2);
  BuiltinGate g;
  switch (id) {
    case QK_H: g.cls = BG_DENSE1; g.m = {s2, s2, s2, -s2}; break;
    case QK_X: g.cls = BG_DENSE1; g.m = {0.0, 1.0, 1.0, 0.0}; break;
    case QK_Y: g.cls = BG_DENSE1; g.m = {0.0, -i1, i1, 0.0}; break;
    case QK_RX: g.cls = BG_DENSE1; g.m = {c, -i1 * sn, -i1 * sn, c}; break;
    case QK_RY: g.cls = BG_DENSE1; g.m = {c, -sn, sn, c}; break;
    case QK_Z: g.cls = BG_PHASE; g.z = -1.0; break;
    case QK_S: g.cls = BG_PHASE; g.z = i1; break;
    case QK_SDG: g.cls = BG_PHASE; g.z = -i1; break;
    case QK_T: g.cls = BG_PHASE; g.z = std::polar(1.0, M_PI / 4); break;
    case QK_TDG: g.cls = BG_PHASE; g.z = std::polar(1.0, -M_PI / 4); break;
    case QK_PHASE: g.cls = BG_PHASE; g.z = std::polar(1.0, p); break;
    case QK_CPHASE: g.cls = BG_PHASE; g.z = std::polar(1.0, p); break;
    case QK_RZ: g.cls = BG_DIAG; g.m = {std::polar(1.0, -p / 2), std::polar(1.0, p / 2)}; break;
    case QK_RZZ: {
      const cd em = std::polar(1.0, -p / 2), ep = std::polar(1.0, p / 2);
      g.cls = BG_DIAG;
      g.m = {em, ep, ep, em};
      break;
    }
    case QK_SWAP: g.cls = BG_SWAP; break;
  }
  return g;
}

}  // namespace qk

namespace {

// Classify a builtin gate into a sweep.
void builtin_desc(int id, double p, GateDesc& d) {
  const BuiltinGate g = builtin_gate(id, p);
  d.fusable = true;
  switch (g.cls) {
    case BG_DENSE1: d.kind = D_BUTTERFLY; d.m = g.m; break;
    case BG_PHASE: d.kind = D_PHASE1; d.z = g.z; break;
    case BG_DIAG: d.kind = D_DIAG; d.m = g.m; break;
    case BG_SWAP: d.kind = D_SWAP; break;
  }
}

// Full 2^k x 2^k matrix on the targets of a matrix-like description.
std::vector<cd> full_matrix(const GateDesc& d) {
  const int k = (int)d.targets.size();
  const int D = 1 << k;
  std::vector<cd> m((size_t)D * D, cd(0, 0));
  switch (d.kind) {
    case D_BUTTERFLY:
    case D_DENSE: return d.m;
    case D_DIAG:
      for (int i = 0; i < D; ++i) m[(size_t)i * D + i] = d.m[i];
      return m;
    case D_PHASE1:
      for (int i = 0; i < D; ++i) m[(size_t)i * D + i] = (i == D - 1) ? d.z : cd(1.0);
      return m;
    case D_SWAP:
      m[0] = 1.0;
      m[1 * 4 + 2] = 1.0;
      m[2 * 4 + 1] = 1.0;
      m[15] = 1.0;
      return m;
  }
  return m;
}

CondArgs make_cond(qk_sim s, const std::vector<qk_cond>& conds) {
  CondArgs c{};
  c.cbits = (const uint8_t*)s->cbits.p;
  c.n = (int)conds.size();
  for (int i = 0; i < c.n; ++i) {
    c.cbit[i] = conds[i].cbit;
    c.val[i] = conds[i].value;
  }
  return c;
}

// Dense states: index bit of a logical qubit, and whether the layout is the
// logical one.
int dbit(qk_sim s, int q) { return q < (int)s->dphys.size() ? s->dphys[q] : q; }
bool dense_identity(qk_sim s) {
  for (int q = 0; q < (int)s->dphys.size(); ++q)
    if (s->dphys[q] != q) return false;
  return true;
}

Launch make_launch(qk_sim s, const std::vector<qk_cond>& conds) {
  Launch L;
  L.stream = s->stream;
  L.n = s->n;
  L.c64 = s->c64;
  L.psi = s->state.p;
  L.cond = make_cond(s, conds);
  L.tune = s->tune;
  return L;
}

qk_status check_launch(qk_sim s, hipError_t e, const char* what) {
  if (e != hipSuccess) return hip_fail(s, e, what);
  s->sweeps++;
  return QK_OK;
}

// Dense matrix of any k (from a description or a fused block) on `targets`.
qk_status run_dense(qk_sim s, const std::vector<int>& targets, const std::vector<int>& controls,
                    const std::vector<qk_cond>& conds, const std::vector<cd>& m, const void* dmat_in) {
  const int k = (int)targets.size();
  Launch L = make_launch(s, conds);
  if (k == 1) {
    Mat2 u;
    for (int i = 0; i < 4; ++i) {
      u.v[2 * i] = m[i].real();
      u.v[2 * i + 1] = m[i].imag();
    }
    return check_launch(s, launch_butterfly(L, targets[0], controls.data(), (int)controls.size(), u), "butterfly");
  }
  const void* dmat = dmat_in;
  if (!dmat) {
    auto packed = pack_matrix(m, s->c64);
    qk_status st = arena_put(s, packed.data(), packed.size(), &dmat);
    if (st) return st;
  }
  const bool lds = s->tune.mfma_lds == 1 || (s->tune.mfma_lds == 2 && mfma_lds_auto(k, targets.data(), s->c64));
  if (lds && mfma_lds_supported(s->n, k, controls.data(), (int)controls.size(), s->c64))
    return check_launch(
        s, launch_dense_lds(L, targets.data(), k, controls.data(), (int)controls.size(), dmat, s->tune.lds_wg),
        "dense (matrix cores, LDS tiles)");
  if (mfma_supported(s->n, k, (int)controls.size(), s->c64))
    return check_launch(
        s, launch_dense_mfma(L, targets.data(), k, controls.data(), (int)controls.size(), dmat, s->tune.mfma_waves),
        "dense (matrix cores)");
  return check_launch(s, launch_dense_generic(L, targets.data(), k, controls.data(), (int)controls.size(), dmat),
                      "dense");
}

qk_status run_diag(qk_sim s, const std::vector<int>& targets, const std::vector<int>& controls,
                   const std::vector<qk_cond>& conds, const std::vector<cd>& diag) {
  const int k = (int)targets.size();
  // all ones except the last entry: only the all-ones subspace changes
  bool phase_only = true;
  for (int i = 0; i + 1 < (int)diag.size(); ++i)
    if (diag[i] != cd(1.0)) phase_only = false;
  Launch L = make_launch(s, conds);
  if (phase_only) {
    std::vector<int> bits(targets);
    bits.insert(bits.end(), controls.begin(), controls.end());
    return check_launch(s, launch_phase_all1(L, bits.data(), (int)bits.size(), diag.back().real(), diag.back().imag()),
                        "phase");
  }
  if (k > 6) {
    const int D = 1 << k;
    std::vector<cd> m((size_t)D * D, cd(0, 0));
    for (int i = 0; i < D; ++i) m[(size_t)i * D + i] = diag[i];
    return run_dense(s, targets, controls, conds, m, nullptr);
  }
  Diag64 d{};
  for (size_t i = 0; i < diag.size(); ++i) {
    d.v[2 * i] = diag[i].real();
    d.v[2 * i + 1] = diag[i].imag();
  }
  return check_launch(s, launch_diag(L, targets.data(), k, controls.data(), (int)controls.size(), d), "diagonal");
}

qk_status ensure_scratch(qk_sim s) {
  const size_t bytes = ((size_t)1 << s->n) * s->amp;
  return ensure(s, s->scratch, bytes, "permutation scratch");
}

qk_status execute(qk_sim s, const GateDesc& d) {
  switch (d.kind) {
    case D_BUTTERFLY:
    case D_DENSE:
      return run_dense(s, d.targets, d.controls, d.conds, d.m, d.ug ? d.ug->dmat.p : nullptr);
    case D_DIAG:
      return run_diag(s, d.targets, d.controls, d.conds, d.m);
    case D_PHASE1: {
      Launch L = make_launch(s, d.conds);
      std::vector<int> bits(d.targets);
      bits.insert(bits.end(), d.controls.begin(), d.controls.end());
      return check_launch(s, launch_phase_all1(L, bits.data(), (int)bits.size(), d.z.real(), d.z.imag()), "phase");
    }
    case D_SWAP: {
      Launch L = make_launch(s, d.conds);
      return check_launch(s, launch_swap(L, d.targets[0], d.targets[1], d.controls.data(), (int)d.controls.size()),
                          "swap");
    }
    case D_PERM: {
      qk_status st = ensure_scratch(s);
      if (st) return st;
      Launch L = make_launch(s, d.conds);
      const int mode = d.ug->kind == U_AFFINE ? 1 : (d.ug->kind == U_MODMUL ? 2 : 0);
      // without controls the gather writes the whole result into the second
      // buffer, which becomes the state (inside a capture the pointers the
      // graph records must stay put, so the state is gathered and copied back)
      const bool oop = d.controls.empty() && !s->capturing;
      st = check_launch(s,
                        launch_perm(L, s->scratch.p, d.targets.data(), (int)d.targets.size(), d.controls.data(),
                                    (int)d.controls.size(), mode == 0 ? (const uint32_t*)d.ug->finv.p : nullptr,
                                    mode, d.A, d.B, d.Ainv, d.N, oop),
                        "permutation");
      if (!st && oop) std::swap(s->state, s->scratch);
      return st;
    }
  }
  return fail(s, QK_E_ARG, "unknown gate class");
}

qk_status sp_flush_run(qk_sim s);

// Diagonal runs.  A diagonal gate on at most two targets (or a phase on the
// all-ones subspace of any qubit set) joins the run; any other operation first
// applies the run.  The run becomes one k_diag_run pass when that pass touches
// no more amplitudes than the gates would one by one; otherwise each gate gets
// its own sweep, as without runs.

bool phase_only_diag(const GateDesc& d) {
  for (size_t i = 0; i + 1 < d.m.size(); ++i)
    if (d.m[i] != cd(1.0)) return false;
  return true;
}

uint64_t bits_of(const std::vector<int>& a) {
  uint64_t m = 0;
  for (int q : a) m |= 1ull << q;
  return m;
}

// A term's qubit set (targets and controls) must fit one factor table.
bool joins_run(const GateDesc& d) {
  if (d.targets.size() + d.controls.size() > (size_t)kDiagRunGroupBits) return false;
  if (d.kind == D_PHASE1) return true;
  return d.kind == D_DIAG && (d.targets.size() <= 2 || phase_only_diag(d));
}

// Bits that must all be 1 for the term to act: the controls, and for a phase
// on the all-ones subspace the targets as well.
uint64_t run_mask(const GateDesc& d) {
  uint64_t m = bits_of(d.controls);
  if (d.kind == D_PHASE1 || phase_only_diag(d)) m |= bits_of(d.targets);
  return m;
}

// Greedy grouping of the terms' qubit sets (without the bits in `drop`, which
// are 1 wherever the pass acts): a term joins the first group whose bits stay
// within kDiagRunGroupBits, else opens a group.  The terms are visited in
// `order`.  Returns false when a term would need more than kDiagRunGroups
// groups.
bool group_terms(const std::vector<GateDesc>& run, uint64_t drop, const std::vector<int>& order,
                 std::vector<uint64_t>& groups, std::vector<int>& of) {
  groups.clear();
  of.assign(run.size(), 0);
  for (int i : order) {
    const GateDesc& d = run[i];
    const uint64_t sq = (bits_of(d.targets) | bits_of(d.controls)) & ~drop;
    int g = 0;
    while (g < (int)groups.size() && __builtin_popcountll(groups[g] | sq) > kDiagRunGroupBits) ++g;
    if (g == (int)groups.size()) {
      if (g == kDiagRunGroups) return false;
      groups.push_back(0);
    }
    groups[g] |= sq;
    of[i] = g;
  }
  return true;
}

std::vector<int> gate_order(size_t n) {
  std::vector<int> o(n);
  for (size_t i = 0; i < n; ++i) o[i] = (int)i;
  return o;
}

// Grouping for a pass: common bits left out, terms visited by their lowest
// remaining bit, so that terms on the low index bits (which differ between
// the lanes of a wave) share as few groups as possible and the other groups'
// table reads are the same for a whole wave.  Falls back to gate order, and
// finally to gate order with the common bits kept, which add_to_run has
// checked to fit (a common bit in a group only leaves half its table unused).
void group_for_pass(const std::vector<GateDesc>& run, uint64_t common, std::vector<uint64_t>& groups,
                    std::vector<int>& of) {
  std::vector<int> order = gate_order(run.size());
  auto low = [&](int i) {
    const uint64_t sq = (bits_of(run[i].targets) | bits_of(run[i].controls)) & ~common;
    return sq ? __builtin_ctzll(sq) : 64;
  };
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return low(a) < low(b); });
  if (group_terms(run, common, order, groups, of)) return;
  if (group_terms(run, common, gate_order(run.size()), groups, of)) return;
  group_terms(run, 0, gate_order(run.size()), groups, of);
}

// Rank of bit q among the set bits of u (its position in the group index).
int local_bit(uint64_t u, int q) { return __builtin_popcountll(u & ((1ull << q) - 1)); }

qk_status execute(qk_sim s, const GateDesc& d);

qk_status flush_drun(qk_sim s) {
  if (s->drun.empty()) return QK_OK;
  std::vector<GateDesc> run;
  run.swap(s->drun);
  s->drun_groups.clear();
  s->drun_conds = 0;
  std::vector<uint64_t> groups;
  std::vector<int> of;
  if (run.size() > 1) {
    // amplitudes touched: the run's pass vs the gates' own sweeps
    uint64_t common = ~0ull;
    double alone = 0;
    for (const GateDesc& d : run) {
      const uint64_t m = run_mask(d);
      common &= m;
      const bool phase = d.kind == D_PHASE1 || phase_only_diag(d);
      alone += std::ldexp(1.0, s->n - (phase ? __builtin_popcountll(m) : (int)d.controls.size()));
    }
    const int nc = __builtin_popcountll(common);
    if (std::ldexp(1.0, s->n - nc) <= alone) {
      group_for_pass(run, common, groups, of);
      DiagRunArgs a{};
      a.cbits = (const uint8_t*)s->cbits.p;
      a.n = (int)run.size();
      a.ng = (int)groups.size();
      for (int g = 0; g < a.ng; ++g) {
        int j = 0;
        for (int q = 0; q < 64; ++q)
          if ((groups[g] >> q) & 1) a.grp[g].pos[j++] = (int8_t)q;
        a.grp[g].nb = (int8_t)j;
      }
      int ncond = 0;
      for (int i = 0; i < a.n; ++i) {
        const GateDesc& d = run[i];
        DiagRunTerm& t = a.t[i];
        const uint64_t u = groups[of[i]];
        t.g = (uint8_t)of[i];
        const uint64_t m = run_mask(d) & ~common;   // common bits are 1 throughout the pass
        for (int q = 0; q < 64; ++q)
          if ((m >> q) & 1) t.lmask |= (uint8_t)(1u << local_bit(u, q));
        if (d.kind == D_PHASE1 || phase_only_diag(d)) {
          const cd z = d.kind == D_PHASE1 ? d.z : d.m.back();
          t.k = 0;
          t.d[0] = z.real();
          t.d[1] = z.imag();
        } else {
          t.k = (int8_t)d.targets.size();
          t.l0 = (int8_t)local_bit(u, d.targets[0]);
          t.l1 = (int8_t)(t.k > 1 ? local_bit(u, d.targets[1]) : 0);
          for (size_t e = 0; e < d.m.size(); ++e) {
            t.d[2 * e] = d.m[e].real();
            t.d[2 * e + 1] = d.m[e].imag();
          }
        }
        t.c0 = (uint8_t)ncond;
        for (const qk_cond& c : d.conds) {
          a.cb[ncond] = c.cbit;
          a.cv[ncond] = (uint8_t)c.value;
          ++ncond;
        }
        t.c1 = (uint8_t)ncond;
      }
      a.ncond = ncond;
      std::vector<int> cpos;
      for (int b = 0; b < 64; ++b)
        if ((common >> b) & 1) cpos.push_back(b);
      qk_status st = ensure_meas(s);   // the run's tables live after the measurement buffers
      if (st) return st;
      Launch L = make_launch(s, {});
      s->fused_blocks++;
      s->fused_gates += (int64_t)run.size();
      return check_launch(s, launch_diag_run(L, a, cpos.data(), (int)cpos.size(), (char*)s->meas.p + kRunTableOffset),
                          "diagonal run");
    }
  }
  for (const GateDesc& d : run) {
    qk_status st = execute(s, d);
    if (st) return st;
  }
  return QK_OK;
}

// The group a term with qubit set sq joins under the gate-order greedy rule
// of group_terms (an index past the end: a new group), or -1 when it would
// need more than kDiagRunGroups groups.
int fit_group(const std::vector<uint64_t>& groups, uint64_t sq) {
  int g = 0;
  while (g < (int)groups.size() && __builtin_popcountll(groups[g] | sq) > kDiagRunGroupBits) ++g;
  return g < kDiagRunGroups ? g : -1;
}

// Appends a diagonal gate to the run, applying the run first when the new
// gate would exceed its terms, conditions or factor-table groups.  The groups
// are kept in step with group_terms in gate order, so the check costs no copy.
qk_status add_to_run(qk_sim s, GateDesc&& d) {
  const uint64_t sq = bits_of(d.targets) | bits_of(d.controls);
  if ((int)s->drun.size() == kDiagRunTerms || s->drun_conds + (int)d.conds.size() > kDiagRunConds ||
      fit_group(s->drun_groups, sq) < 0) {
    qk_status st = flush_drun(s);
    if (st) return st;
  }
  const int g = fit_group(s->drun_groups, sq);   // an empty run always fits
  if (g == (int)s->drun_groups.size()) s->drun_groups.push_back(0);
  s->drun_groups[g] |= sq;
  s->drun_conds += (int)d.conds.size();
  s->drun.push_back(std::move(d));
  return QK_OK;
}

qk_status flush_pending(qk_sim s) {
  if (s->pending.empty()) return QK_OK;
  std::vector<GateDesc> pend;
  pend.swap(s->pending);
  std::vector<FGate> fg;
  fg.reserve(pend.size());
  for (const GateDesc& d : pend)
    fg.push_back(make_fgate(d.targets.data(), (int)d.targets.size(), d.controls.data(), (int)d.controls.size(),
                            full_matrix(d)));
  std::vector<FBlock> blocks = plan_blocks(fg, s->fuse_k);
  const std::vector<qk_cond> none;
  // With diagonal runs on, the gates of diagonal blocks (and diagonal gates
  // left alone) go into the run in plan order instead of a sweep each, so
  // consecutive ones share passes; the run is applied before any other
  // block, which keeps the plan's order.  The run may still be open when
  // this returns.  (Regrouping a stretch of them by a bit they share, for
  // passes over half the state, measured slower on the QFT: the stretches
  // between dense blocks are short, so it multiplied the passes.)
  auto all_join = [&](const FBlock& b) {
    if (!s->tune.diag_runs) return false;
    for (int m : b.members)
      if (!joins_run(pend[m])) return false;
    return true;
  };
  // The matrices of consecutive dense blocks go up in one copy per segment
  // (at most kUploadBatch bytes) instead of one copy per block; a segment's
  // blocks are launched before the next segment is staged, so recycling the
  // constant arena (after a stream sync) never overwrites a matrix that a
  // launched block has yet to read.
  constexpr size_t kUploadBatch = kArenaBytes / 4;
  auto dense = [&](const FBlock& b) { return b.members.size() > 1 && !b.diag && b.qubits.size() > 1; };
  std::vector<const void*> dmat(blocks.size(), nullptr);
  size_t i = 0;
  while (i < blocks.size()) {
    std::vector<unsigned char> stage;
    std::vector<std::pair<size_t, size_t>> at;   // (block, offset in stage)
    size_t j = i;
    for (; j < blocks.size(); ++j) {
      if (!dense(blocks[j])) continue;
      std::vector<unsigned char> packed = pack_matrix(blocks[j].m, s->c64);
      const size_t o = (stage.size() + 255) & ~(size_t)255;
      if (!stage.empty() && o + packed.size() > kUploadBatch) break;
      stage.resize(o + packed.size());
      std::memcpy(stage.data() + o, packed.data(), packed.size());
      at.emplace_back(j, o);
    }
    if (!stage.empty()) {
      const void* base = nullptr;
      qk_status st = arena_put(s, stage.data(), stage.size(), &base);
      if (st) return st;
      for (const auto& bo : at) dmat[bo.first] = (const char*)base + bo.second;
    }
    for (; i < j; ++i) {
      const FBlock& b = blocks[i];
      qk_status st;
      if ((b.diag || b.members.size() == 1) && all_join(b)) {
        for (int m : b.members)
          if ((st = add_to_run(s, std::move(pend[m])))) return st;
        continue;
      }
      if ((st = flush_drun(s))) return st;
      if (b.members.size() == 1) {   // a block of one gate runs through that gate's own sweep
        st = execute(s, pend[b.members[0]]);
        if (st) return st;
        continue;
      }
      s->fused_blocks++;
      s->fused_gates += b.ngates;
      if (b.diag) {
        const int D = 1 << b.qubits.size();
        std::vector<cd> dg(D);
        for (int e = 0; e < D; ++e) dg[e] = b.m[(size_t)e * D + e];
        st = run_diag(s, b.qubits, {}, none, dg);
      } else {
        st = run_dense(s, b.qubits, {}, none, b.m, dmat[i]);
      }
      if (st) return st;
    }
  }
  return QK_OK;
}

// The LDS-tile mode: the held-back builtin gates are grouped into stages of
// stage_chunk_qubits() qubits (gates pass one another only where they
// commute), their records go up through the constant arena, and each stage
// is one launch over every chunk of the state: a chunk (the amplitudes that
// agree on the qubits outside the stage) is gathered into LDS, every gate of
// the stage is applied there, and it is written back, so a stage costs one
// read and one write of the state whatever its gate count.
qk_status flush_stage(qk_sim s) {
  if (s->stage_q.empty()) return QK_OK;
  std::vector<qk_op> q;
  q.swap(s->stage_q);
  std::vector<unsigned char> recs;
  std::vector<uint32_t> heads;
  std::string err;
  qk_status st = stage_plan(s->c64, s->n, s->ncbits, q, recs, heads, err);
  if (st) return fail(s, st, "staged gates: " + err);
  const void* dev = nullptr;
  if ((st = arena_put(s, recs.data(), recs.size(), &dev))) return st;
  for (uint32_t h : heads) {
    launch_stage(s->c64, s->state.p, s->n, dev, h, (const uint8_t*)s->cbits.p, s->ncbits, s->stream);
    s->sweeps++;
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(s, e, "stage launch");
  return QK_OK;
}

// Gates the LDS-tile mode holds back: builtins on a dense state of
// stage_chunk_qubits() to 31 qubits, at most 4 controls, conditions on cbits
// below 256, outside graph capture.
bool stageable(qk_sim s, int nc, const qk_cond* conds, int ncond) {
  if (!s->tune.stages || s->sparse || s->capturing) return false;
  if (s->n < stage_chunk_qubits(s->c64) || s->n > 31 || nc > 4) return false;
  for (int i = 0; i < ncond; ++i)
    if (conds[i].cbit >= 256) return false;
  return true;
}

// Applies every operation held back (stage queue, fusion queue, diagonal run,
// sparse run).
qk_status flush(qk_sim s) {
  if (s->sparse) return sp_flush_run(s);
  qk_status st = flush_stage(s);
  if (st) return st;
  st = flush_pending(s);
  if (st) return st;
  return flush_drun(s);
}

// Puts a relabelled dense state back in logical qubit order (held-back gates
// first, as they act on the current layout): one physical swap per logical
// qubit that is not at its own bit.
qk_status restore_layout(qk_sim s) {
  if (s->sparse || dense_identity(s)) return QK_OK;
  qk_status st = flush(s);
  if (st) return st;
  Launch L = make_launch(s, {});
  for (int q = 0; q < s->n; ++q) {
    const int p = s->dphys[q];
    if (p == q) continue;
    int r = 0;   // the logical qubit now at bit q
    while (s->dphys[r] != q) ++r;
    if ((st = check_launch(s, launch_swap(L, p, q, nullptr, 0), "layout restore"))) return st;
    s->dphys[q] = q;
    s->dphys[r] = p;
  }
  return QK_OK;
}

qk_status sync_stream(qk_sim s) {
  hipError_t e = hipStreamSynchronize(s->stream);
  if (e != hipSuccess) {
    s->latched = QK_E_HIP;
    return hip_fail(s, e, "asynchronous device work failed");
  }
  return QK_OK;
}

std::string upper(const char* s) {
  std::string r(s ? s : "");
  for (auto& ch : r) ch = (char)std::toupper((unsigned char)ch);
  return r;
}

// Inverse of a modulo N (gcd(a, N) = 1), extended Euclid in signed 64-bit.
uint64_t inv_mod(uint64_t a, uint64_t N) {
  int64_t t = 0, nt = 1, r = (int64_t)N, nr = (int64_t)(a % N);
  while (nr != 0) {
    const int64_t q = r / nr;
    int64_t tmp = t - q * nt;
    t = nt;
    nt = tmp;
    tmp = r - q * nr;
    r = nr;
    nr = tmp;
  }
  if (t < 0) t += (int64_t)N;
  return (uint64_t)t;
}

uint64_t gcd_u64(uint64_t a, uint64_t b) {
  while (b) {
    const uint64_t t = a % b;
    a = b;
    b = t;
  }
  return a;
}

uint64_t inv_mod_2_64(uint64_t a) {
  uint64_t x = a;   // correct to 3 bits for odd a; each Newton step doubles them
  for (int i = 0; i < 6; ++i) x *= 2 - a * x;
  return x;
}

qk_status new_user_gate(qk_sim s, UserGate* g, qk_gate* out) {
  s->ugates.push_back(g);
  if (out) *out = kUserBase + (int)s->ugates.size() - 1;
  return QK_OK;
}

qk_status upload_table(qk_sim s, UserGate* g, const std::vector<uint64_t>& table) {
  const uint64_t K = 1ull << g->k;
  std::vector<uint32_t> finv(K);
  for (uint64_t x = 0; x < K; ++x) finv[table[x]] = (uint32_t)x;
  qk_status st = ensure(s, g->finv, K * sizeof(uint32_t), "permutation table");
  if (st) return st;
  hipError_t e = hipMemcpy(g->finv.p, finv.data(), K * sizeof(uint32_t), hipMemcpyHostToDevice);
  if (e != hipSuccess) return hip_fail(s, e, "permutation table upload");
  std::vector<uint32_t> fwd(K);
  for (uint64_t x = 0; x < K; ++x) fwd[x] = (uint32_t)table[x];
  if ((st = ensure(s, g->ftab, K * sizeof(uint32_t), "permutation table"))) return st;
  e = hipMemcpy(g->ftab.p, fwd.data(), K * sizeof(uint32_t), hipMemcpyHostToDevice);
  if (e != hipSuccess) return hip_fail(s, e, "permutation table upload");
  return QK_OK;
}

qk_status define_perm(qk_sim s, const char* name, int32_t k, const std::vector<uint64_t>& table, qk_gate* out) {
  if (s->capturing) return fail(s, QK_E_STATE, "not allowed while capturing a graph");
  const uint64_t K = 1ull << k;
  std::vector<unsigned char> seen(K, 0);
  for (uint64_t x = 0; x < K; ++x) {
    if (table[x] >= K || seen[table[x]])
      return fail(s, QK_E_NOT_PERMUTATION, "index function is not a bijection of [0, 2^k)");
    seen[table[x]] = 1;
  }
  UserGate* g = new UserGate;
  g->kind = U_TABLE;
  g->k = k;
  g->name = name ? name : "";
  qk_status st = upload_table(s, g, table);
  if (st) {
    dev_free(s, g->finv);
    dev_free(s, g->ftab);
    delete g;
    return st;
  }
  return new_user_gate(s, g, out);
}

// ---- sparse state ------------------------------------------------------------

struct SpArray {
  void** p;
  size_t bytes;
};

std::vector<SpArray> sp_arrays(qk_sim s) {
  const size_t c = s->sp.cap;
  return {{(void**)&s->sp.idx, c * 8}, {&s->sp.amp, c * s->amp}, {(void**)&s->sp.idx_b, c * 8},
          {&s->sp.amp_b, c * s->amp}, {(void**)&s->sp.key, c * 8}, {(void**)&s->sp.cnt, c * 4},
          {(void**)&s->sp.off, c * 8}, {(void**)&s->sp.scal, 32}, {&s->sp.temp, s->sp.temp_bytes}};
}

void sp_free(qk_sim s) {
  for (SpArray& a : sp_arrays(s)) {
    DevBuf b{*a.p, a.bytes};
    dev_free(s, b);
    *a.p = nullptr;
  }
  s->sp.nnz = 0;
}

qk_status sp_alloc(qk_sim s) {
  s->sp.temp_bytes = std::max<size_t>(256, sp_temp_bytes(s->sp.cap, s->c64));
  for (SpArray& a : sp_arrays(s)) {
    *a.p = dev_alloc(s, a.bytes);
    if (!*a.p) {
      sp_free(s);
      return fail(s, QK_E_OOM, "device allocation failed: sparse state of " + std::to_string(s->sp.cap) + " entries");
    }
  }
  return QK_OK;
}

qk_status sp_check(qk_sim s, hipError_t e, const char* what) {
  if (e == hipSuccess) return QK_OK;
  if (e == hipErrorOutOfMemory)
    return fail(s, QK_E_OOM, std::string(what) + ": the result would exceed the sparse capacity of " +
                                 std::to_string(s->sp.cap) + " entries (state unchanged)");
  return hip_fail(s, e, what);
}

qk_status sp_flush_run(qk_sim s) {
  if (s->sp_run.n == 0) return QK_OK;
  hipError_t e = sp_diag_run(s->sp, s->c64, s->sp_run, s->stream);
  s->sp_run.n = 0;
  s->sweeps += 1;
  return e == hipSuccess ? QK_OK : hip_fail(s, e, "sparse diagonal run");
}

int sp_bit(qk_sim s, int q) { return s->sp_phys.empty() ? q : s->sp_phys[q]; }

bool sp_identity(qk_sim s) {
  for (int q = 0; q < (int)s->sp_phys.size(); ++q)
    if (s->sp_phys[q] != q) return false;
  return true;
}

qk_status sp_flush_run(qk_sim s);

// Put the entries back in logical index order (before a readout that returns indices).
qk_status sp_normalize(qk_sim s) {
  qk_status st = sp_flush_run(s);
  if (st || sp_identity(s)) return st;
  SpTargets phys{};
  phys.k = s->n;
  for (int q = 0; q < s->n; ++q) phys.pos[q] = s->sp_phys[q];
  hipError_t e = sp_relabel(s->sp, s->n, s->c64, phys, s->stream);
  if (e != hipSuccess) return hip_fail(s, e, "sparse relabel");
  for (int q = 0; q < s->n; ++q) s->sp_phys[q] = q;
  s->sweeps += 1;
  return QK_OK;
}

qk_status sparse_execute(qk_sim s, const GateDesc& dl) {
  GateDesc d = dl;   // logical qubits -> index bits
  for (int& q : d.targets) q = sp_bit(s, q);
  for (int& q : d.controls) q = sp_bit(s, q);
  if (d.kind == D_SWAP && d.controls.empty()) {   // relabel two qubits; no entry moves
    if (!d.conds.empty()) {
      std::vector<uint8_t> cb(s->ncbits);
      hipError_t e = hipMemcpyAsync(cb.data(), s->cbits.p, cb.size(), hipMemcpyDeviceToHost, s->stream);
      if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
      if (e != hipSuccess) return hip_fail(s, e, "condition readback");
      for (const qk_cond& c : d.conds)
        if (cb[c.cbit] != (uint8_t)c.value) return QK_OK;
    }
    std::swap(s->sp_phys[dl.targets[0]], s->sp_phys[dl.targets[1]]);
    return QK_OK;
  }
  if ((d.kind == D_DIAG || d.kind == D_PHASE1) && d.conds.empty() && d.targets.size() <= 2) {
    SpDiagTerm& tm = s->sp_run.t[s->sp_run.n++];
    tm = SpDiagTerm{};
    tm.k = (int)d.targets.size();
    for (int j = 0; j < tm.k; ++j) tm.pos[j] = d.targets[j];
    for (int c : d.controls) tm.cmask |= 1ull << c;
    const int D = 1 << tm.k;
    for (int i = 0; i < D; ++i) {
      const cd v = d.kind == D_DIAG ? d.m[i] : (i == D - 1 ? d.z : cd(1.0));
      tm.d[2 * i] = v.real();
      tm.d[2 * i + 1] = v.imag();
    }
    if (s->sp_run.n == kSpDiagRun) return sp_flush_run(s);
    return QK_OK;
  }
  qk_status fst = sp_flush_run(s);
  if (fst) return fst;
  if (!d.conds.empty()) {   // the sparse engine synchronises anyway: decide on the host
    std::vector<uint8_t> cb(s->ncbits);
    hipError_t e = hipMemcpyAsync(cb.data(), s->cbits.p, cb.size(), hipMemcpyDeviceToHost, s->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    if (e != hipSuccess) return hip_fail(s, e, "condition readback");
    for (const qk_cond& c : d.conds)
      if (cb[c.cbit] != (uint8_t)c.value) return QK_OK;
  }
  SpTargets t{};
  t.k = (int)d.targets.size();
  for (int j = 0; j < t.k; ++j) t.pos[j] = d.targets[j];
  uint64_t cmask = 0;
  for (int c : d.controls) cmask |= 1ull << c;
  hipError_t e = hipSuccess;
  s->sweeps += 1;
  switch (d.kind) {
    case D_BUTTERFLY:
    case D_DENSE: {
      // an uncontrolled one-qubit gate on many entries goes by split and merges instead of sorts
      if (t.k == 1 && cmask == 0 && s->sp.nnz >= kSpMergeMin) {
        Mat2 u{};
        for (int i = 0; i < 4; ++i) {
          u.v[2 * i] = d.m[i].real();
          u.v[2 * i + 1] = d.m[i].imag();
        }
        return sp_check(s, sp_one_qubit(s->sp, s->n, s->c64, t.pos[0], u, s->stream), "sparse gate");
      }
      const void* dmat = d.ug ? d.ug->dmat.p : nullptr;
      if (!dmat) {
        std::vector<unsigned char> packed = pack_matrix(d.m, s->c64);
        qk_status st = arena_put(s, packed.data(), packed.size(), &dmat);
        if (st) return st;
      }
      return sp_check(s, sp_dense_gate(s->sp, s->n, s->c64, t, cmask, dmat, s->stream), "sparse gate");
    }
    case D_DIAG:
    case D_PHASE1: {
      const int D = 1 << t.k;
      std::vector<cd> dg(D, cd(1.0));
      if (d.kind == D_DIAG) dg = d.m;
      else dg[D - 1] = d.z;
      if (t.k > 6) {   // beyond the 64-entry table: as a dense diagonal matrix
        std::vector<cd> m((size_t)D * D, cd(0.0));
        for (int i = 0; i < D; ++i) m[(size_t)i * D + i] = dg[i];
        std::vector<unsigned char> packed = pack_matrix(m, s->c64);
        const void* dmat = nullptr;
        qk_status st = arena_put(s, packed.data(), packed.size(), &dmat);
        if (st) return st;
        return sp_check(s, sp_dense_gate(s->sp, s->n, s->c64, t, cmask, dmat, s->stream), "sparse gate");
      }
      Diag64 dd{};
      for (int i = 0; i < D; ++i) {
        dd.v[2 * i] = dg[i].real();
        dd.v[2 * i + 1] = dg[i].imag();
      }
      e = sp_diag(s->sp, s->c64, t, cmask, dd, s->stream);
      return sp_check(s, e, "sparse diagonal");
    }
    case D_SWAP:
      return sp_check(s, sp_permute(s->sp, s->n, s->c64, t, cmask, SP_PERM_SWAP, nullptr, 0, 0, 0, s->stream),
                      "sparse swap");
    case D_PERM: {
      const int mode = d.ug->kind == U_AFFINE ? SP_PERM_AFFINE
                                                : (d.ug->kind == U_MODMUL ? SP_PERM_MODMUL : SP_PERM_TABLE);
      const uint64_t B = mode == SP_PERM_MODMUL ? ~0ull / d.N : d.B;   // Barrett constant for the modulus
      return sp_check(s,
                      sp_permute(s->sp, s->n, s->c64, t, cmask, mode, (const uint32_t*)d.ug->ftab.p, d.A, B, d.N,
                                 s->stream),
                      "sparse permutation");
    }
  }
  return fail(s, QK_E_ARG, "unknown gate class");
}

}  // namespace

// ============================================================================ ABI

extern "C" {

const char* qk_status_string(qk_status st) {
  switch (st) {
    case QK_OK: return "ok";
    case QK_E_ARG: return "invalid argument";
    case QK_E_NOT_UNITARY: return "matrix is not unitary";
    case QK_E_NOT_PERMUTATION: return "index function is not a permutation";
    case QK_E_OOM: return "out of memory";
    case QK_E_HIP: return "HIP error";
    case QK_E_STATE: return "invalid state";
    case QK_E_UNSUPPORTED: return "unsupported";
  }
  return "unknown status";
}

const char* qk_last_error(qk_sim s) { return s ? s->err.c_str() : g_last_error.c_str(); }

qk_status qk_create(qk_dtype dtype, const qk_allocator* alloc, void* hip_stream, qk_sim* out) {
  if (!out) return fail(nullptr, QK_E_ARG, "out is NULL");
  *out = nullptr;
  if (dtype != QK_C64 && dtype != QK_C128) return fail(nullptr, QK_E_ARG, "dtype must be QK_C64 or QK_C128");
  if (alloc && (!alloc->alloc || !alloc->free)) return fail(nullptr, QK_E_ARG, "allocator needs alloc and free");
  qk_sim s = new qk_sim_s;
  s->dtype = dtype;
  s->c64 = dtype == QK_C64;
  s->amp = s->c64 ? 8 : 16;
  if (alloc) {
    s->alloc = *alloc;
    s->has_alloc = true;
  }
  s->stream = (hipStream_t)hip_stream;
  if (s->c64) {
    s->tune.diag_items = 2;
    s->tune.lane_items = 2;
    s->tune.sweep_items = 2;
  }
  *out = s;
  return QK_OK;
}

qk_status qk_create_sparse(qk_dtype dtype, const qk_allocator* alloc, void* hip_stream, int64_t max_nonzeros,
                           qk_sim* out) {
  if (max_nonzeros < 1 || max_nonzeros > ((int64_t)1 << 32))
    return fail(nullptr, QK_E_ARG, "max_nonzeros must be in [1, 2^32]");
  qk_status st = qk_create(dtype, alloc, hip_stream, out);
  if (st) return st;
  (*out)->sparse = true;
  (*out)->sp.cap = (uint64_t)max_nonzeros;
  return QK_OK;
}

qk_status qk_destroy(qk_sim s) {
  if (!s) return fail(nullptr, QK_E_ARG, "sim is NULL");
  if (s->capturing) {
    hipGraph_t g = nullptr;
    (void)hipStreamEndCapture(s->stream, &g);
    if (g) (void)hipGraphDestroy(g);
    s->capturing = false;
  }
  if (s->state.p || s->meas.p || s->sp.idx || !s->arenas.empty()) {
    // Synchronise only when work is still pending: on a stream that has
    // finished, hipStreamSynchronize still waited behind other streams' work
    // sharing its hardware queue (about 5 ms per simulator in a serving loop
    // that destroys one per job).
    if (hipStreamQuery(s->stream) != hipSuccess) (void)hipStreamSynchronize(s->stream);
    (void)hipGetLastError();
  }
  dev_free(s, s->state);
  dev_free(s, s->scratch);
  dev_free(s, s->cbits);
  dev_free(s, s->meas);
  dev_free(s, s->samp);
  dev_free(s, s->shots);
  if (s->sparse) sp_free(s);
  for (Arena& a : s->arenas) arena_free_chunk(s, a);
  for (Arena& a : s->saved_arenas) arena_free_chunk(s, a);
  for (UserGate* g : s->ugates) {
    dev_free(s, g->dmat);
    dev_free(s, g->finv);
    dev_free(s, g->ftab);
    delete g;
  }
  delete s;
  return QK_OK;
}

qk_status qk_add_qubits(qk_sim s, int32_t count, int32_t* first) {
  if (!s) return fail(nullptr, QK_E_ARG, "sim is NULL");
  if (s->capturing) return fail(s, QK_E_STATE, "not allowed while capturing a graph");
  if (count < 0) return fail(s, QK_E_ARG, "count < 0");
  if (s->sparse) {   // new qubits take the high bits in |0>: the entries keep their indices
    if (s->n + count > kMaxSparseQubits) return fail(s, QK_E_ARG, "too many qubits");
    if (first) *first = s->n;
    if (!s->sp.idx) {
      qk_status st = sp_alloc(s);
      if (st) return st;
      hipError_t e = sp_init(s->sp, s->c64, s->stream);
      if (e != hipSuccess) return hip_fail(s, e, "add_qubits");
    }
    for (int q = s->n; q < s->n + count; ++q) s->sp_phys.push_back(q);
    s->n += count;
    return QK_OK;
  }
  if (s->n + count > kMaxQubits) return fail(s, QK_E_ARG, "too many qubits");
  if (first) *first = s->n;
  if (count == 0 && s->state.p) return QK_OK;
  qk_status st = flush(s);
  if (st) return st;
  const int nn = s->n + count;
  const uint64_t newdim = 1ull << nn;
  DevBuf nb;
  nb.p = dev_alloc(s, newdim * s->amp);
  if (!nb.p) return fail(s, QK_E_OOM, "device allocation failed: state of " + std::to_string(nn) + " qubits");
  nb.bytes = newdim * s->amp;
  hipError_t e;
  if (!s->state.p) {
    e = launch_fill_zero(nb.p, 0, newdim, s->c64, s->stream);
    if (e == hipSuccess) e = launch_set_one(nb.p, 0, s->c64, s->stream);
  } else {
    const uint64_t olddim = 1ull << s->n;
    e = launch_copy(nb.p, s->state.p, olddim, s->c64, s->stream);
    if (e == hipSuccess) e = launch_fill_zero(nb.p, olddim, newdim, s->c64, s->stream);
  }
  if (e != hipSuccess) {
    dev_free(s, nb);
    return hip_fail(s, e, "add_qubits");
  }
  dev_free(s, s->state);
  dev_free(s, s->scratch);
  s->state = nb;
  for (int q = s->n; q < nn; ++q) s->dphys.push_back(q);   // new qubits take the new high bits
  s->n = nn;
  return QK_OK;
}

qk_status qk_add_cbits(qk_sim s, int32_t count, int32_t* first) {
  if (!s) return fail(nullptr, QK_E_ARG, "sim is NULL");
  if (s->capturing) return fail(s, QK_E_STATE, "not allowed while capturing a graph");
  if (count < 0 || s->ncbits + count > (1 << 20)) return fail(s, QK_E_ARG, "bad cbit count");
  if (first) *first = s->ncbits;
  if (count == 0) return QK_OK;
  qk_status st = flush(s);
  if (st) return st;
  const size_t nn = (size_t)s->ncbits + count;
  DevBuf nb;
  nb.p = dev_alloc(s, nn);
  if (!nb.p) return fail(s, QK_E_OOM, "device allocation failed: cbits");
  nb.bytes = nn;
  if (s->cbits.p) hipLaunchKernelGGL(k_u8_copy, dim3(1), dim3(256), 0, s->stream, (uint8_t*)nb.p, (const uint8_t*)s->cbits.p, (size_t)s->ncbits);
  hipLaunchKernelGGL(k_u8_fill, dim3(std::max<size_t>(1, std::min<size_t>(1024, (count + 255) / 256))), dim3(256), 0,
                     s->stream, (uint8_t*)nb.p, (size_t)s->ncbits, nn, (uint8_t)0);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    dev_free(s, nb);
    return hip_fail(s, e, "add_cbits");
  }
  dev_free(s, s->cbits);
  s->cbits = nb;
  s->ncbits = (int)nn;
  return QK_OK;
}

qk_status qk_gate_builtin(const char* name, qk_gate* out) {
  if (!name || !out) return fail(nullptr, QK_E_ARG, "name/out is NULL");
  const std::string u = upper(name);
  for (const auto& b : kBuiltins)
    if (u == b.name) {
      *out = b.id;
      return QK_OK;
    }
  return fail(nullptr, QK_E_ARG, "unknown builtin gate " + u);
}

qk_status qk_define_gate_matrix(qk_sim s, const char* name, int32_t k, const double* m, double tol, qk_gate* out) {
  if (!s) return fail(nullptr, QK_E_ARG, "sim is NULL");
  if (s->capturing) return fail(s, QK_E_STATE, "not allowed while capturing a graph");
  if (!m) return fail(s, QK_E_ARG, "matrix is NULL");
  if (k < 1 || k > QK_MAX_MATRIX_K) return fail(s, QK_E_ARG, "k out of range");
  if (!(tol > 0)) tol = 1e-10;
  const int D = 1 << k;
  std::vector<cd> M((size_t)D * D);
  for (size_t i = 0; i < M.size(); ++i) {
    M[i] = cd(m[2 * i], m[2 * i + 1]);
    if (!std::isfinite(m[2 * i]) || !std::isfinite(m[2 * i + 1])) return fail(s, QK_E_NOT_UNITARY, "non-finite entry");
  }
  double worst = 0;
  for (int r = 0; r < D; ++r)
    for (int c = 0; c < D; ++c) {
      cd acc(0, 0);
      for (int i = 0; i < D; ++i) acc += std::conj(M[(size_t)i * D + r]) * M[(size_t)i * D + c];
      worst = std::max(worst, std::abs(acc - (r == c ? cd(1.0) : cd(0.0))));
    }
  if (worst > tol) {
    char buf[96];
    std::snprintf(buf, sizeof buf, "matrix is not unitary: ||M^H M - I||_max = %.3e", worst);
    return fail(s, QK_E_NOT_UNITARY, buf);
  }
  UserGate* g = new UserGate;
  g->kind = U_MATRIX;
  g->k = k;
  g->name = name ? name : "";
  g->m = M;
  g->diag = true;
  for (int r = 0; r < D && g->diag; ++r)
    for (int c = 0; c < D; ++c)
      if (r != c && M[(size_t)r * D + c] != cd(0, 0)) {
        g->diag = false;
        break;
      }
  if (!g->diag && k >= 2) {
    auto packed = pack_matrix(M, s->c64);
    qk_status st = ensure(s, g->dmat, packed.size(), "gate matrix");
    if (st) {
      delete g;
      return st;
    }
    hipError_t e = hipMemcpy(g->dmat.p, packed.data(), packed.size(), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
      dev_free(s, g->dmat);
      delete g;
      return hip_fail(s, e, "gate matrix upload");
    }
  }
  return new_user_gate(s, g, out);
}

qk_status qk_define_gate_index(qk_sim s, const char* name, int32_t k, uint64_t (*f)(uint64_t, const void*),
                               const void* ctx, qk_gate* out) {
  if (!s) return fail(nullptr, QK_E_ARG, "sim is NULL");
  if (!f) return fail(s, QK_E_ARG, "function is NULL");
  if (k < 1 || k > QK_MAX_PERM_K) return fail(s, QK_E_ARG, "k out of range");
  std::vector<uint64_t> table(1ull << k);
  for (uint64_t x = 0; x < table.size(); ++x) table[x] = f(x, ctx);
  return define_perm(s, name, k, table, out);
}

qk_status qk_define_gate_table(qk_sim s, const char* name, int32_t k, const uint64_t* table, qk_gate* out) {
  if (!s) return fail(nullptr, QK_E_ARG, "sim is NULL");
  if (!table) return fail(s, QK_E_ARG, "table is NULL");
  if (k < 1 || k > QK_MAX_PERM_K) return fail(s, QK_E_ARG, "k out of range");
  std::vector<uint64_t> t(table, table + (1ull << k));
  return define_perm(s, name, k, t, out);
}

qk_status qk_define_gate_affine(qk_sim s, const char* name, int32_t k, uint64_t a, uint64_t b, qk_gate* out) {
  if (!s) return fail(nullptr, QK_E_ARG, "sim is NULL");
  if (k < 1 || k > 32) return fail(s, QK_E_ARG, "k out of range");
  if (!(a & 1)) return fail(s, QK_E_NOT_PERMUTATION, "a must be odd for x -> a x + b mod 2^k to be a bijection");
  UserGate* g = new UserGate;
  g->kind = U_AFFINE;
  g->k = k;
  g->name = name ? name : "";
  const uint64_t mask = (k == 64) ? ~0ull : ((1ull << k) - 1);
  g->a = a & mask;
  g->b = b & mask;
  return new_user_gate(s, g, out);
}

qk_status qk_define_gate_modmul(qk_sim s, const char* name, int32_t k, uint64_t a, uint64_t N, qk_gate* out) {
  if (!s) return fail(nullptr, QK_E_ARG, "sim is NULL");
  if (k < 1 || k > 32) return fail(s, QK_E_ARG, "k out of range");
  if (N < 2 || N > (1ull << k) || N >= (1ull << 32)) return fail(s, QK_E_ARG, "N must satisfy 2 <= N <= 2^k and N < 2^32");
  if (gcd_u64(a % N, N) != 1) return fail(s, QK_E_NOT_PERMUTATION, "a must be coprime to N for y -> a y mod N to be a bijection");
  UserGate* g = new UserGate;
  g->kind = U_MODMUL;
  g->k = k;
  g->name = name ? name : "";
  g->a = a % N;
  g->b = N;
  return new_user_gate(s, g, out);
}

qk_status qk_apply_gate(qk_sim s, qk_gate gate, const int32_t* targets, int32_t nt, const int32_t* controls,
                        int32_t nc, const qk_cond* conds, int32_t ncond, const double* params, int32_t np) {
  if (!s) return fail(nullptr, QK_E_ARG, "sim is NULL");
  if (nt < 1 || (nt > 0 && !targets)) return fail(s, QK_E_ARG, "no targets");
  if (nc < 0 || (nc > 0 && !controls)) return fail(s, QK_E_ARG, "bad controls");
  if (ncond < 0 || ncond > QK_MAX_CONDS || (ncond > 0 && !conds)) return fail(s, QK_E_ARG, "bad conditions");
  if (np < 0 || (np > 0 && !params)) return fail(s, QK_E_ARG, "bad params");
  if (nt + nc > QK_MAX_GATE_QUBITS) return fail(s, QK_E_ARG, "too many qubits in one gate");
  GateDesc d;
  int arity = 0;
  const UserGate* ug = nullptr;
  const BuiltinInfo* bi = nullptr;
  if (gate >= kUserBase && gate - kUserBase < (int)s->ugates.size()) {
    ug = s->ugates[gate - kUserBase];
    arity = ug->k;
    const int maxp = (ug->kind == U_AFFINE || ug->kind == U_MODMUL) ? 1 : 0;
    if (np > maxp) return fail(s, QK_E_ARG, "too many params for this gate");
  } else if ((bi = builtin_by_id(gate))) {
    arity = bi->arity;
    if (np != bi->nparams) return fail(s, QK_E_ARG, std::string("gate ") + bi->name + " takes " +
                                                          std::to_string(bi->nparams) + " param(s)");
  } else {
    return fail(s, QK_E_ARG, "unknown gate id");
  }
  if (nt != arity) return fail(s, QK_E_ARG, "target count does not match the gate");
  uint64_t seen = 0;
  for (int i = 0; i < nt + nc; ++i) {
    const int q = i < nt ? targets[i] : controls[i - nt];
    if (q < 0 || q >= s->n) return fail(s, QK_E_ARG, "qubit index out of range");
    if ((seen >> q) & 1) return fail(s, QK_E_ARG, "qubit used twice in one gate");
    seen |= 1ull << q;
  }
  for (int i = 0; i < ncond; ++i) {
    if (conds[i].cbit < 0 || conds[i].cbit >= s->ncbits) return fail(s, QK_E_ARG, "condition cbit out of range");
    if (conds[i].value != 0 && conds[i].value != 1) return fail(s, QK_E_ARG, "condition value must be 0 or 1");
  }
  if (!s->sparse && bi && bi->id == QK_SWAP && nc == 0 && ncond == 0 && !s->capturing && s->tune.swap_relabel) {
    // no data moves: later gates, measurements and readouts see the two
    // qubits at each other's bits
    std::swap(s->dphys[targets[0]], s->dphys[targets[1]]);
    return QK_OK;
  }
  d.targets.assign(targets, targets + nt);
  d.controls.assign(controls, controls + nc);
  d.conds.assign(conds, conds + ncond);
  if (!s->sparse) {
    for (int& q : d.targets) q = dbit(s, q);
    for (int& q : d.controls) q = dbit(s, q);
  }
  if (bi) {
    builtin_desc(bi->id, np ? params[0] : 0.0, d);
  } else if (ug->kind == U_MATRIX) {
    d.ug = ug;
    d.fusable = true;
    if (ug->diag) {
      d.kind = D_DIAG;
      const int D = 1 << ug->k;
      d.m.resize(D);
      for (int i = 0; i < D; ++i) d.m[i] = ug->m[(size_t)i * D + i];
      d.ug = nullptr;
    } else {
      d.kind = ug->k == 1 ? D_BUTTERFLY : D_DENSE;
      d.m = ug->m;
    }
  } else {
    d.kind = D_PERM;
    d.ug = ug;
    if (ug->kind == U_AFFINE) {
      double jd = np ? params[0] : 0.0;
      if (!(jd >= 0 && jd < 64 && jd == std::floor(jd))) return fail(s, QK_E_ARG, "affine power j must be an integer in [0, 64)");
      const int k = ug->k;
      const uint64_t mask = (k == 64) ? ~0ull : ((1ull << k) - 1);
      uint64_t A = ug->a, B = ug->b;
      for (int i = 0; i < (int)jd; ++i) {   // (A, B) o (A, B) = (A^2, A B + B)
        B = (A * B + B) & mask;
        A = (A * A) & mask;
      }
      d.A = A;
      d.B = B;
      d.Ainv = inv_mod_2_64(A) & mask;
    } else if (ug->kind == U_MODMUL) {
      double jd = np ? params[0] : 0.0;
      if (!(jd >= 0 && jd < 64 && jd == std::floor(jd))) return fail(s, QK_E_ARG, "power j must be an integer in [0, 64)");
      const uint64_t N = ug->b;
      uint64_t A = ug->a % N;
      for (int i = 0; i < (int)jd; ++i) A = (A * A) % N;   // a^(2^j) mod N; N < 2^32, no overflow
      d.A = A;
      d.N = N;
      d.Ainv = inv_mod(A, N);
    }
  }
  if (bi && stageable(s, nc, conds, ncond)) {
    qk_status st = flush_pending(s);
    if (!st) st = flush_drun(s);
    if (st) return st;
    qk_op o{};
    o.kind = QK_OP_GATE;
    o.gate = bi->id;
    o.n_targets = nt;
    for (int i = 0; i < nt; ++i) o.targets[i] = d.targets[i];
    o.n_controls = nc;
    for (int i = 0; i < nc; ++i) o.controls[i] = d.controls[i];
    o.n_conds = ncond;
    for (int i = 0; i < ncond; ++i) o.conds[i] = conds[i];
    o.param = np ? params[0] : 0.0;
    s->stage_q.push_back(o);
    if (s->stage_q.size() >= kStageQueueMax) return flush_stage(s);
    return QK_OK;
  }
  if (!s->stage_q.empty()) {
    qk_status st = flush_stage(s);
    if (st) return st;
  }
  if (s->sparse) return sparse_execute(s, d);
  if (d.conds.empty() && d.fusable && s->fuse_k >= 2 && nt + nc <= s->fuse_k) {
    qk_status st = flush_drun(s);   // gates before this one in the diagonal run act first
    if (st) return st;
    s->pending.push_back(std::move(d));
    return QK_OK;
  }
  if (s->tune.diag_runs && joins_run(d)) {
    qk_status st = flush_pending(s);
    if (st) return st;
    return add_to_run(s, std::move(d));
  }
  qk_status st = flush(s);
  if (st) return st;
  return execute(s, d);
}

qk_status qk_measure(qk_sim s, int32_t qubit, int32_t cbit, double u) {
  if (!s) return fail(nullptr, QK_E_ARG, "sim is NULL");
  if (qubit < 0 || qubit >= s->n) return fail(s, QK_E_ARG, "qubit out of range");
  if (cbit < -1 || cbit >= s->ncbits) return fail(s, QK_E_ARG, "cbit out of range");
  if (!(u >= 0.0 && u < 1.0)) return fail(s, QK_E_ARG, "u must be in [0, 1)");
  qk_status st = flush(s);
  if (st) return st;
  if ((st = ensure_meas(s))) return st;
  if (s->sparse) {   // index-order sums: entries back in logical order first
    if ((st = sp_normalize(s))) return st;
    s->sweeps += 1;
    return sp_check(s, sp_measure(s->sp, s->c64, sp_bit(s, qubit), cbit, u, nullptr, -1, meas_buffers(s), s->stream),
                    "measure");
  }
  Launch L = make_launch(s, {});
  hipError_t e = launch_measure(L, dbit(s, qubit), cbit, u, nullptr, -1, meas_buffers(s));
  if (e != hipSuccess) return hip_fail(s, e, "measure");
  s->sweeps += 2;
  return QK_OK;
}

qk_status qk_measure_dev(qk_sim s, int32_t qubit, int32_t cbit, const double* d_u) {
  if (!s) return fail(nullptr, QK_E_ARG, "sim is NULL");
  if (qubit < 0 || qubit >= s->n) return fail(s, QK_E_ARG, "qubit out of range");
  if (cbit < -1 || cbit >= s->ncbits) return fail(s, QK_E_ARG, "cbit out of range");
  if (!d_u) return fail(s, QK_E_ARG, "d_u is NULL");
  qk_status st = flush(s);
  if (st) return st;
  if ((st = ensure_meas(s))) return st;
  if (s->sparse) {
    if ((st = sp_normalize(s))) return st;
    s->sweeps += 1;
    return sp_check(s, sp_measure(s->sp, s->c64, sp_bit(s, qubit), cbit, 0.0, d_u, -1, meas_buffers(s), s->stream),
                    "measure");
  }
  Launch L = make_launch(s, {});
  hipError_t e = launch_measure(L, dbit(s, qubit), cbit, 0.0, d_u, -1, meas_buffers(s));
  if (e != hipSuccess) return hip_fail(s, e, "measure");
  s->sweeps += 2;
  return QK_OK;
}

qk_status qk_apply_ops(qk_sim s, const qk_op* ops, int32_t n_ops, int32_t* n_done) {
  if (!s) return fail(nullptr, QK_E_ARG, "sim is NULL");
  if (n_done) *n_done = 0;
  if (n_ops < 0 || (n_ops > 0 && !ops)) return fail(s, QK_E_ARG, "bad op list");
  for (int32_t i = 0; i < n_ops; ++i) {
    const qk_op& o = ops[i];
    qk_status st;
    if (o.kind == QK_OP_GATE) {
      if (o.n_targets < 1 || o.n_targets > 2 || o.n_controls < 0 || o.n_controls > 4 || o.n_conds < 0 ||
          o.n_conds > 2) {
        st = fail(s, QK_E_ARG, "counts exceed the record's arrays");
      } else {
        // builtins take their own parameter count; permutation families take j
        int np = 0;
        if (const BuiltinInfo* bi = builtin_by_id(o.gate)) np = bi->nparams;
        else if (o.gate >= kUserBase && o.gate - kUserBase < (int)s->ugates.size()) {
          const int kind = s->ugates[o.gate - kUserBase]->kind;
          np = (kind == U_AFFINE || kind == U_MODMUL) ? 1 : 0;
        }
        st = qk_apply_gate(s, o.gate, o.targets, o.n_targets, o.controls, o.n_controls, o.conds, o.n_conds,
                           &o.param, np);
      }
    } else if (o.kind == QK_OP_MEASURE) {
      st = qk_measure(s, o.qubit, o.cbit, o.u);
    } else {
      st = fail(s, QK_E_ARG, "unknown op kind");
    }
    if (st) {
      s->err = "op " + std::to_string(i) + ": " + s->err;
      return st;
    }
    if (n_done) *n_done = i + 1;
  }
  return QK_OK;
}

qk_status qk_measure_noalloc(qk_dtype dtype, void* d_state, int32_t n_qubits, int32_t qubit, const double* d_u,
                             uint8_t* d_cbit, double* d_result, void* hip_stream) {
  if (dtype != QK_C64 && dtype != QK_C128) return fail(nullptr, QK_E_ARG, "unknown dtype");
  if (!d_state || !d_u) return fail(nullptr, QK_E_ARG, "d_state or d_u is NULL");
  if (n_qubits < 1 || n_qubits > QK_NOALLOC_MAX_QUBITS)
    return fail(nullptr, QK_E_ARG, "n_qubits must be 1.." + std::to_string(QK_NOALLOC_MAX_QUBITS) +
                                       " (the fixed scratch covers one reduction grid of states up to that size)");
  if (qubit < 0 || qubit >= n_qubits) return fail(nullptr, QK_E_ARG, "qubit out of range");
  hipStream_t stream = (hipStream_t)hip_stream;
  int device = -1;
  hipError_t e = stream ? hipStreamGetDevice(stream, &device) : hipGetDevice(&device);
  if (e != hipSuccess) return hip_fail(nullptr, e, "measure_noalloc: device of the stream");
  e = launch_measure_noalloc(device, stream, d_state, n_qubits, dtype == QK_C64, qubit, d_u, d_cbit, d_result);
  if (e != hipSuccess) return hip_fail(nullptr, e, "measure_noalloc");
  return QK_OK;
}

qk_status qk_postselect(qk_sim s, int32_t qubit, int32_t cbit, int32_t outcome) {
  if (!s) return fail(nullptr, QK_E_ARG, "sim is NULL");
  if (s->capturing) return fail(s, QK_E_STATE, "not allowed while capturing a graph");
  if (qubit < 0 || qubit >= s->n) return fail(s, QK_E_ARG, "qubit out of range");
  if (cbit < -1 || cbit >= s->ncbits) return fail(s, QK_E_ARG, "cbit out of range");
  if (outcome != 0 && outcome != 1) return fail(s, QK_E_ARG, "outcome must be 0 or 1");
  qk_status st = flush(s);
  if (st) return st;
  if ((st = ensure_meas(s))) return st;
  if (s->sparse && (st = sp_normalize(s))) return st;
  Launch L = make_launch(s, {});
  MeasBuffers mb = meas_buffers(s);
  hipError_t e = s->sparse ? sp_measure(s->sp, s->c64, sp_bit(s, qubit), cbit, 0.0, nullptr, outcome, mb, s->stream)
                           : launch_measure(L, dbit(s, qubit), cbit, 0.0, nullptr, outcome, mb);
  if (e != hipSuccess) return hip_fail(s, e, "postselect");
  double res[4];
  e = hipMemcpyAsync(res, mb.result, sizeof res, hipMemcpyDeviceToHost, s->stream);
  if (e != hipSuccess) return hip_fail(s, e, "postselect readback");
  if ((st = sync_stream(s))) return st;
  if (res[2] == 0.0) return fail(s, QK_E_STATE, "forced outcome has probability 0");
  return QK_OK;
}

qk_status qk_read_cbits(qk_sim s, uint8_t* out, int32_t n) {
  if (!s) return fail(nullptr, QK_E_ARG, "sim is NULL");
  if (s->capturing) return fail(s, QK_E_STATE, "not allowed while capturing a graph");
  if (n < 0 || n > s->ncbits || (n > 0 && !out)) return fail(s, QK_E_ARG, "bad cbit count");
  qk_status st = flush(s);
  if (st) return st;
  if (n > 0) {
    hipError_t e = hipMemcpyAsync(out, s->cbits.p, (size_t)n, hipMemcpyDeviceToHost, s->stream);
    if (e != hipSuccess) return hip_fail(s, e, "read cbits");
  }
  return sync_stream(s);
}

qk_status qk_read_measure_log(qk_sim s, double* out, int32_t count, int32_t* written) {
  if (!s) return fail(nullptr, QK_E_ARG, "sim is NULL");
  if (s->capturing) return fail(s, QK_E_STATE, "not allowed while capturing a graph");
  if (count < 0 || (count > 0 && !out)) return fail(s, QK_E_ARG, "bad count");
  if (written) *written = 0;
  qk_status st = flush(s);
  if (st) return st;
  if (!s->meas.p) return QK_OK;
  std::vector<double> logbuf(3 * kMeasLog + 1);
  MeasBuffers mb = meas_buffers(s);
  hipError_t e = hipMemcpyAsync(logbuf.data(), mb.log, (3 * kMeasLog + 1) * sizeof(double), hipMemcpyDeviceToHost,
                                s->stream);
  if (e != hipSuccess) return hip_fail(s, e, "read measure log");
  if ((st = sync_stream(s))) return st;
  uint32_t total;
  std::memcpy(&total, &logbuf[3 * kMeasLog], sizeof total);
  const uint32_t avail = std::min<uint32_t>(total, kMeasLog);
  const uint32_t take = std::min<uint32_t>(avail, (uint32_t)count);
  for (uint32_t i = 0; i < take; ++i) {
    const uint32_t idx = total - take + i;
    const uint32_t slot = idx % kMeasLog;
    out[3 * i] = logbuf[3 * slot];
    out[3 * i + 1] = logbuf[3 * slot + 1];
    out[3 * i + 2] = logbuf[3 * slot + 2];
  }
  if (written) *written = (int32_t)take;
  return QK_OK;
}

// ---------------------------------------------------------------- deferred measurement

static qk_status check_qubit_list(qk_sim s, const int32_t* qubits, int32_t nq, int32_t max_nq) {
  if (nq < 0 || nq > max_nq || (nq > 0 && !qubits)) return fail(s, QK_E_ARG, "bad qubit list");
  uint64_t seen = 0;
  for (int j = 0; j < nq; ++j) {
    if (qubits[j] < 0 || qubits[j] >= s->n) return fail(s, QK_E_ARG, "qubit out of range");
    if ((seen >> qubits[j]) & 1) return fail(s, QK_E_ARG, "duplicate qubit in list");
    seen |= 1ull << qubits[j];
  }
  return QK_OK;
}

static uint64_t sample_dim(qk_sim s) { return s->sparse ? s->sp.nnz : (1ull << s->n); }

static qk_status sample_common(qk_sim s, const int32_t* qubits, int32_t nq, int64_t nshots) {
  if (!s) return fail(nullptr, QK_E_ARG, "sim is NULL");
  if (!s->state.p && !s->sp.idx) return fail(s, QK_E_STATE, "no qubits");
  if (nshots < 0 || nshots > ((int64_t)1 << 32)) return fail(s, QK_E_ARG, "n_shots must be in [0, 2^32]");
  qk_status st = check_qubit_list(s, qubits, nq, s->n);
  if (st) return st;
  const size_t need = (s->sparse ? sample_layout_dim(s->sp.cap) : sample_layout(s->n)).doubles * sizeof(double);
  if (s->capturing) {
    if (!s->samp.p || s->samp.bytes < need)
      return fail(s, QK_E_STATE, "sampling work space missing: sample once before capturing");
    return flush(s);
  }
  if ((st = flush(s))) return st;
  if (s->sparse && (st = sp_normalize(s))) return st;   // the CDF runs in logical index order
  if ((st = restore_layout(s))) return st;
  return ensure(s, s->samp, need, "sampling work space");
}

// Distribution sweep and shots.  A sparse state draws positions in its entry
// array (into `pos`, n_shots words) and maps them to indices.
static hipError_t draw_shots(qk_sim s, const int32_t* qubits, int32_t nq, const double* d_u, uint64_t nshots,
                             uint64_t* d_out, uint64_t* pos) {
  double* work = (double*)s->samp.p;
  if (!s->sparse) {
    Launch L = make_launch(s, {});
    hipError_t e = launch_cdf(L, work);
    if (e == hipSuccess) e = launch_draw(L, work, qubits, nq, d_u, nshots, d_out);
    return e;
  }
  hipError_t e = launch_cdf_dim(s->sp.amp, s->sp.nnz, s->c64, s->stream, work);
  if (e == hipSuccess) e = launch_draw_dim(s->sp.amp, s->sp.nnz, s->c64, s->stream, work, d_u, nshots, pos);
  SpTargets ql{};   // logical qubits -> index bits (all qubits when none are listed and the map is not the identity)
  ql.k = nq;
  for (int j = 0; j < nq; ++j) ql.pos[j] = sp_bit(s, qubits[j]);
  if (nq == 0 && !sp_identity(s)) {
    ql.k = s->n;
    for (int q = 0; q < s->n; ++q) ql.pos[q] = sp_bit(s, q);
  }
  if (e == hipSuccess) e = sp_project(s->sp, pos, nshots, ql, d_out, s->stream);
  return e;
}

qk_status qk_sample(qk_sim s, const int32_t* qubits, int32_t nq, const double* uniforms, int64_t nshots,
                    uint64_t* out) {
  if (s && s->capturing) return fail(s, QK_E_STATE, "not allowed while capturing a graph");
  qk_status st = sample_common(s, qubits, nq, nshots);
  if (st) return st;
  if (nshots > 0 && (!uniforms || !out)) return fail(s, QK_E_ARG, "uniforms and out must be given");
  for (int64_t i = 0; i < nshots; ++i)
    if (!(uniforms[i] >= 0.0 && uniforms[i] < 1.0)) return fail(s, QK_E_ARG, "uniforms must lie in [0, 1)");
  const size_t S1 = (size_t)std::max<int64_t>(nshots, 1);
  if ((st = ensure(s, s->shots, S1 * (s->sparse ? 24 : 16), "shot staging"))) return st;
  double* d_u = (double*)s->shots.p;
  uint64_t* d_out = (uint64_t*)((char*)s->shots.p + S1 * 8);
  uint64_t* pos = (uint64_t*)((char*)s->shots.p + S1 * 16);
  hipError_t e = hipSuccess;
  if (nshots > 0) e = hipMemcpyAsync(d_u, uniforms, (size_t)nshots * 8, hipMemcpyHostToDevice, s->stream);
  if (e == hipSuccess) e = draw_shots(s, qubits, nq, d_u, (uint64_t)nshots, d_out, pos);
  if (e != hipSuccess) return hip_fail(s, e, "sample");
  s->sweeps += 1;
  const SampleLayout sl = sample_layout_dim(sample_dim(s));
  double total = 0.0;
  e = hipMemcpyAsync(&total, (double*)s->samp.p + sl.nseg + 2 * sl.nchunk, sizeof total, hipMemcpyDeviceToHost,
                     s->stream);
  if (e == hipSuccess && nshots > 0)
    e = hipMemcpyAsync(out, d_out, (size_t)nshots * 8, hipMemcpyDeviceToHost, s->stream);
  if (e != hipSuccess) return hip_fail(s, e, "sample readback");
  if ((st = sync_stream(s))) return st;
  if (!(total > 0.0)) return fail(s, QK_E_STATE, "state has zero norm");
  return QK_OK;
}

qk_status qk_sample_dev(qk_sim s, const int32_t* qubits, int32_t nq, const double* d_u, int64_t nshots,
                        uint64_t* d_out) {
  qk_status st = sample_common(s, qubits, nq, nshots);
  if (st) return st;
  if (nshots > 0 && (!d_u || !d_out)) return fail(s, QK_E_ARG, "d_uniforms and d_out must be given");
  uint64_t* pos = nullptr;
  if (s->sparse) {
    if ((st = ensure(s, s->shots, (size_t)std::max<int64_t>(nshots, 1) * 8, "shot positions"))) return st;
    pos = (uint64_t*)s->shots.p;
  }
  hipError_t e = draw_shots(s, qubits, nq, d_u, (uint64_t)nshots, d_out, pos);
  if (e != hipSuccess) return hip_fail(s, e, "sample");
  s->sweeps += 1;
  return QK_OK;
}

qk_status qk_probabilities(qk_sim s, const int32_t* qubits, int32_t nq, double* out) {
  if (!s) return fail(nullptr, QK_E_ARG, "sim is NULL");
  if (s->sparse) return fail(s, QK_E_UNSUPPORTED, "probabilities of a sparse state: draw shots instead");
  if (s->capturing) return fail(s, QK_E_STATE, "not allowed while capturing a graph");
  if (!s->state.p) return fail(s, QK_E_STATE, "no qubits");
  if (nq < 1) return fail(s, QK_E_ARG, "list at least one qubit");
  qk_status st = check_qubit_list(s, qubits, nq, std::min(s->n, 24));
  if (st) return st;
  if (!out) return fail(s, QK_E_ARG, "out is NULL");
  if ((st = flush(s))) return st;
  if ((st = restore_layout(s))) return st;
  const MarginalLayout ml = marginal_layout(s->n, nq);
  const size_t need = (ml.partial_doubles + ml.nrows) * sizeof(double);
  if ((st = ensure(s, s->samp, std::max(need, sample_layout(s->n).doubles * sizeof(double)), "distribution work space")))
    return st;
  double* partial = (double*)s->samp.p;
  double* d_out = partial + ml.partial_doubles;
  Launch L = make_launch(s, {});
  hipError_t e = launch_marginal(L, qubits, nq, partial, d_out);
  if (e == hipSuccess) e = hipMemcpyAsync(out, d_out, ml.nrows * sizeof(double), hipMemcpyDeviceToHost, s->stream);
  if (e != hipSuccess) return hip_fail(s, e, "probabilities");
  s->sweeps += 1;
  if ((st = sync_stream(s))) return st;
  double total = 0.0;
  for (uint64_t m = 0; m < ml.nrows; ++m) total += out[m];
  if (!(total > 0.0)) return fail(s, QK_E_STATE, "state has zero norm");
  for (uint64_t m = 0; m < ml.nrows; ++m) out[m] /= total;
  return QK_OK;
}

// Copy the sparse entries to host memory (synchronises).
static qk_status sp_read(qk_sim s, std::vector<uint64_t>& idx, std::vector<unsigned char>& amp) {
  idx.resize(s->sp.nnz);
  amp.resize(s->sp.nnz * s->amp);
  hipError_t e = hipSuccess;
  if (s->sp.nnz) {
    e = hipMemcpyAsync(idx.data(), s->sp.idx, s->sp.nnz * 8, hipMemcpyDeviceToHost, s->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(amp.data(), s->sp.amp, amp.size(), hipMemcpyDeviceToHost, s->stream);
  }
  if (e != hipSuccess) return hip_fail(s, e, "sparse readback");
  return sync_stream(s);
}

qk_status qk_get_state(qk_sim s, void* host_out, size_t bytes) {
  if (!s) return fail(nullptr, QK_E_ARG, "sim is NULL");
  if (s->capturing) return fail(s, QK_E_STATE, "not allowed while capturing a graph");
  if (s->sparse) {   // the dense vector, assembled on the host from the entries
    if (s->n > kMaxQubits || !host_out || bytes != ((size_t)1 << s->n) * s->amp)
      return fail(s, QK_E_ARG, "buffer size must be 2^n * amplitude size (n <= 40)");
    if (!s->sp.idx) return fail(s, QK_E_STATE, "no qubits");
    qk_status st = sp_normalize(s);
    if (st) return st;
    std::vector<uint64_t> idx;
    std::vector<unsigned char> amp;
    st = sp_read(s, idx, amp);
    if (st) return st;
    std::memset(host_out, 0, bytes);
    for (size_t i = 0; i < idx.size(); ++i)
      std::memcpy((char*)host_out + idx[i] * s->amp, amp.data() + i * s->amp, s->amp);
    return QK_OK;
  }
  const size_t need = ((size_t)1 << s->n) * s->amp;
  if (!host_out || bytes != need) return fail(s, QK_E_ARG, "buffer size must be 2^n * amplitude size");
  if (!s->state.p) return fail(s, QK_E_STATE, "no qubits");
  qk_status st = flush(s);
  if (!st) st = restore_layout(s);
  if (st) return st;
  hipError_t e = hipMemcpyAsync(host_out, s->state.p, need, hipMemcpyDeviceToHost, s->stream);
  if (e != hipSuccess) return hip_fail(s, e, "get_state");
  return sync_stream(s);
}

qk_status qk_set_state(qk_sim s, const void* host_in, size_t bytes) {
  if (!s) return fail(nullptr, QK_E_ARG, "sim is NULL");
  if (s->capturing) return fail(s, QK_E_STATE, "not allowed while capturing a graph");
  if (s->sparse) {   // keep the nonzero amplitudes, in index order
    if (s->n > kMaxQubits || !host_in || bytes != ((size_t)1 << s->n) * s->amp)
      return fail(s, QK_E_ARG, "buffer size must be 2^n * amplitude size (n <= 40)");
    if (!s->sp.idx) return fail(s, QK_E_STATE, "no qubits");
    std::vector<uint64_t> idx;
    std::vector<unsigned char> amp;
    const unsigned char* src = (const unsigned char*)host_in;
    for (uint64_t i = 0; i < (1ull << s->n); ++i) {
      // zero by value, so -0.0 parts count as zero too
      bool zero;
      if (s->c64) {
        float v[2];
        std::memcpy(v, src + i * 8, 8);
        zero = v[0] == 0.0f && v[1] == 0.0f;
      } else {
        double v[2];
        std::memcpy(v, src + i * 16, 16);
        zero = v[0] == 0.0 && v[1] == 0.0;
      }
      if (zero) continue;
      idx.push_back(i);
      amp.insert(amp.end(), src + i * s->amp, src + (i + 1) * s->amp);
    }
    if (idx.size() > s->sp.cap) return fail(s, QK_E_OOM, "state has more nonzeros than the sparse capacity");
    qk_status st = flush(s);   // gates held back act on the state being replaced
    if (!st) st = sync_stream(s);
    if (st) return st;
    hipError_t e = hipSuccess;
    if (!idx.empty()) {
      e = hipMemcpy(s->sp.idx, idx.data(), idx.size() * 8, hipMemcpyHostToDevice);
      if (e == hipSuccess) e = hipMemcpy(s->sp.amp, amp.data(), amp.size(), hipMemcpyHostToDevice);
    }
    if (e != hipSuccess) return hip_fail(s, e, "set_state");
    s->sp.nnz = idx.size();
    for (int q = 0; q < s->n; ++q) s->sp_phys[q] = q;
    return QK_OK;
  }
  const size_t need = ((size_t)1 << s->n) * s->amp;
  if (!host_in || bytes != need) return fail(s, QK_E_ARG, "buffer size must be 2^n * amplitude size");
  if (!s->state.p) return fail(s, QK_E_STATE, "no qubits");
  qk_status st = flush(s);
  if (st) return st;
  for (int q = 0; q < s->n; ++q) s->dphys[q] = q;   // the new data is in logical order
  hipError_t e = hipMemcpyAsync(s->state.p, host_in, need, hipMemcpyHostToDevice, s->stream);
  if (e != hipSuccess) return hip_fail(s, e, "set_state");
  return sync_stream(s);
}

qk_status qk_state_ptr(qk_sim s, void** dev_ptr, size_t* bytes) {
  if (!s) return fail(nullptr, QK_E_ARG, "sim is NULL");
  if (s->sparse) return fail(s, QK_E_UNSUPPORTED, "a sparse state has no dense vector");
  qk_status st = flush(s);
  if (!st) st = restore_layout(s);
  if (st) return st;
  if (dev_ptr) *dev_ptr = s->state.p;
  if (bytes) *bytes = s->state.p ? ((size_t)1 << s->n) * s->amp : 0;
  return QK_OK;
}

qk_status qk_sparse_nnz(qk_sim s, int64_t* nnz) {
  if (!s || !nnz) return fail(s, QK_E_ARG, "sim or nnz is NULL");
  if (!s->sparse) return fail(s, QK_E_UNSUPPORTED, "not a sparse simulator");
  *nnz = (int64_t)s->sp.nnz;
  return QK_OK;
}

qk_status qk_sparse_entries(qk_sim s, uint64_t* idx, void* amps, int64_t cap, int64_t* nnz) {
  if (!s) return fail(nullptr, QK_E_ARG, "sim is NULL");
  if (!s->sparse) return fail(s, QK_E_UNSUPPORTED, "not a sparse simulator");
  if (s->capturing) return fail(s, QK_E_STATE, "not allowed while capturing a graph");
  if (nnz) *nnz = (int64_t)s->sp.nnz;
  if (cap < (int64_t)s->sp.nnz) return fail(s, QK_E_ARG, "cap is smaller than the number of entries");
  qk_status st = sp_normalize(s);
  if (st) return st;
  if (s->sp.nnz && (!idx || !amps)) return fail(s, QK_E_ARG, "idx and amps must be given");
  if (!s->sp.nnz) return QK_OK;   // no qubits added yet
  hipError_t e = hipMemcpyAsync(idx, s->sp.idx, s->sp.nnz * 8, hipMemcpyDeviceToHost, s->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(amps, s->sp.amp, s->sp.nnz * s->amp, hipMemcpyDeviceToHost, s->stream);
  if (e != hipSuccess) return hip_fail(s, e, "sparse entries");
  return sync_stream(s);
}

qk_status qk_inner_product(qk_sim a, qk_sim b, double* re, double* im) {
  if (!a || !b) return fail(nullptr, QK_E_ARG, "sim is NULL");
  if (a->sparse || b->sparse) {
    if (a != b) return fail(a, QK_E_UNSUPPORTED, "inner product with a sparse state");
    if (!a->sp.idx) return fail(a, QK_E_STATE, "no qubits");
    qk_status st = flush(a);
    if (st) return st;
    if ((st = ensure_meas(a))) return st;
    if (st) return st;
    const int nb = reduce_blocks_for(a->sp.nnz);
    MeasBuffers mb = meas_buffers(a);
    hipError_t e = sp_norm_partials(a->sp, a->c64, mb.partials, nb, a->stream);
    std::vector<double> part(nb);
    if (e == hipSuccess)
      e = hipMemcpyAsync(part.data(), mb.partials, nb * sizeof(double), hipMemcpyDeviceToHost, a->stream);
    if (e != hipSuccess) return hip_fail(a, e, "norm");
    if ((st = sync_stream(a))) return st;
    double sum = 0;
    for (int i = 0; i < nb; ++i) sum += part[i];
    if (re) *re = sum;
    if (im) *im = 0.0;
    return QK_OK;
  }
  if (a->n != b->n || !a->state.p || !b->state.p) return fail(a, QK_E_ARG, "qubit counts differ or no state");
  if (a->capturing || b->capturing) return fail(a, QK_E_STATE, "not allowed while capturing a graph");
  qk_status st = flush(a);
  if (!st) st = flush(b);
  // two states are compared index by index in logical order (a norm needs no order)
  if (!st && b != a) st = restore_layout(a);
  if (!st && b != a) st = restore_layout(b);
  if (st) return st;
  if (b != a && (st = sync_stream(b))) return st;
  if ((st = ensure_meas(a))) return st;
  const uint64_t dim = 1ull << a->n;
  const int nb = reduce_blocks_for(dim);
  MeasBuffers mb = meas_buffers(a);
  hipError_t e = launch_inner_partials(a->state.p, a->c64, b->state.p, b->c64, dim, mb.partials, nb, a->stream);
  if (e != hipSuccess) return hip_fail(a, e, "inner product");
  std::vector<double> part(2 * nb);
  e = hipMemcpyAsync(part.data(), mb.partials, part.size() * sizeof(double), hipMemcpyDeviceToHost, a->stream);
  if (e != hipSuccess) return hip_fail(a, e, "inner product readback");
  if ((st = sync_stream(a))) return st;
  double sr = 0, si = 0;
  for (int i = 0; i < nb; ++i) {
    sr += part[2 * i];
    si += part[2 * i + 1];
  }
  if (re) *re = sr;
  if (im) *im = si;
  return QK_OK;
}

qk_status qk_norm2_async(qk_sim s, double* host_partials, int32_t capacity, int32_t* count) {
  if (!s) return fail(nullptr, QK_E_ARG, "sim is NULL");
  if (!count || (capacity > 0 && !host_partials)) return fail(s, QK_E_ARG, "NULL argument");
  if (s->sparse) return fail(s, QK_E_UNSUPPORTED, "asynchronous norm of a sparse state");
  if (s->capturing) return fail(s, QK_E_STATE, "not allowed while capturing a graph");
  if (!s->state.p) return fail(s, QK_E_STATE, "no qubits");
  qk_status st = flush(s);
  if (st) return st;
  if ((st = ensure_meas(s))) return st;
  const uint64_t dim = 1ull << s->n;
  const int nb = reduce_blocks_for(dim);
  if (capacity < 2 * nb) return fail(s, QK_E_ARG, "capacity below 2 x " + std::to_string(nb) + " partial sums");
  MeasBuffers mb = meas_buffers(s);
  hipError_t e = launch_inner_partials(s->state.p, s->c64, s->state.p, s->c64, dim, mb.partials, nb, s->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(host_partials, mb.partials, 2 * (size_t)nb * sizeof(double), hipMemcpyDeviceToHost, s->stream);
  if (e != hipSuccess) return hip_fail(s, e, "asynchronous norm");
  *count = nb;
  return QK_OK;
}

qk_status qk_read_cbits_async(qk_sim s, uint8_t* host_out, int32_t n) {
  if (!s) return fail(nullptr, QK_E_ARG, "sim is NULL");
  if (s->capturing) return fail(s, QK_E_STATE, "not allowed while capturing a graph");
  if (n < 0 || n > s->ncbits || (n > 0 && !host_out)) return fail(s, QK_E_ARG, "bad cbit count");
  qk_status st = flush(s);
  if (st) return st;
  if (n > 0) {
    hipError_t e = hipMemcpyAsync(host_out, s->cbits.p, (size_t)n, hipMemcpyDeviceToHost, s->stream);
    if (e != hipSuccess) return hip_fail(s, e, "asynchronous cbit read");
  }
  return QK_OK;
}

qk_status qk_norm2(qk_sim s, double* out) {
  double re = 0;
  qk_status st = qk_inner_product(s, s, &re, nullptr);
  if (st == QK_OK && out) *out = re;
  return st;
}


// ---------------------------------------------------------------- reset / graphs

struct qk_graph_s {
  qk_sim sim = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  void* state = nullptr;       // the state buffer the graph's kernels address
  std::vector<Arena> arenas;   // constants the captured copies read on every replay
};

qk_status qk_reset(qk_sim s) {
  if (!s) return fail(nullptr, QK_E_ARG, "sim is NULL");
  if (!s->state.p && !s->sp.idx) return fail(s, QK_E_STATE, "no qubits");
  qk_status st = flush(s);
  if (st) return st;
  hipError_t e;
  if (s->sparse) {
    e = sp_init(s->sp, s->c64, s->stream);
    for (int q = 0; q < s->n; ++q) s->sp_phys[q] = q;
  } else {
    const uint64_t dim = 1ull << s->n;
    e = launch_fill_zero(s->state.p, 0, dim, s->c64, s->stream);
    if (e == hipSuccess) e = launch_set_one(s->state.p, 0, s->c64, s->stream);
    for (int q = 0; q < s->n; ++q) s->dphys[q] = q;
  }
  if (e == hipSuccess && s->ncbits > 0) {
    hipLaunchKernelGGL(k_u8_fill, dim3(std::max<size_t>(1, std::min<size_t>(1024, (s->ncbits + 255) / 256))),
                       dim3(256), 0, s->stream, (uint8_t*)s->cbits.p, (size_t)0, (size_t)s->ncbits, (uint8_t)0);
    e = hipGetLastError();
  }
  if (e != hipSuccess) return hip_fail(s, e, "reset");
  return QK_OK;
}

qk_status qk_capture_begin(qk_sim s) {
  if (!s) return fail(nullptr, QK_E_ARG, "sim is NULL");
  if (s->sparse) return fail(s, QK_E_UNSUPPORTED, "a sparse simulator cannot be captured (it reads entry counts back)");
  if (s->capturing) return fail(s, QK_E_STATE, "already capturing");
  if (!s->state.p) return fail(s, QK_E_STATE, "add qubits before capturing");
  qk_status st = flush(s);
  if (st) return st;
  // a replay starts from the logical layout (swaps inside a capture move data)
  if ((st = restore_layout(s))) return st;
  // everything a replay touches is allocated now, outside the capture
  if ((st = ensure_meas(s))) return st;
  bool perms = false;
  for (const UserGate* g : s->ugates) perms = perms || g->kind != U_MATRIX;
  if (perms && (st = ensure_scratch(s))) return st;
  s->saved_arenas = std::move(s->arenas);
  s->arenas.clear();
  if ((st = arena_new_chunk(s))) {
    s->arenas = std::move(s->saved_arenas);
    return st;
  }
  hipError_t e = hipStreamBeginCapture(s->stream, hipStreamCaptureModeRelaxed);
  if (e != hipSuccess) {
    for (Arena& a : s->arenas) arena_free_chunk(s, a);
    s->arenas = std::move(s->saved_arenas);
    return hip_fail(s, e, "begin capture");
  }
  s->capturing = true;
  return QK_OK;
}

qk_status qk_capture_end(qk_sim s, qk_graph* out) {
  if (!s || !out) return fail(s, QK_E_ARG, "NULL argument");
  if (!s->capturing) return fail(s, QK_E_STATE, "not capturing");
  qk_status st = flush(s);
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamEndCapture(s->stream, &g);
  s->capturing = false;
  std::vector<Arena> mine = std::move(s->arenas);
  s->arenas = std::move(s->saved_arenas);
  s->saved_arenas.clear();
  if (st || e != hipSuccess || !g) {
    if (g) (void)hipGraphDestroy(g);
    (void)hipStreamSynchronize(s->stream);
    for (Arena& a : mine) arena_free_chunk(s, a);
    return st ? st : hip_fail(s, e, "end capture");
  }
  hipGraphExec_t x = nullptr;
  e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    (void)hipGraphDestroy(g);
    for (Arena& a : mine) arena_free_chunk(s, a);
    return hip_fail(s, e, "instantiate graph");
  }
  qk_graph q = new qk_graph_s;
  q->sim = s;
  q->graph = g;
  q->exec = x;
  q->state = s->state.p;
  q->arenas = std::move(mine);
  *out = q;
  return QK_OK;
}

qk_status qk_graph_launch(qk_graph g) {
  if (!g) return fail(nullptr, QK_E_ARG, "graph is NULL");
  if (g->sim->capturing) return fail(g->sim, QK_E_STATE, "not allowed while capturing a graph");
  qk_sim s = g->sim;
  qk_status st = flush(s);
  if (!st) st = restore_layout(s);   // the graph was recorded in the logical layout
  if (st) return st;
  if (s->state.p != g->state) {
    // an uncontrolled permutation gate since the capture left the state in the
    // other buffer: copy it back to the one the graph's kernels address
    if (s->scratch.p != g->state) return fail(s, QK_E_STATE, "the state was reallocated since the capture");
    hipError_t e = launch_copy(s->scratch.p, s->state.p, 1ull << s->n, s->c64, s->stream);
    if (e != hipSuccess) return hip_fail(s, e, "graph launch: state copy");
    std::swap(s->state, s->scratch);
  }
  hipError_t e = hipGraphLaunch(g->exec, s->stream);
  if (e != hipSuccess) return hip_fail(g->sim, e, "graph launch");
  return QK_OK;
}

qk_status qk_graph_destroy(qk_graph g) {
  if (!g) return fail(nullptr, QK_E_ARG, "graph is NULL");
  (void)hipStreamSynchronize(g->sim->stream);
  if (g->exec) (void)hipGraphExecDestroy(g->exec);
  if (g->graph) (void)hipGraphDestroy(g->graph);
  for (Arena& a : g->arenas) arena_free_chunk(g->sim, a);
  delete g;
  return QK_OK;
}


qk_status qk_plan_fusion(int32_t n, const qk_op* ops, int32_t nops, int32_t max_k, int32_t* n_blocks,
                         uint64_t* block_masks, int32_t* block_gates, int32_t max_blocks, double* matrices,
                         size_t matrices_len) {
  if (n < 1 || n > 64 || nops < 0 || (nops > 0 && !ops) || !n_blocks) return fail(nullptr, QK_E_ARG, "bad arguments");
  if (max_k < 1 || max_k > QK_MAX_FUSION_K) return fail(nullptr, QK_E_ARG, "max_k must be 1..6");
  std::vector<FGate> fg;
  for (int i = 0; i < nops; ++i) {
    const qk_op& o = ops[i];
    int arity = 0, np = 0;
    if (o.kind != QK_OP_GATE || o.n_conds != 0 || !builtin_info(o.gate, &arity, &np) || o.n_targets != arity ||
        o.n_controls < 0 || o.n_controls > 4)
      return fail(nullptr, QK_E_ARG, "op " + std::to_string(i) + ": only unconditioned builtin gates are planned");
    uint64_t seen = 0;
    for (int q = 0; q < o.n_targets + o.n_controls; ++q) {
      const int x = q < o.n_targets ? o.targets[q] : o.controls[q - o.n_targets];
      if (x < 0 || x >= n || ((seen >> x) & 1)) return fail(nullptr, QK_E_ARG, "op " + std::to_string(i) + ": bad qubit");
      seen |= 1ull << x;
    }
    if (o.n_targets + o.n_controls > max_k)
      return fail(nullptr, QK_E_ARG, "op " + std::to_string(i) + ": gate wider than max_k");
    GateDesc d;
    d.targets.assign(o.targets, o.targets + o.n_targets);
    d.controls.assign(o.controls, o.controls + o.n_controls);
    builtin_desc(o.gate, np ? o.param : 0.0, d);
    fg.push_back(make_fgate(d.targets.data(), (int)d.targets.size(), d.controls.data(), (int)d.controls.size(),
                            full_matrix(d)));
  }
  std::vector<FBlock> blocks = plan_blocks(fg, max_k);
  *n_blocks = (int32_t)blocks.size();
  size_t off = 0;
  for (size_t b = 0; b < blocks.size() && (int)b < max_blocks; ++b) {
    uint64_t m = 0;
    for (int q : blocks[b].qubits) m |= 1ull << q;
    if (block_masks) block_masks[b] = m;
    if (block_gates) block_gates[b] = blocks[b].ngates;
    if (matrices) {
      const size_t need = blocks[b].m.size() * 2;
      if (off + need > matrices_len) return fail(nullptr, QK_E_ARG, "matrices buffer too small");
      for (size_t e = 0; e < blocks[b].m.size(); ++e) {
        matrices[off + 2 * e] = blocks[b].m[e].real();
        matrices[off + 2 * e + 1] = blocks[b].m[e].imag();
      }
      off += need;
    }
  }
  return QK_OK;
}

qk_status qk_set_fusion(qk_sim s, int32_t max_k) {
  if (!s) return fail(nullptr, QK_E_ARG, "sim is NULL");
  if (max_k != 0 && (max_k < 2 || max_k > QK_MAX_FUSION_K)) return fail(s, QK_E_ARG, "max_k must be 0 or 2..6");
  if (s->sparse && max_k != 0) return fail(s, QK_E_UNSUPPORTED, "fusion applies to dense states only");
  qk_status st = flush(s);
  if (st) return st;
  s->fuse_k = max_k;
  return QK_OK;
}

qk_status qk_flush(qk_sim s) {
  if (!s) return fail(nullptr, QK_E_ARG, "sim is NULL");
  return flush(s);
}

qk_status qk_sync(qk_sim s) {
  if (!s) return fail(nullptr, QK_E_ARG, "sim is NULL");
  if (s->capturing) return fail(s, QK_E_STATE, "not allowed while capturing a graph");
  qk_status st = flush(s);
  if (st) return st;
  if (s->latched) return fail(s, s->latched, "an earlier asynchronous failure was latched");
  if (!s->state.p && !s->sp.idx && !s->meas.p && s->arenas.empty() && !s->cbits.p) return QK_OK;
  st = sync_stream(s);
  if (st == QK_OK)
    for (Arena& a : s->arenas) a.used = 0;
  return st;
}

qk_status qk_set_tuning(qk_sim s, const char* key, int32_t value) {
  if (!s || !key) return fail(s, QK_E_ARG, "NULL argument");
  const std::string k = key;
  if (k == "nt") {
    if (value < 0 || value > 2) return fail(s, QK_E_ARG, "nt must be 0, 1 or 2");
    s->tune.nt = value;
  } else if (k == "lane_bfly") {
    s->tune.lane_bfly = value != 0;
  } else if (k == "sweep_items") {
    if (value != 1 && value != 2 && value != 4) return fail(s, QK_E_ARG, "sweep_items must be 1, 2 or 4");
    s->tune.sweep_items = value;
  } else if (k == "diag_items") {
    if (value != 1 && value != 2 && value != 4) return fail(s, QK_E_ARG, "diag_items must be 1, 2 or 4");
    s->tune.diag_items = value;
  } else if (k == "lane_items") {
    if (value != 1 && value != 2 && value != 4) return fail(s, QK_E_ARG, "lane_items must be 1, 2 or 4");
    s->tune.lane_items = value;
  } else if (k == "mfma_areg") {
    s->tune.mfma_areg = value != 0;
  } else if (k == "mfma_lds") {
    if (value < 0 || value > 2) return fail(s, QK_E_ARG, "mfma_lds must be 0, 1 or 2");
    s->tune.mfma_lds = value;
  } else if (k == "lds_wg") {
    if (value < 1 || value > 8) return fail(s, QK_E_ARG, "lds_wg must be 1..8");
    s->tune.lds_wg = value;

  } else if (k == "stages") {
    if (value != 0 && value != 1) return fail(s, QK_E_ARG, "stages must be 0 or 1");
    qk_status st = flush(s);
    if (st) return st;
    s->tune.stages = value;
  } else if (k == "diag_runs") {
    if (value != 0 && value != 1) return fail(s, QK_E_ARG, "diag_runs must be 0 or 1");
    qk_status st = flush(s);
    if (st) return st;
    s->tune.diag_runs = value;
  } else if (k == "swap_relabel") {
    if (value != 0 && value != 1) return fail(s, QK_E_ARG, "swap_relabel must be 0 or 1");
    s->tune.swap_relabel = value;   // qubits already relabelled stay so (every gate goes through the map)
  } else if (k == "xcd") {
    s->tune.xcd = value != 0;
  } else if (k == "mfma_cols") {
    if (value != 16 && value != 32 && value != 64) return fail(s, QK_E_ARG, "mfma_cols must be 16, 32 or 64");
    s->tune.mfma_cols = value;
  } else if (k == "mfma_waves") {
    if (value < 4 || value > 32 || value % 4) return fail(s, QK_E_ARG, "mfma_waves must be 4..32, a multiple of 4");
    s->tune.mfma_waves = value;
  } else {
    return fail(s, QK_E_ARG, "unknown tuning key " + k);
  }
  return QK_OK;
}

qk_status qk_get_tuning(qk_sim s, const char* key, int32_t* value) {
  if (!s || !key || !value) return fail(s, QK_E_ARG, "NULL argument");
  const std::string k = key;
  if (k == "nt") *value = s->tune.nt;
  else if (k == "lane_bfly") *value = s->tune.lane_bfly;
  else if (k == "sweep_items") *value = s->tune.sweep_items;
  else if (k == "lane_items") *value = s->tune.lane_items;
  else if (k == "diag_items") *value = s->tune.diag_items;
  else if (k == "mfma_waves") *value = s->tune.mfma_waves;
  else if (k == "mfma_cols") *value = s->tune.mfma_cols;
  else if (k == "mfma_areg") *value = s->tune.mfma_areg;
  else if (k == "mfma_lds") *value = s->tune.mfma_lds;
  else if (k == "lds_wg") *value = s->tune.lds_wg;
  else if (k == "diag_runs") *value = s->tune.diag_runs;
  else if (k == "stages") *value = s->tune.stages;
  else if (k == "swap_relabel") *value = s->tune.swap_relabel;
  else if (k == "xcd") *value = s->tune.xcd;
  else return fail(s, QK_E_ARG, "unknown tuning key " + k);
  return QK_OK;
}

qk_status qk_num_qubits(qk_sim s, int32_t* n) {
  if (!s || !n) return fail(s, QK_E_ARG, "NULL argument");
  *n = s->n;
  return QK_OK;
}

qk_status qk_stats(qk_sim s, int64_t* sweeps, int64_t* fused_blocks, int64_t* fused_gates) {
  if (!s) return fail(nullptr, QK_E_ARG, "sim is NULL");
  if (sweeps) *sweeps = s->sweeps;
  if (fused_blocks) *fused_blocks = s->fused_blocks;
  if (fused_gates) *fused_gates = s->fused_gates;
  return QK_OK;
}

}  // extern "C"
