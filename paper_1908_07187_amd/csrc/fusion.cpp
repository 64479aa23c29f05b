// Gate fusion planner: groups consecutive matrix gates into blocks acting on at
// most kmax qubits and composes each block into one dense 2^k x 2^k matrix in
// FP64, so a run of gates costs one sweep of the state instead of one per gate.
//
// Grouping is greedy and commutation-aware in the two ways that need no
// algebra: gates on disjoint qubits commute, and diagonal gates commute with
// one another, so a gate may join the current block once every earlier gate
// on its qubits that it does not commute with is scheduled (plan_blocks).
#include <algorithm>
#include <cstring>

#include "qk_internal.h"

namespace qk {

static inline int bit_of(uint64_t x, int j) { return (int)((x >> j) & 1ull); }

FGate make_fgate(const int* targets, int k, const int* controls, int nc, const std::vector<cd>& g) {
  FGate f;
  for (int j = 0; j < k; ++j) f.qubits.push_back(targets[j]);
  for (int j = 0; j < nc; ++j) f.qubits.push_back(controls[j]);
  std::sort(f.qubits.begin(), f.qubits.end());
  const int q = (int)f.qubits.size();
  const int D = 1 << q, K = 1 << k;
  // position of each target / control inside the sorted qubit list
  std::vector<int> tp(k), cp(nc);
  for (int j = 0; j < k; ++j) tp[j] = (int)(std::find(f.qubits.begin(), f.qubits.end(), targets[j]) - f.qubits.begin());
  for (int j = 0; j < nc; ++j) cp[j] = (int)(std::find(f.qubits.begin(), f.qubits.end(), controls[j]) - f.qubits.begin());
  uint64_t cmask = 0, tmask = 0;
  for (int j = 0; j < nc; ++j) cmask |= 1ull << cp[j];
  for (int j = 0; j < k; ++j) tmask |= 1ull << tp[j];
  f.m.assign((size_t)D * D, cd(0, 0));
  for (int col = 0; col < D; ++col) {
    if ((col & cmask) != cmask) {
      f.m[(size_t)col * D + col] = 1.0;   // controls not all 1: identity
      continue;
    }
    int mc = 0;
    for (int j = 0; j < k; ++j) mc |= bit_of(col, tp[j]) << j;
    for (int mr = 0; mr < K; ++mr) {
      int row = col & ~(int)tmask;
      for (int j = 0; j < k; ++j) row |= bit_of(mr, j) << tp[j];
      f.m[(size_t)row * D + col] = g[(size_t)mr * K + mc];
    }
  }
  f.diag = true;
  for (int r = 0; r < D && f.diag; ++r)
    for (int c = 0; c < D; ++c)
      if (r != c && f.m[(size_t)r * D + c] != cd(0, 0)) {
        f.diag = false;
        break;
      }
  return f;
}

// b <- G b where gate g acts on a subset of the block's qubits; b is kept as
// separate real and imaginary parts (row-major, Db x Db each) so that the
// row updates below run over contiguous doubles.  The rows of b that differ
// only in the gate's bits form groups of 2^kg; each group's rows are replaced
// by G times them, a whole row at a time; a diagonal gate scales rows.
static void left_multiply(std::vector<double>& bre, std::vector<double>& bim, std::vector<double>& tre,
                          std::vector<double>& tim, const std::vector<int>& qubits, const FGate& g) {
  const int kb = (int)qubits.size(), kg = (int)g.qubits.size();
  const int Db = 1 << kb, Dg = 1 << kg;
  int off[64];   // row offset of each combination of the gate's bits
  uint32_t gmask = 0;
  {
    int pos[6];
    for (int j = 0; j < kg; ++j) {
      pos[j] = (int)(std::find(qubits.begin(), qubits.end(), g.qubits[j]) - qubits.begin());
      gmask |= 1u << pos[j];
    }
    for (int m = 0; m < Dg; ++m) {
      off[m] = 0;
      for (int j = 0; j < kg; ++j) off[m] |= bit_of(m, j) << pos[j];
    }
  }
  if (g.diag) {
    for (int r = 0; r < Db; ++r) {
      if (r & gmask) continue;
      for (int m = 0; m < Dg; ++m) {
        const cd z = g.m[(size_t)m * Dg + m];
        const double zr = z.real(), zi = z.imag();
        if (zr == 1.0 && zi == 0.0) continue;
        double* xr = &bre[(size_t)(r | off[m]) * Db];
        double* xi = &bim[(size_t)(r | off[m]) * Db];
        for (int c = 0; c < Db; ++c) {
          const double a = xr[c], b = xi[c];
          xr[c] = zr * a - zi * b;
          xi[c] = zr * b + zi * a;
        }
      }
    }
    return;
  }
  tre.resize((size_t)Dg * Db);
  tim.resize((size_t)Dg * Db);
  for (int r = 0; r < Db; ++r) {
    if (r & gmask) continue;
    for (int m = 0; m < Dg; ++m) {
      std::memcpy(&tre[(size_t)m * Db], &bre[(size_t)(r | off[m]) * Db], Db * sizeof(double));
      std::memcpy(&tim[(size_t)m * Db], &bim[(size_t)(r | off[m]) * Db], Db * sizeof(double));
    }
    for (int m = 0; m < Dg; ++m) {
      double* yr = &bre[(size_t)(r | off[m]) * Db];
      double* yi = &bim[(size_t)(r | off[m]) * Db];
      bool first = true;
      for (int j = 0; j < Dg; ++j) {
        const cd a = g.m[(size_t)m * Dg + j];
        const double ar = a.real(), ai = a.imag();
        if (ar == 0.0 && ai == 0.0) continue;
        const double* xr = &tre[(size_t)j * Db];
        const double* xi = &tim[(size_t)j * Db];
        if (first) {
          for (int c = 0; c < Db; ++c) {
            yr[c] = ar * xr[c] - ai * xi[c];
            yi[c] = ar * xi[c] + ai * xr[c];
          }
          first = false;
        } else {
          for (int c = 0; c < Db; ++c) {
            yr[c] += ar * xr[c] - ai * xi[c];
            yi[c] += ar * xi[c] + ai * xr[c];
          }
        }
      }
      if (first)
        for (int c = 0; c < Db; ++c) yr[c] = yi[c] = 0.0;
    }
  }
}

// Ready-frontier grouping.  A gate is ready when every earlier gate on each of
// its qubits that it does not commute with is already scheduled: for a
// non-diagonal gate that is every earlier gate on its qubits, for a diagonal
// gate (diagonal including its controls) every earlier non-diagonal gate on
// them, since diagonal gates commute with one another.  Absorbing ready gates
// in any order is then a valid reordering: two gates change order only when
// they act on disjoint qubits or are both diagonal.  A block grows one ready
// gate at a time: gates already inside the block's qubit set first; otherwise
// the fitting gate whose qubit set, added to the block's, lets the most gates
// join the block without adding further qubits (the closure: gates inside the
// set that become ready one after another), ties to the earliest.  On the
// 30-qubit layered recipe this takes 319 five-qubit blocks where scoring by
// the upcoming gates of a fixed look-ahead window took 360.
std::vector<FBlock> plan_blocks(const std::vector<FGate>& gates, int kmax) {
  const int N = (int)gates.size();
  std::vector<uint64_t> gm(N, 0);
  int nq = 0;
  for (int i = 0; i < N; ++i)
    for (int q : gates[i].qubits) {
      gm[i] |= 1ull << q;
      nq = std::max(nq, q + 1);
    }
  // per-qubit program-order queues: all gates, and the non-diagonal ones
  std::vector<std::vector<int>> onq(nq), ndq(nq);
  for (int i = 0; i < N; ++i)
    for (int q : gates[i].qubits) {
      onq[q].push_back(i);
      if (!gates[i].diag) ndq[q].push_back(i);
    }
  std::vector<size_t> head(nq, 0), nhead(nq, 0);
  std::vector<char> done(N, 0);
  // first unscheduled gate (all / non-diagonal) on q, or N when none is left
  auto front = [&](int q) {
    while (head[q] < onq[q].size() && done[onq[q][head[q]]]) ++head[q];
    return head[q] < onq[q].size() ? onq[q][head[q]] : N;
  };
  auto nd_front = [&](int q) {
    while (nhead[q] < ndq[q].size() && done[ndq[q][nhead[q]]]) ++nhead[q];
    return nhead[q] < ndq[q].size() ? ndq[q][nhead[q]] : N;
  };
  auto ready = [&](int i) {
    for (int q : gates[i].qubits)
      if (gates[i].diag ? nd_front(q) < i : front(q) != i) return false;
    return true;
  };
  const int kDiagScan = 8;   // diagonal gates looked at behind the first unscheduled gate of a qubit
  // readiness against tentative marks too (done != 0), without moving the heads
  auto ready_scan = [&](int i) {
    for (int q : gates[i].qubits)
      for (size_t p = head[q]; p < onq[q].size(); ++p) {
        const int j = onq[q][p];
        if (j == i) break;
        if (done[j]) continue;
        if (gates[i].diag && gates[j].diag) continue;
        return false;
      }
    return true;
  };
  // gates that could join a block of qubit set s2 without new qubits (marked
  // tentatively while counting, then unmarked)
  std::vector<int> marked;
  auto closure = [&](uint64_t s2) {
    marked.clear();
    for (bool changed = true; changed;) {
      changed = false;
      for (int q = 0; q < nq; ++q) {
        if (!((s2 >> q) & 1)) continue;
        for (size_t p = head[q]; p < onq[q].size(); ++p) {
          const int i = onq[q][p];
          if (done[i]) continue;
          if ((gm[i] & ~s2) == 0 && ready_scan(i)) {
            done[i] = 2;
            marked.push_back(i);
            changed = true;
          } else if (!gates[i].diag) {
            break;
          }
        }
      }
    }
    for (int i : marked) done[i] = 0;
    return (long)marked.size();
  };
  std::vector<FBlock> out;
  std::vector<double> bre, bim, tre, tim;   // block matrix being composed (real, imaginary) and row scratch
  int first = 0;   // earliest unscheduled gate
  std::vector<int> cand;
  while (true) {
    while (first < N && done[first]) ++first;
    if (first >= N) break;
    FBlock blk;
    blk.ngates = 0;
    blk.diag = true;
    uint64_t smask = 0;
    std::vector<int> members;
    while (true) {
      // ready gates: the first unscheduled gate of some qubit, and the
      // diagonal gates right behind it on that qubit
      cand.clear();
      for (int q = 0; q < nq; ++q) {
        if (front(q) >= N) continue;
        int seen = 0;
        for (size_t p = head[q]; p < onq[q].size() && seen <= kDiagScan; ++p) {
          const int i = onq[q][p];
          if (done[i]) continue;
          ++seen;
          if (seen > 1 && !gates[i].diag) break;
          if (__builtin_popcountll(smask | gm[i]) > kmax || !ready(i)) {
            if (!gates[i].diag) break;
            continue;
          }
          if (std::find(cand.begin(), cand.end(), i) == cand.end()) cand.push_back(i);
          if (!gates[i].diag) break;
        }
      }
      if (cand.empty()) break;
      int pick = -1;
      for (int i : cand)   // no growth first, earliest
        if ((gm[i] & ~smask) == 0 && (pick < 0 || i < pick)) pick = i;
      if (pick < 0) {
        bool have = false;
        long best = 0;
        for (int i : cand) {
          const long score = closure(smask | gm[i]) * 8 - __builtin_popcountll(gm[i] & ~smask);
          if (!have || score > best || (score == best && i < pick)) {
            have = true;
            best = score;
            pick = i;
          }
        }
      }
      smask |= gm[pick];
      members.push_back(pick);
      done[pick] = 1;
    }
    for (int q = 0; q < 64; ++q)
      if ((smask >> q) & 1) blk.qubits.push_back(q);
    const int kb = (int)blk.qubits.size();
    const int Db = 1 << kb;
    bre.assign((size_t)Db * Db, 0.0);
    bim.assign((size_t)Db * Db, 0.0);
    for (int r = 0; r < Db; ++r) bre[(size_t)r * Db + r] = 1.0;
    blk.members = members;
    for (int i : members) {
      left_multiply(bre, bim, tre, tim, blk.qubits, gates[i]);
      blk.ngates++;
      blk.diag = blk.diag && gates[i].diag;
    }
    blk.m.resize((size_t)Db * Db);
    for (size_t e = 0; e < blk.m.size(); ++e) blk.m[e] = cd(bre[e], bim[e]);
    out.push_back(std::move(blk));
  }
  return out;
}

}  // namespace qk
