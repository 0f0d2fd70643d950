// Plan of the sparse-front / dense-tail Newton solve (see frontlu.h).
#include "frontlu.h"

#include <algorithm>
#include <climits>
#include <numeric>

namespace ac {

namespace {

// Square bit matrix with row and column views kept in step.
struct BitMat {
  int n = 0, w = 0;
  std::vector<uint64_t> r, c;   // r[i*w + j/64] bit j: entry (i, j); c the transpose
  explicit BitMat(int n_) : n(n_), w((n_ + 63) / 64), r(size_t(n_) * w, 0), c(size_t(n_) * w, 0) {}
  bool get(int i, int j) const { return (r[size_t(i) * w + j / 64] >> (j % 64)) & 1u; }
  void set(int i, int j) {
    r[size_t(i) * w + j / 64] |= uint64_t(1) << (j % 64);
    c[size_t(j) * w + i / 64] |= uint64_t(1) << (i % 64);
  }
  std::vector<int> row(int i) const { return bits(&r[size_t(i) * w]); }
  std::vector<int> colv(int j) const { return bits(&c[size_t(j) * w]); }
  std::vector<int> bits(const uint64_t *p) const {
    std::vector<int> out;
    for (int q = 0; q < w; ++q)
      for (uint64_t v = p[q]; v; v &= v - 1) out.push_back(q * 64 + __builtin_ctzll(v));
    return out;
  }
  // The structural effect of sweeping pivot k: every (i, j) with (i, k)
  // and (k, j) present becomes present (i, j != k).
  void sweep(int k, long long *ops) {
    std::vector<uint64_t> rb(&c[size_t(k) * w], &c[size_t(k) * w] + w);
    std::vector<uint64_t> cb(&r[size_t(k) * w], &r[size_t(k) * w] + w);
    rb[k / 64] &= ~(uint64_t(1) << (k % 64));
    cb[k / 64] &= ~(uint64_t(1) << (k % 64));
    const std::vector<int> rows = bits(rb.data()), cols = bits(cb.data());
    if (ops) *ops += (long long)rows.size() * (long long)cols.size();
    for (int i : rows)
      for (int q = 0; q < w; ++q) r[size_t(i) * w + q] |= cb[q];
    for (int j : cols)
      for (int q = 0; q < w; ++q) c[size_t(j) * w + q] |= rb[q];
  }
};

// Minimum-degree order on the symmetric pattern G (explicit elimination
// graph; ties go to the smaller index).
std::vector<int> min_degree(int n, const BitMat &P) {
  const int w = P.w;
  std::vector<uint64_t> G(size_t(n) * w), alive(w, 0);
  for (int i = 0; i < n; ++i)
    for (int q = 0; q < w; ++q) G[size_t(i) * w + q] = P.r[size_t(i) * w + q] | P.c[size_t(i) * w + q];
  for (int i = 0; i < n; ++i) alive[i / 64] |= uint64_t(1) << (i % 64);
  std::vector<int> order;
  order.reserve(n);
  std::vector<uint64_t> nb(w);
  for (int step = 0; step < n; ++step) {
    int best = -1, bd = INT_MAX;
    for (int i = 0; i < n; ++i) {
      if (!((alive[i / 64] >> (i % 64)) & 1u)) continue;
      int d = 0;
      for (int q = 0; q < w; ++q) d += __builtin_popcountll(G[size_t(i) * w + q] & alive[q]);
      if (d < bd) {
        bd = d;
        best = i;
      }
    }
    order.push_back(best);
    alive[best / 64] &= ~(uint64_t(1) << (best % 64));
    for (int q = 0; q < w; ++q) nb[q] = G[size_t(best) * w + q] & alive[q];
    for (int q = 0; q < w; ++q)
      for (uint64_t v = nb[q]; v; v &= v - 1) {
        const int i = q * 64 + __builtin_ctzll(v);
        for (int t = 0; t < w; ++t) G[size_t(i) * w + t] |= nb[t];
      }
  }
  return order;
}

BitMat permuted_pattern(int n, const std::vector<int32_t> &rp, const std::vector<int32_t> &col,
                        const std::vector<int> &pos) {
  BitMat P(n);
  for (int i = 0; i < n; ++i) {
    P.set(pos[i], pos[i]);
    for (int e = rp[i]; e < rp[i + 1]; ++e) P.set(pos[i], pos[col[e]]);
  }
  return P;
}

// Modelled time of one factorisation and the solves that reuse it: the
// integrator solves about 28 times per factorisation (3 Newton iterations
// per step, a factorisation every 9 steps); solves stream the dense factors
// and the sparse values (2.8 TB/s with every slot busy), the dense LU runs
// at 7.8 TFLOP/s over all slots, a sweep update costs about 20 ps of the
// chip's time.
double model_cost(int n2, long long nv, long long ops) {
  const double solve_bytes = 8.0 * double(n2) * n2 + 8.0 * double(nv);
  return 28.0 * solve_bytes / 2.8e12 + (2.0 / 3.0) * double(n2) * n2 * n2 / 7.8e12 + double(ops) * 2e-11;
}

// The front's fixed latency per factorisation cycle, in the same chip time:
// each solve adds about six dependent rounds (permutations, two gathers
// and their sums, about 1 us each), each sweep level three; a workgroup
// waits for them alone, so they cost the chip 1/64 of that time (a
// quarter of the slots in that state at once).
double front_overhead(int n_lev) {
  return (28.0 * 6.0 + 3.0 * n_lev + 4.0) * 1e-6 / 64.0;
}

int round16(int x) { return (x + 15) / 16 * 16; }
int vofs_of(int n2) { return (n2 * round16(n2) + 31) / 32 * 32; }

// Greedy levels of the first n1 pivots of the minimum-degree order:
// lev_ptr (starting {0}) gets the level boundaries, order the md
// positions in sweep order.
void front_order_of(int n, const std::vector<int32_t> &j_row_ptr, const std::vector<int32_t> &j_col,
                    const std::vector<int> &md_pos, int n1, std::vector<int32_t> &lev_ptr,
                    std::vector<int> &front_order) {
  front_order.clear();
  BitMat Fm = permuted_pattern(n, j_row_ptr, j_col, md_pos);
  std::vector<char> done(n1, 0);
  int left = n1;
  while (left > 0) {
    std::vector<int> lev;
    for (int k = 0; k < n1; ++k) {
      if (done[k]) continue;
      bool ok = true;
      for (int m : lev)
        if (Fm.get(k, m) || Fm.get(m, k)) {
          ok = false;
          break;
        }
      if (ok) lev.push_back(k);
    }
    for (int k : lev) {
      Fm.sweep(k, nullptr);
      done[k] = 1;
      front_order.push_back(k);
    }
    left -= int(lev.size());
    lev_ptr.push_back(int(front_order.size()));
  }
}

}  // namespace

FrontPlan build_front_plan(int n, const std::vector<int32_t> &j_row_ptr,
                           const std::vector<int32_t> &j_col, size_t max_doubles) {
  FrontPlan F;
  F.n = n;
  if (n <= 0) return F;
  std::vector<int> ident(n);
  std::iota(ident.begin(), ident.end(), 0);
  const BitMat P0 = permuted_pattern(n, j_row_ptr, j_col, ident);
  const std::vector<int> md = min_degree(n, P0);
  std::vector<int> md_pos(n);
  for (int p = 0; p < n; ++p) md_pos[md[p]] = p;

  // Cost of every front size: sweep the minimum-degree order and count,
  // before each pivot, the values in front rows / columns and the updates.
  int best_n1 = 0;
  {
    BitMat Fm = permuted_pattern(n, j_row_ptr, j_col, md_pos);
    long long ops = 0;
    double best = 0.0;
    std::vector<uint64_t> lt(Fm.w, 0);   // bits j < k
    for (int k = 0; k <= n; ++k) {
      long long nv = 0;
      for (int i = 0; i < n; ++i) {
        const uint64_t *ri = &Fm.r[size_t(i) * Fm.w];
        for (int q = 0; q < Fm.w; ++q) nv += __builtin_popcountll(i < k ? ri[q] : (ri[q] & lt[q]));
      }
      const int n2 = n - k;
      const double cst = model_cost(n2, nv, ops);
      // the values fit the slot's region, and every gather's pieces (at most
      // nv / FRONT_PIECE + n) fit the solves' LDS block
      const bool fits = size_t(vofs_of(n2)) + size_t(nv) <= max_doubles &&
                        nv / FRONT_PIECE + n <= FRONT_MAX_PIECES;
      if (k == 0) {
        best = cst;
        F.cost_dense = cst;
      } else if (fits && cst < best) {
        best = cst;
        best_n1 = k;
      }
      if (k == n) break;
      Fm.sweep(k, &ops);
      lt[k / 64] |= uint64_t(1) << (k % 64);
    }
    F.cost_front = best;
  }

  // Levels: greedy maximal sets of front pivots that share no entry, in
  // minimum-degree order, each set swept before the next is chosen. A
  // front that does not save more than its fixed latency is dropped (n1 =
  // 0: the whole matrix is factored densely).
  int n1 = best_n1;
  std::vector<int> front_order;   // md positions in sweep order
  for (;;) {
    F.lev_ptr.assign(1, 0);
    front_order_of(n, j_row_ptr, j_col, md_pos, n1, F.lev_ptr, front_order);
    const int n_lev = int(F.lev_ptr.size()) - 1;
    if (n1 == 0 || F.cost_front + front_overhead(n_lev) < F.cost_dense) break;
    n1 = 0;
    F.cost_front = F.cost_dense;
  }
  if (n1 > 0) F.cost_front += front_overhead(int(F.lev_ptr.size()) - 1);
  F.n1 = n1;
  F.n2 = n - n1;
  F.n_lev = int(F.lev_ptr.size()) - 1;
  F.lda2 = round16(F.n2);
  F.vofs = vofs_of(F.n2);

  // final positions: the front in sweep order, then the tail in md order
  F.perm.resize(n);
  for (int p = 0; p < n1; ++p) F.perm[p] = md[front_order[p]];
  for (int p = n1; p < n; ++p) F.perm[p] = md[p];
  std::vector<int> pos(n);
  for (int p = 0; p < n; ++p) pos[F.perm[p]] = p;

  // Sweep in the final order, recording each level's products.
  BitMat Fs = permuted_pattern(n, j_row_ptr, j_col, pos);
  struct Op { int i, j, k, seq; };
  std::vector<std::vector<Op>> lev_ops(F.n_lev);
  for (int l = 0; l < F.n_lev; ++l) {
    int seq = 0;
    for (int k = F.lev_ptr[l]; k < F.lev_ptr[l + 1]; ++k) {
      std::vector<int> rows = Fs.colv(k), cols = Fs.row(k);
      for (int i : rows)
        if (i != k)
          for (int j : cols)
            if (j != k) lev_ops[l].push_back({i, j, k, seq++});
    }
    for (int k = F.lev_ptr[l]; k < F.lev_ptr[l + 1]; ++k) Fs.sweep(k, nullptr);
  }

  // Sparse values: front rows in full, tail rows at front columns.
  std::vector<int32_t> idx(size_t(n) * n, -1);
  F.row_ptr.assign(n + 1, 0);
  for (int i = 0; i < n; ++i) {
    for (int j : Fs.row(i))
      if (i < n1 || j < n1) {
        idx[size_t(i) * n + j] = int(F.col.size());
        F.col.push_back(j);
      }
    F.row_ptr[i + 1] = int(F.col.size());
  }
  F.nv = int(F.col.size());
  F.rsplit.resize(n1);
  F.vdiag.resize(n1);
  for (int k = 0; k < n1; ++k) {
    int q = F.row_ptr[k];
    while (q < F.row_ptr[k + 1] && F.col[q] < n1) ++q;
    F.rsplit[k] = q;
    F.vdiag[k] = idx[size_t(k) * n + k];
  }
  F.cptr.assign(n + 1, 0);
  for (int j = 0; j < n; ++j) {
    for (int i : Fs.colv(j))
      if (idx[size_t(i) * n + j] >= 0) {
        F.crow.push_back(i);
        F.cidx.push_back(idx[size_t(i) * n + j]);
      }
    F.cptr[j + 1] = int(F.crow.size());
  }
  F.csplit.resize(n1);
  for (int k = 0; k < n1; ++k) {
    int q = F.cptr[k];
    while (q < F.cptr[k + 1] && F.crow[q] < n1) ++q;
    F.csplit[k] = q;
  }
  auto code = [&](int i, int j) {
    if (i < n1 || j < n1) return idx[size_t(i) * n + j];
    return -(1 + (i - n1) * F.lda2 + (j - n1));
  };
  F.asm_dst.resize(j_col.size());
  for (int r = 0; r < n; ++r)
    for (int e = j_row_ptr[r]; e < j_row_ptr[r + 1]; ++e) F.asm_dst[e] = code(pos[r], pos[j_col[e]]);

  // Pieces of the solves' four sparse products.
  F.gseg.assign(size_t(4) * (n + 1), 0);
  for (int g = 0; g < 4; ++g) {
    F.gbase[g] = int(F.gpc.size() / 2);
    int32_t *seg = &F.gseg[size_t(g) * (n + 1)];
    seg[0] = F.gbase[g];
    for (int r = 0; r < n; ++r) {
      int b = 0, e = 0;
      const bool fr = r < n1;
      if (g == 0) { b = F.row_ptr[r]; e = fr ? F.rsplit[r] : F.row_ptr[r + 1]; }
      if (g == 1 && fr) { b = F.rsplit[r]; e = F.row_ptr[r + 1]; }
      if (g == 2) { b = F.cptr[r]; e = fr ? F.csplit[r] : F.cptr[r + 1]; }
      if (g == 3 && fr) { b = F.csplit[r]; e = F.cptr[r + 1]; }
      for (int q = b; q < e; q += FRONT_PIECE) {
        F.gpc.push_back(q);
        F.gpc.push_back(std::min(e, q + FRONT_PIECE));
      }
      seg[r + 1] = int(F.gpc.size() / 2);
    }
  }
  F.gbase[4] = int(F.gpc.size() / 2);

  // Per level: targets, most products first; products in sweep order.
  F.tg_ptr.push_back(0);
  F.op_ptr.push_back(0);
  for (int l = 0; l < F.n_lev; ++l) {
    std::vector<Op> &v = lev_ops[l];
    std::stable_sort(v.begin(), v.end(), [](const Op &a, const Op &b) {
      return a.i != b.i ? a.i < b.i : a.j != b.j ? a.j < b.j : a.seq < b.seq;
    });
    std::vector<std::pair<size_t, size_t>> runs;   // [begin, end) per target
    for (size_t a = 0; a < v.size();) {
      size_t b = a;
      while (b < v.size() && v[b].i == v[a].i && v[b].j == v[a].j) ++b;
      runs.emplace_back(a, b);
      a = b;
    }
    std::stable_sort(runs.begin(), runs.end(), [](const std::pair<size_t, size_t> &a,
                                                  const std::pair<size_t, size_t> &b) {
      return a.second - a.first > b.second - b.first;
    });
    for (const auto &rg : runs) {
      F.tgt.push_back(code(v[rg.first].i, v[rg.first].j));
      for (size_t t = rg.first; t < rg.second; ++t) {
        F.ops.push_back(idx[size_t(v[t].i) * n + v[t].k]);
        F.ops.push_back(idx[size_t(v[t].k) * n + v[t].j]);
      }
      F.op_ptr.push_back(int(F.ops.size() / 2));
    }
    F.tg_ptr.push_back(int(F.tgt.size()));
  }
  return F;
}

FrontPlan build_front_plan_thermal(int ns, const std::vector<int32_t> &j_row_ptr,
                                   const std::vector<int32_t> &j_col, size_t max_doubles) {
  // augmented CSR: every species row gains the column T (= ns, last), then
  // the row T is full
  const int nnz = j_row_ptr[ns];
  std::vector<int32_t> rp(ns + 2), col;
  col.reserve(size_t(nnz) + 2 * size_t(ns) + 1);
  for (int r = 0; r < ns; ++r) {
    rp[r] = int32_t(col.size());
    for (int e = j_row_ptr[r]; e < j_row_ptr[r + 1]; ++e) col.push_back(j_col[e]);
    col.push_back(ns);
  }
  rp[ns] = int32_t(col.size());
  for (int a = 0; a <= ns; ++a) col.push_back(a);
  rp[ns + 1] = int32_t(col.size());
  FrontPlan F = build_front_plan(ns + 1, rp, col, max_doubles);
  if (F.n1 == 0) return F;
  const std::vector<int32_t> aug = F.asm_dst;
  F.asm_dst.resize(nnz);
  F.tcol_dst.resize(ns);
  F.trow_dst.resize(ns);
  for (int r = 0; r < ns; ++r) {
    for (int e = j_row_ptr[r]; e < j_row_ptr[r + 1]; ++e) F.asm_dst[e] = aug[size_t(e) + r];
    F.tcol_dst[r] = aug[size_t(j_row_ptr[r + 1]) + r];
  }
  for (int a = 0; a < ns; ++a) F.trow_dst[a] = aug[size_t(nnz) + ns + a];
  F.corner_dst = aug[size_t(nnz) + 2 * size_t(ns)];
  return F;
}

}  // namespace ac
