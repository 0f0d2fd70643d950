// Host-side network build (runs once per network).
#include "netbuild.h"

#include <algorithm>
#include <cstdint>
#include <cmath>
#include <cstring>
#include <map>
#include <numeric>
#include <queue>

#include "../../include/astrochem.h"

namespace ac {

std::vector<int32_t> species_order(int ns, const std::vector<int32_t> &row_ptr,
                                   const std::vector<int32_t> &col, int nr, int ordering) {
  std::vector<int32_t> perm(ns);
  std::iota(perm.begin(), perm.end(), 0);
  if (ordering == AC_ORDER_NNZ_DESC) {
    // Sec. 3: rows reordered by their number of nonzeros; most first, ties
    // kept in natural order.
    std::stable_sort(perm.begin(), perm.end(), [&](int a, int b) {
      return (row_ptr[a + 1] - row_ptr[a]) > (row_ptr[b + 1] - row_ptr[b]);
    });
  } else if (ordering == AC_ORDER_RCM) {
    // Species graph: two species are adjacent when they share a reaction
    // (the off-diagonal pattern of S S^T).
    std::vector<std::vector<int32_t>> by_rx(nr);
    for (int i = 0; i < ns; ++i)
      for (int p = row_ptr[i]; p < row_ptr[i + 1]; ++p) by_rx[col[p]].push_back(i);
    std::vector<std::vector<int32_t>> adj(ns);
    for (int j = 0; j < nr; ++j)
      for (int a : by_rx[j])
        for (int b : by_rx[j])
          if (a != b) adj[a].push_back(b);
    for (auto &v : adj) {
      std::sort(v.begin(), v.end());
      v.erase(std::unique(v.begin(), v.end()), v.end());
    }
    std::vector<int> deg(ns);
    for (int i = 0; i < ns; ++i) deg[i] = int(adj[i].size());
    std::vector<char> seen(ns, 0);
    std::vector<int32_t> order;
    order.reserve(ns);
    auto bfs_levels = [&](int root, std::vector<int> &level) {
      level.assign(ns, -1);
      std::queue<int> q;
      q.push(root);
      level[root] = 0;
      int last = root;
      while (!q.empty()) {
        int u = q.front();
        q.pop();
        last = u;
        for (int v : adj[u])
          if (level[v] < 0) {
            level[v] = level[u] + 1;
            q.push(v);
          }
      }
      return last;
    };
    for (;;) {
      // start each component at a minimum-degree node, then move to a
      // pseudo-peripheral node (farthest level, minimum degree) a few times
      int root = -1;
      for (int i = 0; i < ns; ++i)
        if (!seen[i] && (root < 0 || deg[i] < deg[root])) root = i;
      if (root < 0) break;
      std::vector<int> level;
      int ecc = -1;
      for (int it = 0; it < 8; ++it) {
        bfs_levels(root, level);
        int maxl = 0;
        for (int i = 0; i < ns; ++i)
          if (!seen[i] && level[i] > maxl) maxl = level[i];
        if (maxl <= ecc) break;
        ecc = maxl;
        int cand = root;
        for (int i = 0; i < ns; ++i)
          if (!seen[i] && level[i] == maxl && (cand == root || deg[i] < deg[cand])) cand = i;
        if (cand == root) break;
        root = cand;
      }
      // Cuthill-McKee from root: neighbours by increasing degree
      std::queue<int> q;
      q.push(root);
      seen[root] = 1;
      while (!q.empty()) {
        int u = q.front();
        q.pop();
        order.push_back(u);
        std::vector<int> nb;
        for (int v : adj[u])
          if (!seen[v]) nb.push_back(v);
        std::stable_sort(nb.begin(), nb.end(), [&](int a, int b) { return deg[a] < deg[b]; });
        for (int v : nb) {
          seen[v] = 1;
          q.push(v);
        }
      }
    }
    std::reverse(order.begin(), order.end());
    perm = order;
  }
  return perm;
}

void build_schedule(const std::vector<std::vector<uint32_t>> &seg_items,
                    const std::vector<int32_t> &order, int chunk, int sell_c, int sell_sigma,
                    Schedule &s) {
  s = Schedule();
  s.chunk = chunk;
  s.n_seg = int(order.size());
  s.seg_out = order;
  s.seg_chunk.push_back(0);
  s.chunk_ptr.push_back(0);
  s.multi_slot.push_back(0);
  for (int k = 0; k < s.n_seg; ++k) {
    const auto &it = seg_items[order[k]];
    const int n = int(it.size());
    const int nch = n == 0 ? 1 : (n + chunk - 1) / chunk;
    for (int c = 0; c < nch; ++c) {
      const int p = c * chunk, e = std::min(n, p + chunk);
      for (int q = p; q < e; ++q) {
        s.items.push_back(it[q]);
        s.coo_out.push_back(order[k]);
      }
      s.chunk_ptr.push_back(int32_t(s.items.size()));
      s.chunk_dst.push_back(nch == 1 ? order[k] : -1 - s.n_slot++);
    }
    if (nch > 1) {
      s.multi_out.push_back(order[k]);
      s.multi_slot.push_back(s.n_slot);
    }
    s.seg_chunk.push_back(int32_t(s.chunk_ptr.size() - 1));
  }
  s.n_multi = int(s.multi_out.size());
  s.n_chunk = int(s.chunk_ptr.size() - 1);
  s.n_item = int(s.items.size());

  // equal runs of RUN_LEN items over the whole list (merge-style partition:
  // every lane gets the same amount of work whatever the segment lengths)
  s.n_run = (s.n_item + RUN_LEN - 1) / RUN_LEN;
  s.run_mask.assign(s.n_run, 0u);
  s.run_slot.assign(s.n_run, 0);
  s.seg_run.assign(size_t(2) * s.n_seg, 0);
  {
    std::vector<int32_t> seg_of(s.n_item);
    for (int k = 0; k < s.n_seg; ++k)
      for (int q = s.chunk_ptr[s.seg_chunk[k]]; q < s.chunk_ptr[s.seg_chunk[k + 1]]; ++q) seg_of[q] = k;
    int slot = 0;
    for (int t = 0; t < s.n_run; ++t) {
      s.run_slot[t] = slot;
      for (int k = 0; k < RUN_LEN; ++k) {
        const int i = t * RUN_LEN + k;
        if (i >= s.n_item) break;
        if (k == 0 || seg_of[i] != seg_of[i - 1]) {
          s.run_mask[t] |= 1u << k;
          const int g = seg_of[i];
          if (s.seg_run[2 * g + 1] == 0) s.seg_run[2 * g] = slot;
          ++s.seg_run[2 * g + 1];
          ++slot;
        }
      }
    }
    s.n_rslot = slot;
  }
  const uint32_t pad_item = pack_item(0, -1, 0);
  {
    const int nblk = (s.n_run + 63) / 64;
    s.run_items.assign(size_t(nblk) * 64 * RUN_LEN, pad_item);
    for (int t = 0; t < s.n_run; ++t) {
      const int blk = t / 64, l = t % 64;
      for (int k = 0; k < RUN_LEN; ++k) {
        const int i = t * RUN_LEN + k;
        if (i >= s.n_item) break;
        const size_t w = (size_t(blk) * (RUN_LEN / 4) + k / 4) * 64 + l;
        s.run_items[w * 4 + k % 4] = s.items[i];
      }
    }
  }

  // SELL-C-sigma: positions are chunk ids sorted by length (descending,
  // stable) inside windows of sigma chunks, grouped into slices of C.
  s.sell_c = sell_c;
  s.sell_sigma = sell_sigma;
  std::vector<int32_t> pos(s.n_chunk);
  std::iota(pos.begin(), pos.end(), 0);
  auto clen = [&](int c) { return s.chunk_ptr[c + 1] - s.chunk_ptr[c]; };
  for (int w = 0; w < s.n_chunk; w += sell_sigma) {
    const int e = std::min(s.n_chunk, w + sell_sigma);
    std::stable_sort(pos.begin() + w, pos.begin() + e,
                     [&](int a, int b) { return clen(a) > clen(b); });
  }
  s.n_slice = (s.n_chunk + sell_c - 1) / sell_c;
  s.slice_ptr.assign(1, 0);
  s.sell_chunk.assign(size_t(s.n_slice) * sell_c, -1);
  s.sell_len.assign(size_t(s.n_slice) * sell_c, 0);
  s.sell_dst.assign(size_t(s.n_slice) * sell_c, INT32_MIN);
  for (int sl = 0; sl < s.n_slice; ++sl) {
    int width = 0;
    for (int l = 0; l < sell_c; ++l) {
      const int p = sl * sell_c + l;
      if (p < s.n_chunk) {
        s.sell_chunk[p] = pos[p];
        s.sell_len[p] = clen(pos[p]);
        s.sell_dst[p] = s.chunk_dst[pos[p]];
        width = std::max(width, s.sell_len[p]);
      }
    }
    for (int k = 0; k < width; ++k)
      for (int l = 0; l < sell_c; ++l) {
        const int p = sl * sell_c + l;
        uint32_t v = pack_item(0, -1, 0);
        if (p < s.n_chunk && k < s.sell_len[p]) v = s.items[s.chunk_ptr[pos[p]] + k];
        s.sell_items.push_back(v);
      }
    s.slice_ptr.push_back(int32_t(s.sell_items.size()));
  }
}

std::string build_network(int ns, int nr, const int32_t *reactants, const int32_t *products,
                          const double *alpha, const double *beta, const double *gamma,
                          const int8_t *law, const int8_t *composition, int n_elem,
                          bool check_balance, int layout, int ordering, int chunk, int sell_c,
                          int sell_sigma, HostNet &H, int *code) {
  *code = AC_EINVAL;
  if (ns <= 0 || nr <= 0) return "n_species and n_reactions must be positive";
  if (ns > AC_MAX_SPECIES || nr > AC_MAX_REACTIONS) {
    *code = AC_ELIMIT;
    return "network larger than AC_MAX_SPECIES / AC_MAX_REACTIONS";
  }
  if (!reactants || !products || !alpha || !beta || !gamma) return "null network array";
  if (layout < 0 || layout > 4) return "unknown layout";
  if (ordering < 0 || ordering > 2) return "unknown ordering";
  if (chunk < 0 || sell_c < 0 || sell_sigma < 0) return "negative chunk/sell parameter";
  chunk = chunk ? chunk : 32;
  if (sell_c != 0 && sell_c != 64) return "sell_c must be 64 (one wavefront per slice)";
  sell_c = 64;
  sell_sigma = sell_sigma ? sell_sigma : (1 << 30);
  if (check_balance && (!composition || n_elem <= 0)) return "balance check needs a composition";

  H = HostNet();
  H.ns = ns;
  H.nr = nr;
  H.layout = layout;
  H.ordering = ordering;
  H.log_alpha.resize(nr);
  H.beta.assign(beta, beta + nr);
  H.gamma.assign(gamma, gamma + nr);
  if (law) H.law.assign(law, law + nr);
  H.rpair.resize(nr);
  // net stoichiometry per reaction (sorted by species)
  std::vector<std::map<int, int>> col(nr);
  for (int j = 0; j < nr; ++j) {
    if (!(alpha[j] > 0.0) || !std::isfinite(alpha[j]) || !std::isfinite(beta[j]) ||
        !std::isfinite(gamma[j]))
      return "reaction " + std::to_string(j) + ": alpha must be positive and finite, beta/gamma finite";
    H.log_alpha[j] = std::log(alpha[j]);
    if (law && (law[j] < AC_LAW_KOOIJ || law[j] > AC_LAW_PHOTO))
      return "reaction " + std::to_string(j) + ": unknown rate law";
    if (law && law[j] == AC_LAW_CRPHOT && !(gamma[j] > 0.0))
      return "reaction " + std::to_string(j) + ": cosmic-ray photon efficiency gamma must be > 0";
    int nreac = 0, slot[2] = {-1, -1};
    for (int s = 0; s < AC_MAX_REACTANTS; ++s) {
      int a = reactants[j * AC_MAX_REACTANTS + s];
      if (a < -1 || a >= ns) return "reaction " + std::to_string(j) + ": reactant index out of range";
      if (a >= 0) {
        slot[nreac++] = a;
        col[j][a] -= 1;
      }
    }
    if (nreac == 0) return "reaction " + std::to_string(j) + ": no reactant";
    for (int s = 0; s < AC_MAX_PRODUCTS; ++s) {
      int p = products[j * AC_MAX_PRODUCTS + s];
      if (p < -1 || p >= ns) return "reaction " + std::to_string(j) + ": product index out of range";
      if (p >= 0) col[j][p] += 1;
    }
    H.rpair[j] = uint32_t(slot[0]) | (uint32_t(slot[1] < 0 ? 0xFFFF : slot[1]) << 16);
  }
  if (check_balance) {
    for (int j = 0; j < nr; ++j)
      for (int e = 0; e < n_elem; ++e) {
        long tot = 0;
        for (auto &kv : col[j]) tot += long(kv.second) * composition[size_t(kv.first) * n_elem + e];
        if (tot != 0) {
          *code = AC_EUNBALANCED;
          return "reaction " + std::to_string(j) + " does not conserve element/charge " +
                 std::to_string(e);
        }
      }
  }
  // CSR and CCS of the net S (zero entries dropped)
  std::vector<std::vector<std::pair<int, int>>> rows(ns);
  H.s_col_ptr.assign(1, 0);
  for (int j = 0; j < nr; ++j) {
    for (auto &kv : col[j])
      if (kv.second != 0) {
        rows[kv.first].push_back({j, kv.second});
        H.s_row.push_back(kv.first);
        H.s_cval.push_back(kv.second);
      }
    H.s_col_ptr.push_back(int32_t(H.s_row.size()));
  }
  H.s_row_ptr.assign(1, 0);
  for (int i = 0; i < ns; ++i) {
    for (auto &e : rows[i]) {
      H.s_col.push_back(e.first);
      H.s_val.push_back(e.second);
    }
    H.s_row_ptr.push_back(int32_t(H.s_col.size()));
  }
  H.perm = species_order(ns, H.s_row_ptr, H.s_col, nr, ordering);

  // RHS rows: dydt_i = sum_j S_ij R_j
  std::vector<std::vector<uint32_t>> seg(ns);
  for (int i = 0; i < ns; ++i)
    for (auto &e : rows[i]) seg[i].push_back(pack_item(e.first, -1, e.second));
  build_schedule(seg, H.perm, chunk, sell_c, sell_sigma, H.rhs);

  // Jacobian: for each reactant species a of reaction j, dR_j/dn_a =
  // mult * k_j * n_b (b the other reactant, none for one-body, mult 2 for
  // A + A); entry (i, a) collects S_ij * that.
  std::vector<std::map<int, std::vector<uint32_t>>> jrow(ns);
  std::vector<std::vector<uint32_t>> gyseg(ns);
  for (int j = 0; j < nr; ++j) {
    const int a0 = int(H.rpair[j] & 0xFFFF), b0 = int(H.rpair[j] >> 16);
    const int a1 = b0 == 0xFFFF ? -1 : b0;
    struct D { int a, other, mult; };
    D d[2];
    int nd = 0;
    if (a1 < 0) d[nd++] = {a0, -1, 1};
    else if (a1 == a0) d[nd++] = {a0, a0, 2};
    else {
      d[nd++] = {a0, a1, 1};
      d[nd++] = {a1, a0, 1};
    }
    for (int q = 0; q < nd; ++q) {
      gyseg[d[q].a].push_back(pack_item(j, d[q].other, d[q].mult));
      for (auto &kv : col[j])
        if (kv.second != 0)
          jrow[kv.first][d[q].a].push_back(pack_item(j, d[q].other, kv.second * d[q].mult));
    }
  }
  H.j_row_ptr.assign(1, 0);
  std::vector<std::vector<uint32_t>> jseg;
  std::vector<int32_t> &entry_row = H.jent_row;
  for (int i = 0; i < ns; ++i) {
    for (auto &kv : jrow[i]) {
      H.j_col.push_back(kv.first);
      jseg.push_back(kv.second);
      entry_row.push_back(i);
    }
    H.j_row_ptr.push_back(int32_t(H.j_col.size()));
  }
  // Jacobian entries traversed row by row in the species order
  std::vector<int32_t> jorder;
  jorder.reserve(H.j_col.size());
  for (int k = 0; k < ns; ++k)
    for (int e = H.j_row_ptr[H.perm[k]]; e < H.j_row_ptr[H.perm[k] + 1]; ++e) jorder.push_back(e);
  // Jacobian and VJP term lists keep their natural chunk order in SELL
  // (sigma = 1), so consecutive lanes write consecutive outputs
  build_schedule(jseg, jorder, chunk, sell_c, 1, H.jac);
  {
    const size_t ne = jseg.size();
    const uint32_t pad = pack_item(0, -1, 0);
    H.jhead0.assign(ne, pad);
    H.jhead1.assign(ne, pad);
    H.jtaildesc.assign(ne, 0u);
    std::vector<std::vector<uint32_t>> tails(ne);
    std::vector<int32_t> tail_order;
    for (size_t e = 0; e < ne; ++e) {
      const auto &t = jseg[e];
      if (t.size() > 0) H.jhead0[e] = t[0];
      if (t.size() > 1) H.jhead1[e] = t[1];
      if (t.size() > 2) {
        tails[e].assign(t.begin() + 2, t.end());
        tail_order.push_back(int32_t(e));
      }
    }
    build_schedule(tails, tail_order, chunk, sell_c, 1 << 30, H.jtail);
    // tail partials come from equal runs (RUN_LEN terms per lane); an entry
    // adds its consecutive run partials
    for (int k = 0; k < H.jtail.n_seg; ++k) {
      const int e = H.jtail.seg_out[k];
      const int first = H.jtail.seg_run[2 * k], cnt = H.jtail.seg_run[2 * k + 1];
      if (cnt > 255 || first >= (1 << 24)) return "Jacobian entry with too many terms";
      H.jtaildesc[e] = (uint32_t(first) << 8) | uint32_t(cnt);
    }
    H.jtail.n_slot = H.jtail.n_rslot;
    H.jtail.n_multi = 0;
    H.jtail.multi_out.clear();
    H.jtail.multi_slot.assign(1, 0);
  }
  build_schedule(gyseg, H.perm, chunk, sell_c, 1 << 30, H.gy);
  // packed per-reaction records (see HostNet::rxpack), three planes of nr
  // 16-byte words so that consecutive reactions are contiguous
  H.rxpack.assign(size_t(nr) * 12, 0u);
  for (int j = 0; j < nr; ++j) {
    uint32_t *p0 = &H.rxpack[size_t(j) * 4];
    uint32_t *p1 = &H.rxpack[(size_t(nr) + j) * 4];
    uint32_t *p2 = &H.rxpack[(size_t(2) * nr + j) * 4];
    // every law as ln k = ln alpha + beta' ln(T/300) - gamma' X + Y, with X
    // and Y per-cell terms chosen by the law (devchem.h rate_k)
    const int lw = H.law.empty() ? AC_LAW_KOOIJ : H.law[j];
    double b2 = H.beta[j], g2 = H.gamma[j];
    if (lw == AC_LAW_CRP) {
      b2 = 0.0;
      g2 = 0.0;
    } else if (lw == AC_LAW_CRPHOT) {
      g2 = -std::log(H.gamma[j] / (1.0 - AC_GRAIN_ALBEDO));   // X = 1
    } else if (lw == AC_LAW_PHOTO) {
      b2 = 0.0;
    }
    const double la_b[2] = {H.log_alpha[j], b2};
    std::memcpy(p0, la_b, sizeof(la_b));
    std::memcpy(p1, &g2, sizeof(double));
    p1[2] = H.rpair[j];
    p1[3] = uint32_t(lw);
    uint16_t half[8];
    for (int q = 0; q < 8; ++q) half[q] = 0xFFFF;
    int q = 0;
    for (int p = H.s_col_ptr[j]; p < H.s_col_ptr[j + 1]; ++p)
      half[q++] = uint16_t(H.s_row[p] | ((H.s_cval[p] & 31) << 11));
    std::memcpy(p2, half, sizeof(half));
  }
  H.front = build_front_plan(ns, H.j_row_ptr, H.j_col, newton_region_doubles(ns));
  H.front_th = build_front_plan_thermal(ns, H.j_row_ptr, H.j_col, newton_region_doubles(ns));
  *code = AC_OK;
  return "";
}

}  // namespace ac
