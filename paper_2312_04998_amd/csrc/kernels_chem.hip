// Rate coefficients, RHS, Jacobian and VJP kernels for gfx950.
//
// Mapping: one workgroup of NT threads (NT/64 wavefronts) works on one cell
// at a time and strides over cells. A cell's densities are staged in LDS
// with a coalesced load; the per-reaction quantities (rates R_j for the
// RHS, coefficients k_j for the Jacobian, k_j (S^T v)_j for the VJP) are
// computed once per cell into an LDS block; the product with S is then a
// gather over precomputed term lists (rows of S, entries of the Jacobian
// pattern, reactant slots of a species), split into short chunks so heavy
// rows (H, H2, e- take part in 15-30 % of reactions) are shared by many
// lanes. Network data (a few hundred KB) stays in L2 for all cells; every
// lane keeps several independent loads in flight because the walks are
// otherwise bound by L2 latency, not bandwidth.
#include "devchem.h"

namespace ac {

// ------------------------------------------------------------------ rates

template <int NT>
__global__ __launch_bounds__(NT) void k_rates(DNet n, const double *__restrict__ la_over,
                                              int64_t n_cells, const double *__restrict__ T,
                                              double *__restrict__ k) {
  for (int64_t c = blockIdx.x; c < n_cells; c += gridDim.x) {
    const Env env = cell_env(T, c, n.n_cond);
    double *kc = k + c * n.nr;
    for_reactions<NT>(n, la_over, env,
                      [&](int j, double kj, uint32_t) { __builtin_nontemporal_store(kj, kc + j); });
  }
}

// -------------------------------------------------------------------- RHS

template <int NT, int LAYOUT, bool PREK>
__global__ __launch_bounds__(NT) void k_rhs(DNet n, const double *__restrict__ la_over,
                                            int64_t n_cells, const double *__restrict__ y,
                                            const double *__restrict__ T,
                                            const double *__restrict__ kin,
                                            double *__restrict__ dydt) {
  extern __shared__ double sm[];
  const int ns = n.ns, nr = n.nr;
  double *ys = sm;
  double *rs = sm + ns;
  double *part = rs + nr;
  for (int64_t c = blockIdx.x; c < n_cells; c += gridDim.x) {
    load_cell<NT>(y + c * ns, ys, ns);
    if (LAYOUT == LAYOUT_CCS)
      for (int i = threadIdx.x; i < ns; i += NT) part[i] = 0.0;
    Env env{};
    if (!PREK) env = cell_env(T, c, n.n_cond);
    __syncthreads();
    if (PREK) {
      // every coefficient and reactant pair of a lane requested before use
      constexpr int KU = 8;
      const double *kc = kin + c * nr;
      for (int j0 = threadIdx.x; j0 < nr; j0 += KU * NT) {
        double kv[KU];
        uint32_t pr[KU];
#pragma unroll
        for (int u = 0; u < KU; ++u) {
          const int j = j0 + u * NT;
          kv[u] = j < nr ? __builtin_nontemporal_load(kc + j) : 0.0;
          pr[u] = j < nr ? n.rpair[j] : 0u;
        }
#pragma unroll
        for (int u = 0; u < KU; ++u)
          if (j0 + u * NT < nr) rs[j0 + u * NT] = reaction_rate(pr[u], kv[u], ys);
      }
    } else {
      for_reactions<NT>(n, la_over, env,
                        [&](int j, double kj, uint32_t pair) { rs[j] = reaction_rate(pair, kj, ys); });
    }
    __syncthreads();
    if (LAYOUT == LAYOUT_CCS) {
      // column by column (Sec. 2.2's CCS traversal): every reaction adds
      // S_ij R_j to each species of its packed net column, with LDS atomics
      // (the order of additions varies from run to run)
      for (int j = threadIdx.x; j < nr; j += NT) {
        const uint4 col = n.rxpack[2 * nr + j];
        const uint32_t w4[4] = {col.x, col.y, col.z, col.w};
        const double r = rs[j];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          const uint32_t h = (w4[q >> 1] >> (16 * (q & 1))) & 0xFFFFu;
          if (h != 0xFFFFu) atomicAdd(&part[h & 2047u], double(int32_t(h << 16) >> 27) * r);
        }
      }
      __syncthreads();
      double *out = dydt + c * ns;
      for (int i = threadIdx.x; i < ns; i += NT) out[i] = part[i];
    } else {
      segsum<NT, LAYOUT, false>(n.rhs, rs, ys, part, dydt + c * ns);   // rows of S: no density factor
    }
    __syncthreads();
  }
}

// SELL RHS with fused coefficients for two cells per pass: reaction
// records and SELL items are loaded and decoded once for both cells, whose
// densities, rates and partials sit side by side in LDS (16-byte pairs), so
// one LDS access serves both (one 1024-thread workgroup per CU holds both
// cells' LDS). Results are those of k_rhs bit for bit.
template <int NT>
__global__ __launch_bounds__(NT) void k_rhs2(DNet n, const double *__restrict__ la_over,
                                             int64_t n_cells, const double *__restrict__ y,
                                             const double *__restrict__ T,
                                             double *__restrict__ dydt) {
  extern __shared__ double sm[];
  const int ns = n.ns, nr = n.nr;
  double2 *yy = reinterpret_cast<double2 *>(sm);   // ns
  double2 *rr = yy + ns;                             // nr
  double2 *pp = rr + nr;                             // n_slot
  for (int64_t c = 2 * int64_t(blockIdx.x); c < n_cells; c += 2 * int64_t(gridDim.x)) {
    const bool two = c + 1 < n_cells;
    for (int i = threadIdx.x; i < ns; i += NT)
      yy[i] = make_double2(y[c * ns + i], two ? y[(c + 1) * ns + i] : 0.0);
    const Env e0 = cell_env(T, c, n.n_cond), e1 = cell_env(T, two ? c + 1 : c, n.n_cond);
    __syncthreads();
    for (int j0 = threadIdx.x; j0 < nr; j0 += RXU * NT) {
      Rx r[RXU];
#pragma unroll
      for (int u = 0; u < RXU; ++u) {
        const int j = j0 + u * NT;
        if (j < nr) {
          r[u] = load_rx(n, j);
          if (la_over) r[u].la = la_over[j];
        }
      }
#pragma unroll
      for (int u = 0; u < RXU; ++u) {
        const int j = j0 + u * NT;
        if (j < nr) {
          const double2 ya = yy[r[u].pair & 0xFFFFu];
          double r0 = rate_k(r[u], e0) * ya.x;
          double r1 = rate_k(r[u], e1) * ya.y;
          const uint32_t b = r[u].pair >> 16;
          if (b != 0xFFFFu) {
            const double2 yb = yy[b];
            r0 *= yb.x;
            r1 *= yb.y;
          }
          rr[j] = make_double2(r0, r1);
        }
      }
    }
    __syncthreads();
    double *out0 = dydt + c * ns, *out1 = two ? out0 + ns : nullptr;
    sell_pairs<NT>(n.rhs, rr, nullptr, 0u, pp, out0, out1);
    __syncthreads();
    segsum_finish_pairs<NT>(n.rhs, pp, out0, out1);
    __syncthreads();
  }
}

// --------------------------------------------------------------- Jacobian
//
// Two tiers: the tails (terms beyond the second of an entry; a few
// hundred entries hold half of all terms) are summed chunk-wise into LDS
// slots, then every entry adds its two head terms and its tail slots and
// is written once, coalesced and non-temporal.

template <int NT>
__global__ __launch_bounds__(NT) void k_jac(DNet n, const double *__restrict__ la_over,
                                            int64_t n_cells, const double *__restrict__ y,
                                            const double *__restrict__ T,
                                            double *__restrict__ jvals) {
  extern __shared__ double sm[];
  const int ns = n.ns, nr = n.nr;
  double *ys = sm;
  double *ks = sm + ns;
  double *part = ks + nr;
  for (int64_t c = blockIdx.x; c < n_cells; c += gridDim.x) {
    load_cell<NT>(y + c * ns, ys, ns);
    const Env env = cell_env(T, c, n.n_cond);
    for_reactions<NT>(n, la_over, env, [&](int j, double kj, uint32_t) { ks[j] = kj; });
    __syncthreads();
    runsum_partials<NT>(n.jtail, ks, ys, part);
    __syncthreads();
    double *out = jvals + c * n.nnz_j;
    constexpr int EU = 4;
    for (int e0 = threadIdx.x; e0 < n.nnz_j; e0 += EU * NT) {
      uint32_t h0[EU], h1[EU], td[EU];
#pragma unroll
      for (int u = 0; u < EU; ++u) {
        const int e = e0 + u * NT;
        const bool ok = e < n.nnz_j;
        h0[u] = ok ? n.jhead0[e] : PAD_ITEM;
        h1[u] = ok ? n.jhead1[e] : PAD_ITEM;
        td[u] = ok ? n.jtaildesc[e] : 0u;
      }
#pragma unroll
      for (int u = 0; u < EU; ++u) {
        const int e = e0 + u * NT;
        if (e < n.nnz_j) {
          double acc = term(h0[u], ks, ys);
          acc = __dadd_rn(acc, term(h1[u], ks, ys));
          const int q0 = int(td[u] >> 8), nq = int(td[u] & 255u);
          for (int q = 0; q < nq; ++q) acc = __dadd_rn(acc, part[q0 + q]);
          __builtin_nontemporal_store(acc, out + e);
        }
      }
    }
    __syncthreads();
  }
}

// The same two tiers for two cells per pass: every network word (reaction
// record, run, entry descriptor) is loaded and decoded once and serves both
// cells. The two cells' values sit side by side in LDS (a 16-byte pair per
// species, reaction and tail slot), so one LDS access and one address serve
// both cells. The species pair after the last holds (1, 1) for terms
// without a density factor and the slot pair after the last holds (0, 0),
// so every entry reads its two head terms and its first two tail slots
// without branching; only the few entries with more tail slots loop. Needs
// twice the LDS, so one 1024-thread workgroup per CU takes the place of two
// 512-thread ones.
// One pass of k_jac2 over the cell pair (c, c+1) (the second absent unless
// two): densities and coefficients into LDS, tail runs, then every entry
// written. zslot is the index of the (0, 0) slot pair. Leaves kk (the
// coefficients) and yy in LDS; the caller places the next barrier.
template <int NT>
__device__ __forceinline__ void jac2_pass(const DNet &n, const double *__restrict__ la_over,
                                          int64_t c, bool two, const double *__restrict__ y,
                                          const double *__restrict__ T,
                                          double *__restrict__ jvals, double2 *yy, double2 *kk,
                                          double2 *pp, uint32_t zslot) {
  const int ns = n.ns, nr = n.nr, nnz = n.nnz_j;
  for (int i = threadIdx.x; i < ns; i += NT)
    yy[i] = make_double2(y[c * ns + i], two ? y[(c + 1) * ns + i] : 0.0);
  const Env e0 = cell_env(T, c, n.n_cond), e1 = cell_env(T, two ? c + 1 : c, n.n_cond);
  for (int j0 = threadIdx.x; j0 < nr; j0 += RXU * NT) {
    Rx r[RXU];
#pragma unroll
    for (int u = 0; u < RXU; ++u) {
      const int j = j0 + u * NT;
      if (j < nr) {
        r[u] = load_rx(n, j);
        if (la_over) r[u].la = la_over[j];
      }
    }
#pragma unroll
    for (int u = 0; u < RXU; ++u) {
      const int j = j0 + u * NT;
      if (j < nr)
        kk[j] = make_double2(rate_k(r[u], e0),
                             rate_k(r[u], e1));
    }
  }
  __syncthreads();
  runsum_pairs<NT>(n.jtail, kk, yy, uint32_t(ns), pp);
  __syncthreads();
  double *out0 = jvals + c * nnz, *out1 = out0 + nnz;
  const uint32_t unnz = uint32_t(nnz);
  constexpr int EU = 4;
  for (uint32_t e0 = threadIdx.x; e0 < unnz; e0 += EU * NT) {
    uint32_t h0[EU], h1[EU], td[EU];
#pragma unroll
    for (int u = 0; u < EU; ++u) {
      const uint32_t e = e0 + u * NT;
      const bool ok = e < unnz;
      h0[u] = ok ? n.jhead0[e] : PAD_ITEM;
      h1[u] = ok ? n.jhead1[e] : PAD_ITEM;
      td[u] = ok ? n.jtaildesc[e] : 0u;
    }
#pragma unroll
    for (int u = 0; u < EU; ++u) {
      const uint32_t e = e0 + u * NT;
      if (e < unnz) {
        double a0 = 0.0, a1 = 0.0;
        term_pair(h0[u], kk, yy, uint32_t(ns), a0, a1);
        term_pair(h1[u], kk, yy, uint32_t(ns), a0, a1);
        const uint32_t q0 = td[u] >> 8, nq = td[u] & 255u;
        const double2 p0 = pp[nq > 0u ? q0 : zslot], p1 = pp[nq > 1u ? q0 + 1u : zslot];
        a0 = __dadd_rn(__dadd_rn(a0, p0.x), p1.x);
        a1 = __dadd_rn(__dadd_rn(a1, p0.y), p1.y);
        for (uint32_t q = 2; q < nq; ++q) {
          const double2 pq = pp[q0 + q];
          a0 = __dadd_rn(a0, pq.x);
          a1 = __dadd_rn(a1, pq.y);
        }
        __builtin_nontemporal_store(a0, out0 + e);
        if (two) __builtin_nontemporal_store(a1, out1 + e);
      }
    }
  }
}

template <int NT>
__global__ __launch_bounds__(NT) void k_jac2(DNet n, const double *__restrict__ la_over,
                                             int64_t n_cells, const double *__restrict__ y,
                                             const double *__restrict__ T,
                                             double *__restrict__ jvals) {
  extern __shared__ double sm[];
  const int ns = n.ns, nr = n.nr;
  const uint32_t nslot = uint32_t(n.jtail.n_slot > 0 ? n.jtail.n_slot : 0);
  double2 *yy = reinterpret_cast<double2 *>(sm);   // ns + 1
  double2 *kk = yy + ns + 1;                         // nr
  double2 *pp = kk + nr;                             // nslot + 1
  if (threadIdx.x == 0) {
    yy[ns] = make_double2(1.0, 1.0);
    pp[nslot] = make_double2(0.0, 0.0);
  }
  for (int64_t c = 2 * int64_t(blockIdx.x); c < n_cells; c += 2 * int64_t(gridDim.x)) {
    jac2_pass<NT>(n, la_over, c, c + 1 < n_cells, y, T, jvals, yy, kk, pp, nslot);
    __syncthreads();
  }
}

// RHS and Jacobian together, two cells per pass (SELL rows of S): the
// Jacobian pass of k_jac2, then the coefficients in LDS become the rates in
// place (k_j times the reactant densities, multiplied in k_rhs2's order)
// and the SELL row sums of k_rhs2 run on them, their partials in the slot
// region. One coefficient evaluation and one density load serve both
// outputs; both are bit-identical to k_jac2's and k_rhs2's.
template <int NT>
__global__ __launch_bounds__(NT) void k_rhs_jac2(DNet n, const double *__restrict__ la_over,
                                                 int64_t n_cells, const double *__restrict__ y,
                                                 const double *__restrict__ T,
                                                 double *__restrict__ dydt,
                                                 double *__restrict__ jvals) {
  extern __shared__ double sm[];
  const int ns = n.ns, nr = n.nr;
  const int js = n.jtail.n_slot > 0 ? n.jtail.n_slot : 0, rs = n.rhs.n_slot > 0 ? n.rhs.n_slot : 0;
  const uint32_t zslot = uint32_t(js > rs ? js : rs);   // beyond both kinds of partials
  double2 *yy = reinterpret_cast<double2 *>(sm);   // ns + 1
  double2 *kk = yy + ns + 1;                         // nr
  double2 *pp = kk + nr;                             // zslot + 1
  if (threadIdx.x == 0) {
    yy[ns] = make_double2(1.0, 1.0);
    pp[zslot] = make_double2(0.0, 0.0);
  }
  for (int64_t c = 2 * int64_t(blockIdx.x); c < n_cells; c += 2 * int64_t(gridDim.x)) {
    const bool two = c + 1 < n_cells;
    jac2_pass<NT>(n, la_over, c, two, y, T, jvals, yy, kk, pp, zslot);
    __syncthreads();
    for (int j = threadIdx.x; j < nr; j += NT) {
      const uint32_t pair = n.rpair[j];
      const double2 kv = kk[j], ya = yy[pair & 0xFFFFu];
      double r0 = kv.x * ya.x, r1 = kv.y * ya.y;
      if ((pair >> 16) != 0xFFFFu) {
        const double2 yb = yy[pair >> 16];
        r0 *= yb.x;
        r1 *= yb.y;
      }
      kk[j] = make_double2(r0, r1);
    }
    __syncthreads();
    double *out0 = dydt + c * ns, *out1 = two ? out0 + ns : nullptr;
    sell_pairs<NT>(n.rhs, kk, nullptr, 0u, pp, out0, out1);
    __syncthreads();
    segsum_finish_pairs<NT>(n.rhs, pp, out0, out1);
    __syncthreads();
  }
}


// -------------------------------------------------------------------- VJP
//
// w_j = (S^T v)_j from the packed net column of S; gy_a = sum over reactant
// slots of a of mult * k_j * n_other * w_j. The log-alpha gradient
// sum_c R_cj w_cj goes to a per-workgroup row of partial sums: a thread
// always owns the same reactions and a workgroup the same cells (fixed
// grid), so the row is updated without atomics, and the rows are added in
// workgroup order.

template <int NT>
__global__ __launch_bounds__(NT) void k_vjp(DNet n, const double *__restrict__ la_over,
                                            int64_t n_cells, const double *__restrict__ y,
                                            const double *__restrict__ T,
                                            const double *__restrict__ v,
                                            double *__restrict__ gy,
                                            double *__restrict__ part_glog) {
  extern __shared__ double sm[];
  const int ns = n.ns, nr = n.nr;
  double *ys = sm;
  double *vs = ys + ns;
  double *kw = vs + ns;
  double *part = kw + nr;
  double *prow = part_glog ? part_glog + size_t(blockIdx.x) * nr : nullptr;
  if (prow)
    for (int j = threadIdx.x; j < nr; j += NT) prow[j] = 0.0;
  for (int64_t c = blockIdx.x; c < n_cells; c += gridDim.x) {
    load_cell<NT>(y + c * ns, ys, ns);
    load_cell<NT>(v + c * ns, vs, ns);
    const Env env = cell_env(T, c, n.n_cond);
    __syncthreads();
    for_reactions<NT>(n, la_over, env, [&](int j, double kj, uint32_t pair) {
      const uint4 col = n.rxpack[2 * n.nr + j];
      const uint32_t w4[4] = {col.x, col.y, col.z, col.w};
      double w = 0.0;
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const uint32_t h = (w4[q >> 1] >> (16 * (q & 1))) & 0xFFFFu;
        if (h != 0xFFFFu) {
          const int coef = int32_t(h << 16) >> 27;
          w += double(coef) * vs[h & 2047u];
        }
      }
      kw[j] = kj * w;
      if (prow) prow[j] += reaction_rate(pair, kj, ys) * w;
    });
    __syncthreads();
    if (gy) {
      double *out = gy + c * ns;
      segsum_chunks<NT, LAYOUT_SELL, false>(n.gy, kw, ys, part, out);
      __syncthreads();
      segsum_finish<NT, false>(n.gy, part, out);
    }
    __syncthreads();
  }
}

// The VJP for two cells per pass, their values side by side in LDS (16-byte
// pairs; the species pair after the last holds (1, 1) for terms without a
// density factor): each packed column of S and each gy item is decoded once
// for both cells, and one LDS access serves both. The log-alpha partial row
// of a workgroup adds the first cell's term, then the second's.
template <int NT>
__global__ __launch_bounds__(NT) void k_vjp2(DNet n, const double *__restrict__ la_over,
                                             int64_t n_cells, const double *__restrict__ y,
                                             const double *__restrict__ T,
                                             const double *__restrict__ v,
                                             double *__restrict__ gy,
                                             double *__restrict__ part_glog) {
  extern __shared__ double sm[];
  const int ns = n.ns, nr = n.nr;
  double2 *yy = reinterpret_cast<double2 *>(sm);   // ns + 1
  double2 *vv = yy + ns + 1;                         // ns
  double2 *kw = vv + ns;                             // nr
  double2 *pp = kw + nr;                             // gy slots
  double *prow = part_glog ? part_glog + size_t(blockIdx.x) * nr : nullptr;
  if (prow)
    for (int j = threadIdx.x; j < nr; j += NT) prow[j] = 0.0;
  if (threadIdx.x == 0) yy[ns] = make_double2(1.0, 1.0);
  for (int64_t c = 2 * int64_t(blockIdx.x); c < n_cells; c += 2 * int64_t(gridDim.x)) {
    const bool two = c + 1 < n_cells;
    for (int i = threadIdx.x; i < ns; i += NT) {
      yy[i] = make_double2(y[c * ns + i], two ? y[(c + 1) * ns + i] : 0.0);
      vv[i] = make_double2(v[c * ns + i], two ? v[(c + 1) * ns + i] : 0.0);
    }
    const Env e0 = cell_env(T, c, n.n_cond), e1 = cell_env(T, two ? c + 1 : c, n.n_cond);
    __syncthreads();
    for (int j0 = threadIdx.x; j0 < nr; j0 += RXU * NT) {
      Rx r[RXU];
      uint4 col[RXU];
#pragma unroll
      for (int u = 0; u < RXU; ++u) {
        const int j = j0 + u * NT;
        if (j < nr) {
          r[u] = load_rx(n, j);
          col[u] = n.rxpack[2 * nr + j];
          if (la_over) r[u].la = la_over[j];
        }
      }
#pragma unroll
      for (int u = 0; u < RXU; ++u) {
        const int j = j0 + u * NT;
        if (j >= nr) continue;
        const uint32_t w4[4] = {col[u].x, col[u].y, col[u].z, col[u].w};
        double w0 = 0.0, w1 = 0.0;
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          const uint32_t h = (w4[q >> 1] >> (16 * (q & 1))) & 0xFFFFu;
          if (h != 0xFFFFu) {
            const double coef = double(int32_t(h << 16) >> 27);
            const double2 vq = vv[h & 2047u];
            w0 += coef * vq.x;
            w1 += coef * vq.y;
          }
        }
        const double k0 = rate_k(r[u], e0);
        const double k1 = rate_k(r[u], e1);
        kw[j] = make_double2(k0 * w0, k1 * w1);
        if (prow) {
          const uint32_t pair = r[u].pair;
          const double2 ya = yy[pair & 0xFFFFu];
          double r0 = k0 * ya.x, r1 = k1 * ya.y;
          if ((pair >> 16) != 0xFFFFu) {
            const double2 yb = yy[pair >> 16];
            r0 *= yb.x;
            r1 *= yb.y;
          }
          double g = prow[j] + r0 * w0;
          if (two) g += r1 * w1;
          prow[j] = g;
        }
      }
    }
    __syncthreads();
    if (gy) {
      double *out0 = gy + c * ns, *out1 = two ? out0 + ns : nullptr;
      sell_pairs<NT, true>(n.gy, kw, yy, uint32_t(ns), pp, out0, out1);
      __syncthreads();
      segsum_finish_pairs<NT>(n.gy, pp, out0, out1);
    }
    __syncthreads();
  }
}

constexpr int RED_NT = 256;

__global__ __launch_bounds__(RED_NT) void k_fill(double *__restrict__ p, int64_t n, double v) {
  for (int64_t i = blockIdx.x * int64_t(RED_NT) + threadIdx.x; i < n;
       i += int64_t(gridDim.x) * RED_NT)
    p[i] = v;
}

// out[j] = (acc ? out[j] : 0) + rows added one by one in row order, so that
// sums taken in consecutive chunks of rows equal one sum over all of them.
__global__ __launch_bounds__(RED_NT) void k_sum_rows(const double *__restrict__ part, int rows,
                                                     int nr, double *__restrict__ out, int acc) {
  const int j = blockIdx.x * RED_NT + threadIdx.x;
  if (j >= nr) return;
  double s = acc ? out[j] : 0.0;
  for (int r = 0; r < rows; ++r) s += part[size_t(r) * nr + j];
  out[j] = s;
}

// ---------------------------------------------------------------- launch

static int device_cus() {
  static int cus = 0;
  if (!cus) {
    int dev = 0;
    hipGetDevice(&dev);
    hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (cus <= 0) cus = 256;
  }
  return cus;
}

template <typename K>
static int grid_for(K kernel, int nt, size_t lds, int64_t n_cells) {
  if (lds > 65536) hipFuncSetAttribute(reinterpret_cast<const void *>(kernel),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, int(lds));
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, nt, lds) != hipSuccess ||
      per_cu <= 0)
    per_cu = 1;
  const int64_t g = int64_t(per_cu) * device_cus();
  return int(n_cells < g ? n_cells : g);
}

size_t rhs_lds_bytes(const DNet &n) {
  const int extra = (n.layout == LAYOUT_COO || n.layout == LAYOUT_CCS) ? n.ns
                    : n.layout == LAYOUT_RUNS ? n.rhs.n_rslot
                                              : n.rhs.n_slot;
  return sizeof(double) * size_t(n.ns + n.nr + (extra > 0 ? extra : 1));
}

// Dispatch on the network's workgroup size.
#define AC_DISPATCH_NT(nt, CALL) \
  ((nt) == 256 ? CALL(256) : (nt) == 1024 ? CALL(1024) : CALL(512))

// The workgroup size of a one-cell kernel using `lds` bytes: the network's,
// or when it asks for none, 1024 threads if the LDS leaves room for only
// one workgroup per CU (so that the CU still runs 16 waves), else 512.
static int block_for(const DNet &n, size_t lds) {
  if (n.block) return n.block;
  return lds > 80 * 1024 ? 1024 : 512;
}

template <int NT>
static hipError_t rates_nt(const DNet &n, const double *la, int64_t n_cells, const double *T,
                           double *k, hipStream_t st) {
  const int g = grid_for(k_rates<NT>, NT, 0, n_cells);
  hipLaunchKernelGGL(k_rates<NT>, dim3(g), dim3(NT), 0, st, n, la, n_cells, T, k);
  return hipGetLastError();
}

hipError_t launch_rates(const DNet &n, const double *la, int64_t n_cells, const double *T,
                        double *k, hipStream_t st) {
  if (n_cells == 0) return hipSuccess;
#define CALL(NT) rates_nt<NT>(n, la, n_cells, T, k, st)
  return AC_DISPATCH_NT(block_for(n, 0), CALL);
#undef CALL
}

template <int NT, int LAYOUT, bool PREK>
static hipError_t rhs_variant(const DNet &n, const double *la, int64_t n_cells, const double *y,
                              const double *T, const double *k, double *dydt, hipStream_t st) {
  const size_t lds = rhs_lds_bytes(n);
  auto kern = k_rhs<NT, LAYOUT, PREK>;
  const int g = grid_for(kern, NT, lds, n_cells);
  hipLaunchKernelGGL(kern, dim3(g), dim3(NT), lds, st, n, la, n_cells, y, T, k, dydt);
  return hipGetLastError();
}

template <int NT>
static hipError_t rhs_nt(const DNet &n, const double *la, int64_t n_cells, const double *y,
                         const double *T, const double *k, double *dydt, hipStream_t st) {
  if (k) {
    if (n.layout == LAYOUT_SELL) return rhs_variant<NT, LAYOUT_SELL, true>(n, la, n_cells, y, T, k, dydt, st);
    if (n.layout == LAYOUT_RUNS) return rhs_variant<NT, LAYOUT_RUNS, true>(n, la, n_cells, y, T, k, dydt, st);
    if (n.layout == LAYOUT_CCS) return rhs_variant<NT, LAYOUT_CCS, true>(n, la, n_cells, y, T, k, dydt, st);
    if (n.layout == LAYOUT_COO) return rhs_variant<NT, LAYOUT_COO, true>(n, la, n_cells, y, T, k, dydt, st);
    return rhs_variant<NT, LAYOUT_CSR, true>(n, la, n_cells, y, T, k, dydt, st);
  }
  if (n.layout == LAYOUT_SELL) return rhs_variant<NT, LAYOUT_SELL, false>(n, la, n_cells, y, T, k, dydt, st);
  if (n.layout == LAYOUT_RUNS) return rhs_variant<NT, LAYOUT_RUNS, false>(n, la, n_cells, y, T, k, dydt, st);
  if (n.layout == LAYOUT_CCS) return rhs_variant<NT, LAYOUT_CCS, false>(n, la, n_cells, y, T, k, dydt, st);
  if (n.layout == LAYOUT_COO) return rhs_variant<NT, LAYOUT_COO, false>(n, la, n_cells, y, T, k, dydt, st);
  return rhs_variant<NT, LAYOUT_CSR, false>(n, la, n_cells, y, T, k, dydt, st);
}

hipError_t launch_rhs(const DNet &n, const double *la, int64_t n_cells, const double *y,
                      const double *T, const double *k, double *dydt, hipStream_t st) {
  if (n_cells == 0) return hipSuccess;
  // SELL with fused coefficients: two cells per pass when their LDS fits
  const size_t lds2 = 2 * sizeof(double) * size_t(n.ns + n.nr + (n.rhs.n_slot > 0 ? n.rhs.n_slot : 1));
  if (!k && n.layout == LAYOUT_SELL && n_cells > 1 && lds2 <= 160 * 1024) {
    const int g = grid_for(k_rhs2<1024>, 1024, lds2, (n_cells + 1) / 2);
    hipLaunchKernelGGL(k_rhs2<1024>, dim3(g), dim3(1024), lds2, st, n, la, n_cells, y, T, dydt);
    return hipGetLastError();
  }
#define CALL(NT) rhs_nt<NT>(n, la, n_cells, y, T, k, dydt, st)
  return AC_DISPATCH_NT(block_for(n, rhs_lds_bytes(n)), CALL);
#undef CALL
}

template <int NT>
static hipError_t jac_nt(const DNet &n, const double *la, int64_t n_cells, const double *y,
                         const double *T, double *jvals, hipStream_t st) {
  const size_t lds = sizeof(double) * size_t(n.ns + n.nr + (n.jtail.n_slot > 0 ? n.jtail.n_slot : 1));
  const int g = grid_for(k_jac<NT>, NT, lds, n_cells);
  hipLaunchKernelGGL(k_jac<NT>, dim3(g), dim3(NT), lds, st, n, la, n_cells, y, T, jvals);
  return hipGetLastError();
}

// RHS + Jacobian in one pass per cell pair when the layout is SELL with
// fused coefficients and the pair's LDS fits; otherwise the two launches.
hipError_t launch_rhs_jac(const DNet &n, const double *la, int64_t n_cells, const double *y,
                          const double *T, double *dydt, double *jvals, hipStream_t st) {
  if (n_cells == 0) return hipSuccess;
  const int js = n.jtail.n_slot > 0 ? n.jtail.n_slot : 0, rs = n.rhs.n_slot > 0 ? n.rhs.n_slot : 0;
  const size_t lds2 = 2 * sizeof(double) * size_t(n.ns + 1 + n.nr + (js > rs ? js : rs) + 1);
  if (n.layout == LAYOUT_SELL && n_cells > 1 && lds2 <= 160 * 1024) {
    const int g = grid_for(k_rhs_jac2<1024>, 1024, lds2, (n_cells + 1) / 2);
    hipLaunchKernelGGL(k_rhs_jac2<1024>, dim3(g), dim3(1024), lds2, st, n, la, n_cells, y, T,
                       dydt, jvals);
    return hipGetLastError();
  }
  hipError_t e = launch_rhs(n, la, n_cells, y, T, nullptr, dydt, st);
  if (e != hipSuccess) return e;
  return launch_jac(n, la, n_cells, y, T, jvals, st);
}

hipError_t launch_jac(const DNet &n, const double *la, int64_t n_cells, const double *y,
                      const double *T, double *jvals, hipStream_t st) {
  if (n_cells == 0) return hipSuccess;
  // two cells per pass when their LDS fits one workgroup
  // pairs of doubles: species + (1, 1), reactions, tail slots + (0, 0)
  const size_t lds2 = 2 * sizeof(double) *
                      size_t(n.ns + 1 + n.nr + (n.jtail.n_slot > 0 ? n.jtail.n_slot : 0) + 1);
  if (n_cells > 1 && lds2 <= 160 * 1024) {
    const int g = grid_for(k_jac2<1024>, 1024, lds2, (n_cells + 1) / 2);
    hipLaunchKernelGGL(k_jac2<1024>, dim3(g), dim3(1024), lds2, st, n, la, n_cells, y, T, jvals);
    return hipGetLastError();
  }
#define CALL(NT) jac_nt<NT>(n, la, n_cells, y, T, jvals, st)
  return AC_DISPATCH_NT(
      block_for(n, sizeof(double) * size_t(n.ns + n.nr + (n.jtail.n_slot > 0 ? n.jtail.n_slot : 1))),
      CALL);
#undef CALL
}

template <int NT>
static hipError_t vjp_nt(const DNet &n, const double *la, int64_t n_cells, const double *y,
                         const double *T, const double *v, double *gy, double *g_logalpha,
                         double *part, int part_rows, hipStream_t st) {
  const size_t lds = sizeof(double) * size_t(2 * n.ns + n.nr + (n.gy.n_slot > 0 ? n.gy.n_slot : 1));
  // a fixed grid (independent of occupancy) keeps the cell-to-workgroup
  // assignment, and so the summation order, the same on every call
  const int g = int(n_cells < part_rows ? n_cells : part_rows);
  if (lds > 65536) hipFuncSetAttribute(reinterpret_cast<const void *>(k_vjp<NT>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, int(lds));
  hipLaunchKernelGGL(k_vjp<NT>, dim3(g), dim3(NT), lds, st, n, la, n_cells, y, T, v, gy,
                     g_logalpha ? part : nullptr);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || !g_logalpha) return e;
  hipLaunchKernelGGL(k_sum_rows, dim3((n.nr + RED_NT - 1) / RED_NT), dim3(RED_NT), 0, st, part, g,
                     n.nr, g_logalpha, 0);
  return hipGetLastError();
}

hipError_t launch_sum_rows(const double *part, int64_t rows, int nr, double *out, bool acc,
                           hipStream_t st) {
  if (rows == 0) {
    if (acc) return hipSuccess;
    hipLaunchKernelGGL(k_fill, dim3((nr + RED_NT - 1) / RED_NT), dim3(RED_NT), 0, st, out,
                       int64_t(nr), 0.0);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(k_sum_rows, dim3((nr + RED_NT - 1) / RED_NT), dim3(RED_NT), 0, st, part,
                     int(rows), nr, out, acc ? 1 : 0);
  return hipGetLastError();
}

hipError_t launch_vjp(const DNet &n, const double *la, int64_t n_cells, const double *y,
                      const double *T, const double *v, double *gy, double *g_logalpha,
                      double *part, int part_rows, hipStream_t st) {
  if (n_cells == 0) {
    if (g_logalpha) {
      hipLaunchKernelGGL(k_fill, dim3((n.nr + RED_NT - 1) / RED_NT), dim3(RED_NT), 0, st,
                         g_logalpha, int64_t(n.nr), 0.0);
      return hipGetLastError();
    }
    return hipSuccess;
  }
  // pairs of doubles: species + (1, 1), v, reactions, gy slots
  const size_t lds2 = 2 * sizeof(double) *
                      size_t(2 * n.ns + 1 + n.nr + (n.gy.n_slot > 0 ? n.gy.n_slot : 1));
  if (n_cells > 1 && lds2 <= 160 * 1024 && part_rows >= 2) {
    // fixed grid, as in vjp_nt: at most half the partial rows, one
    // workgroup per CU at this LDS size
    const int64_t pairs = (n_cells + 1) / 2;
    const int g = int(pairs < part_rows / 2 ? pairs : part_rows / 2);
    hipFuncSetAttribute(reinterpret_cast<const void *>(k_vjp2<1024>),
                        hipFuncAttributeMaxDynamicSharedMemorySize, int(lds2));
    hipLaunchKernelGGL(k_vjp2<1024>, dim3(g), dim3(1024), lds2, st, n, la, n_cells, y, T, v, gy,
                       g_logalpha ? part : nullptr);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || !g_logalpha) return e;
    hipLaunchKernelGGL(k_sum_rows, dim3((n.nr + RED_NT - 1) / RED_NT), dim3(RED_NT), 0, st, part,
                       g, n.nr, g_logalpha, 0);
    return hipGetLastError();
  }
#define CALL(NT) vjp_nt<NT>(n, la, n_cells, y, T, v, gy, g_logalpha, part, part_rows, st)
  return AC_DISPATCH_NT(
      block_for(n, sizeof(double) *
                       size_t(2 * n.ns + n.nr + (n.gy.n_slot > 0 ? n.gy.n_slot : 1))),
      CALL);
#undef CALL
}

}  // namespace ac
