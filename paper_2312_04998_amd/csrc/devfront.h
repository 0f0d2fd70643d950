// Workgroup-level Newton factorisation and solves with a sparse front and a
// dense Schur tail (the plan and its algebra: frontlu.h). One workgroup
// owns one matrix; the Schur complement S (n2 x lda2, row-major) sits at
// the start of the slot's matrix region and the swept sparse values after
// it; right-hand sides live in LDS.
#pragma once

#include <climits>

#include "devla.h"
#include "devnet.h"

namespace ac {

// sum_{q in [b, e)} V[q] x[col[q]] (rows) or V[idx[q]] x[row[q]]
// (columns), eight entries' loads in flight.
__device__ __forceinline__ double dot_rows(const double *__restrict__ V,
                                           const int32_t *__restrict__ col, const double *x,
                                           int b, int e) {
  double acc = 0.0;
  int q = b;
  for (; q + 8 <= e; q += 8) {
    int c[8];
    double v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      c[u] = col[q + u];
      v[u] = V[q + u];
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) acc = fma(v[u], x[c[u]], acc);
  }
  for (; q < e; ++q) acc = fma(V[q], x[col[q]], acc);
  return acc;
}

__device__ __forceinline__ double dot_cols(const double *__restrict__ V,
                                           const int32_t *__restrict__ idx,
                                           const int32_t *__restrict__ row, const double *x,
                                           int b, int e) {
  double acc = 0.0;
  int q = b;
  for (; q + 8 <= e; q += 8) {
    int i[8], r[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      i[u] = idx[q + u];
      r[u] = row[q + u];
    }
    double v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = V[i[u]];
#pragma unroll
    for (int u = 0; u < 8; ++u) acc = fma(v[u], x[r[u]], acc);
  }
  for (; q < e; ++q) acc = fma(V[idx[q]], x[row[q]], acc);
  return acc;
}

// Partial sums of gather g's pieces (plan: frontlu.h) into part (LDS).
template <int NT, bool COLS>
__device__ __forceinline__ void gather_pieces(const DFront &F, int g, const double *V,
                                              const double *x, double *part) {
  const int p0 = F.gbase[g], p1 = F.gbase[g + 1];
  for (int p = p0 + int(threadIdx.x); p < p1; p += NT) {
    const int2 r = F.gpc[p];
    part[p - p0] = COLS ? dot_cols(V, F.cidx, F.crow, x, r.x, r.y) : dot_rows(V, F.col, x, r.x, r.y);
  }
}

// Sum of output r's pieces of gather g, in piece order.
__device__ __forceinline__ double gather_sum(const DFront &F, int g, int r, const double *part) {
  const int32_t *seg = F.gseg + size_t(g) * (F.n + 1);
  const int p0 = F.gbase[g];
  double acc = 0.0;
  for (int p = seg[r]; p < seg[r + 1]; ++p) acc += part[p - p0];
  return acc;
}

// M = I - c J from the pattern values Jg (natural order), swept over the
// front pivots level by level, then S factored with partial pivoting
// (wg_lu: piv, perm2 of n2 entries). Returns 0, or 1 + the position of a
// zero pivot (the front's first, else the tail's).
// Jaux (temperature-coupled plan only, else null): the Jacobian's T column,
// T row and corner after the pattern values.
template <int NT>
__device__ __forceinline__ int front_factor(const DNet &n, const DFront &F,
                                            const double *__restrict__ Jg,
                                            const double *__restrict__ Jaux, double c,
                                            double *M, int *piv, int *perm2, double *pan,
                                            double *red, int *redi, int *ipiv) {
  double *S = M, *V = M + F.vofs;
  const int n2 = F.n2, lda2 = F.lda2;
  if (threadIdx.x == 0) redi[0] = INT_MAX;
  for (int e = threadIdx.x; e < F.nv; e += NT) V[e] = 0.0;
  for (int e = threadIdx.x; e < n2 * lda2; e += NT) S[e] = 0.0;
  __syncthreads();
  for (int k = threadIdx.x; k < F.n1; k += NT) V[F.vdiag[k]] = 1.0;
  for (int i = threadIdx.x; i < n2; i += NT) S[size_t(i) * lda2 + i] = 1.0;
  __syncthreads();
  constexpr int EU = 4;
  for (int e0 = threadIdx.x; e0 < n.nnz_j; e0 += EU * NT) {
    int dst[EU];
    bool dg[EU];
    double jv[EU];
#pragma unroll
    for (int u = 0; u < EU; ++u) {
      const int e = e0 + u * NT;
      const bool ok = e < n.nnz_j;
      dst[u] = ok ? F.asm_dst[e] : 0;
      dg[u] = ok && n.jent_row[e] == n.jent_col[e];
      jv[u] = ok ? Jg[e] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < EU; ++u)
      if (e0 + u * NT < n.nnz_j) {
        const double v = (dg[u] ? 1.0 : 0.0) - c * jv[u];
        if (dst[u] >= 0) V[dst[u]] = v;
        else S[-1 - dst[u]] = v;
      }
  }
  if (Jaux) {
    const int ns = n.ns;
    for (int i = threadIdx.x; i < ns; i += NT) {
      const int d1 = F.tcol_dst[i], d2 = F.trow_dst[i];
      const double v1 = -c * Jaux[i], v2 = -c * Jaux[ns + i];
      if (d1 >= 0) V[d1] = v1;
      else S[-1 - d1] = v1;
      if (d2 >= 0) V[d2] = v2;
      else S[-1 - d2] = v2;
    }
    if (threadIdx.x == 0) {
      const int d3 = F.corner_dst;
      const double v3 = 1.0 - c * Jaux[2 * ns];
      if (d3 >= 0) V[d3] = v3;
      else S[-1 - d3] = v3;
    }
  }
  __syncthreads();
  for (int l = 0; l < F.n_lev; ++l) {
    const int k0 = F.lev_ptr[l], k1 = F.lev_ptr[l + 1];
    // pivot rows over their pivots
    for (int k = k0 + int(threadIdx.x); k < k1; k += NT) {
      const int d = F.vdiag[k];
      const double p = V[d];
      if (p == 0.0) atomicMin(&redi[0], k);
      const double inv = 1.0 / p;
      int q = F.row_ptr[k];
      const int qe = F.row_ptr[k + 1];
      for (; q + 8 <= qe; q += 8) {
        double v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = V[q + u];
#pragma unroll
        for (int u = 0; u < 8; ++u)
          if (q + u != d) V[q + u] = v[u] * inv;
      }
      for (; q < qe; ++q)
        if (q != d) V[q] *= inv;
    }
    __syncthreads();
    // a_ij -= a_ik (a_kj / a_kk) for the level's pivots k, one target per thread
    for (int t = F.tg_ptr[l] + int(threadIdx.x); t < F.tg_ptr[l + 1]; t += NT) {
      const int d = F.tgt[t];
      double *dst = d >= 0 ? V + d : S + (-1 - d);
      double a = *dst;
      int o = F.op_ptr[t];
      const int oe = F.op_ptr[t + 1];
      for (; o + 8 <= oe; o += 8) {
        int2 op[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) op[u] = F.ops[o + u];
        double l[8], r[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          l[u] = V[op[u].x];
          r[u] = V[op[u].y];
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) a = fma(-l[u], r[u], a);
      }
      for (; o < oe; ++o) {
        const int2 op = F.ops[o];
        a = fma(-V[op.x], V[op.y], a);
      }
      *dst = a;
    }
    __syncthreads();
    // pivot columns: a_ik = -a_ik / a_kk, then a_kk = 1 / a_kk
    for (int k = k0 + int(threadIdx.x); k < k1; k += NT) {
      const int d = F.vdiag[k];
      const double inv = 1.0 / V[d];
      int q = F.cptr[k];
      const int qe = F.cptr[k + 1];
      for (; q + 8 <= qe; q += 8) {
        int vi[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) vi[u] = F.cidx[q + u];
        double v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = V[vi[u]];
#pragma unroll
        for (int u = 0; u < 8; ++u)
          if (vi[u] != d) V[vi[u]] = -v[u] * inv;
      }
      for (; q < qe; ++q) {
        const int vi = F.cidx[q];
        if (vi != d) V[vi] = -V[vi] * inv;
      }
      V[d] = inv;
    }
    __syncthreads();
  }
  const int zk = redi[0];
  __syncthreads();   // redi is wg_lu's scratch from here on
  int info = zk < INT_MAX ? 1 + zk : 0;
  if (n2 > 0) {
    const int i2 = wg_lu<NT>(S, lda2, n2, piv, perm2, pan, red, redi, ipiv);
    if (!info && i2) info = F.n1 + i2;
  }
  return info;
}

// Solves M x = b (trans = false) or M^T x = b with the factors of
// front_factor: x (LDS, natural order) holds b on entry and x on return;
// tmp (LDS, n doubles) is scratch; blk (LDS) holds the dense solves' blocks
// and, before and after them, the gathers' partial sums (at most
// FRONT_MAX_PIECES doubles).
template <int NT>
__device__ __forceinline__ void front_solve(const DFront &F, const double *M, const int *perm2,
                                            double *x, double *tmp, bool trans, double *blk) {
  const double *S = M, *V = M + F.vofs;
  const int n = F.n, n1 = F.n1, n2 = F.n2;
  for (int i = threadIdx.x; i < n; i += NT) tmp[i] = x[F.perm[i]];
  __syncthreads();
  if (!trans) {
    // front: A^-1 b1; tail: b2 - C A^-1 b1 (the stored values are -C A^-1)
    gather_pieces<NT, false>(F, 0, V, tmp, blk);
    __syncthreads();
    for (int r = threadIdx.x; r < n; r += NT) x[r] = (r < n1 ? 0.0 : tmp[r]) + gather_sum(F, 0, r, blk);
    __syncthreads();
    if (n2 > 0) wg_solve<NT>(S, F.lda2, n2, perm2, x + n1, tmp + n1, false, blk);
    // front: z1 = A^-1 b1 - A^-1 B z2
    gather_pieces<NT, false>(F, 1, V, x, blk);
    __syncthreads();
    for (int r = threadIdx.x; r < n; r += NT) tmp[r] = x[r] - gather_sum(F, 1, r, blk);
  } else {
    // front: A^-T b1; tail: b2 - (A^-1 B)^T b1
    gather_pieces<NT, true>(F, 2, V, tmp, blk);
    __syncthreads();
    for (int q = threadIdx.x; q < n; q += NT) {
      const double g = gather_sum(F, 2, q, blk);
      x[q] = q < n1 ? g : tmp[q] - g;
    }
    __syncthreads();
    if (n2 > 0) wg_solve<NT>(S, F.lda2, n2, perm2, x + n1, tmp + n1, true, blk);
    // front: z1 = A^-T b1 + (-C A^-1)^T z2
    gather_pieces<NT, true>(F, 3, V, x, blk);
    __syncthreads();
    for (int q = threadIdx.x; q < n; q += NT) tmp[q] = x[q] + gather_sum(F, 3, q, blk);
  }
  __syncthreads();
  for (int i = threadIdx.x; i < n; i += NT) x[F.perm[i]] = tmp[i];
  __syncthreads();
}

}  // namespace ac
