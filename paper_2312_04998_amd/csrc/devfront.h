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

// acc + sum_{q in [b, e)} sgn * V[q] x[col[q]], four loads in flight.
template <bool NEG>
__device__ __forceinline__ double sp_dot_rows(const double *__restrict__ V,
                                              const int32_t *__restrict__ col,
                                              const double *x, int b, int e, double acc) {
  int q = b;
  for (; q + 4 <= e; q += 4) {
    const int c0 = col[q], c1 = col[q + 1], c2 = col[q + 2], c3 = col[q + 3];
    const double v0 = V[q], v1 = V[q + 1], v2 = V[q + 2], v3 = V[q + 3];
    acc = fma(NEG ? -v0 : v0, x[c0], acc);
    acc = fma(NEG ? -v1 : v1, x[c1], acc);
    acc = fma(NEG ? -v2 : v2, x[c2], acc);
    acc = fma(NEG ? -v3 : v3, x[c3], acc);
  }
  for (; q < e; ++q) acc = fma(NEG ? -V[q] : V[q], x[col[q]], acc);
  return acc;
}

// acc + sum_{q in [b, e)} sgn * V[idx[q]] x[row[q]] (column order).
template <bool NEG>
__device__ __forceinline__ double sp_dot_cols(const double *__restrict__ V,
                                              const int32_t *__restrict__ idx,
                                              const int32_t *__restrict__ row, const double *x,
                                              int b, int e, double acc) {
  int q = b;
  for (; q + 4 <= e; q += 4) {
    const int i0 = idx[q], i1 = idx[q + 1], i2 = idx[q + 2], i3 = idx[q + 3];
    const int r0 = row[q], r1 = row[q + 1], r2 = row[q + 2], r3 = row[q + 3];
    const double v0 = V[i0], v1 = V[i1], v2 = V[i2], v3 = V[i3];
    acc = fma(NEG ? -v0 : v0, x[r0], acc);
    acc = fma(NEG ? -v1 : v1, x[r1], acc);
    acc = fma(NEG ? -v2 : v2, x[r2], acc);
    acc = fma(NEG ? -v3 : v3, x[r3], acc);
  }
  for (; q < e; ++q) acc = fma(NEG ? -V[idx[q]] : V[idx[q]], x[row[q]], acc);
  return acc;
}

// M = I - c J from the pattern values Jg (natural order), swept over the
// front pivots level by level, then S factored with partial pivoting
// (wg_lu: piv, perm2 of n2 entries). Returns 0, or 1 + the position of a
// zero pivot (the front's first, else the tail's).
template <int NT>
__device__ __forceinline__ int front_factor(const DNet &n, const double *__restrict__ Jg, double c,
                                            double *M, int *piv, int *perm2, double *pan,
                                            double *red, int *redi, int *ipiv) {
  const DFront &F = n.fr;
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
  __syncthreads();
  for (int l = 0; l < F.n_lev; ++l) {
    const int k0 = F.lev_ptr[l], k1 = F.lev_ptr[l + 1];
    // pivot rows over their pivots
    for (int k = k0 + int(threadIdx.x); k < k1; k += NT) {
      const int d = F.vdiag[k];
      const double p = V[d];
      if (p == 0.0) atomicMin(&redi[0], k);
      const double inv = 1.0 / p;
      for (int q = F.row_ptr[k]; q < F.row_ptr[k + 1]; ++q)
        if (q != d) V[q] *= inv;
    }
    __syncthreads();
    // a_ij -= a_ik (a_kj / a_kk) for the level's pivots k, one target per thread
    for (int t = F.tg_ptr[l] + int(threadIdx.x); t < F.tg_ptr[l + 1]; t += NT) {
      const int d = F.tgt[t];
      double *dst = d >= 0 ? V + d : S + (-1 - d);
      double a = *dst;
      for (int o = F.op_ptr[t]; o < F.op_ptr[t + 1]; ++o) {
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
      for (int q = F.cptr[k]; q < F.cptr[k + 1]; ++q) {
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
// tmp (LDS, n doubles) is scratch; blk: the dense solves' LDS blocks.
template <int NT>
__device__ __forceinline__ void front_solve(const DFront &F, const double *M, const int *perm2,
                                            double *x, double *tmp, bool trans, double *blk) {
  const double *S = M, *V = M + F.vofs;
  const int n = F.n, n1 = F.n1, n2 = F.n2;
  for (int i = threadIdx.x; i < n; i += NT) tmp[i] = x[F.perm[i]];
  __syncthreads();
  if (!trans) {
    // front: A^-1 b1; tail: b2 - C A^-1 b1 (positions, into x)
    for (int r = threadIdx.x; r < n; r += NT) {
      const bool fr = r < n1;
      x[r] = sp_dot_rows<false>(V, F.col, tmp, F.row_ptr[r], fr ? F.rsplit[r] : F.row_ptr[r + 1],
                                fr ? 0.0 : tmp[r]);
    }
    __syncthreads();
    if (n2 > 0) wg_solve<NT>(S, F.lda2, n2, perm2, x + n1, tmp + n1, false, blk);
    // front: z1 = A^-1 b1 - A^-1 B z2
    for (int r = threadIdx.x; r < n; r += NT)
      tmp[r] = r < n1 ? sp_dot_rows<true>(V, F.col, x, F.rsplit[r], F.row_ptr[r + 1], x[r]) : x[r];
  } else {
    // front: A^-T b1; tail: b2 - (A^-1 B)^T b1
    for (int q = threadIdx.x; q < n; q += NT) {
      if (q < n1) x[q] = sp_dot_cols<false>(V, F.cidx, F.crow, tmp, F.cptr[q], F.csplit[q], 0.0);
      else x[q] = sp_dot_cols<true>(V, F.cidx, F.crow, tmp, F.cptr[q], F.cptr[q + 1], tmp[q]);
    }
    __syncthreads();
    if (n2 > 0) wg_solve<NT>(S, F.lda2, n2, perm2, x + n1, tmp + n1, true, blk);
    // front: z1 = A^-T b1 - (C A^-1)^T z2 (the stored values are -C A^-1)
    for (int q = threadIdx.x; q < n; q += NT)
      tmp[q] = q < n1 ? sp_dot_cols<false>(V, F.cidx, F.crow, x, F.csplit[q], F.cptr[q + 1], x[q])
                      : x[q];
  }
  __syncthreads();
  for (int i = threadIdx.x; i < n; i += NT) x[F.perm[i]] = tmp[i];
  __syncthreads();
}

}  // namespace ac
