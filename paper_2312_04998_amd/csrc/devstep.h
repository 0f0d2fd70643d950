// Per-cell building blocks of the implicit integrator shared by the
// forward kernel and its discrete adjoint: the workgroup's view of one
// cell, RHS / Jacobian / Newton-matrix evaluation into LDS and the slot,
// the BDF constants and the difference-array operations.
#pragma once

#include "devchem.h"
#include "devla.h"
#include "devbdf.h"
#include "devfront.h"

namespace ac {

constexpr int QMAX = 5, NDROW = QMAX + 3, NEWTON_MAXITER = 4;
constexpr double MIN_FACTOR = 0.2, MAX_FACTOR = 10.0;

// gamma_q = sum_{m=1..q} 1/m (summed in increasing m), alpha_q = gamma_q,
// error constant 1/(q+1)
__device__ __forceinline__ double bdf_gamma(int q) {
  double g = 0.0;
  for (int m = 1; m <= q; ++m) g += 1.0 / m;
  return g;
}
__device__ __forceinline__ double bdf_errc(int q) { return 1.0 / (q + 1); }

__device__ __forceinline__ double pow_neg(double x, double e) {
  return x == 0.0 ? INFINITY : pow(x, -e);
}

// One LDS region serves, at different times, the RHS (or VJP) per-reaction
// block and its partial-sum slots, the LU panel, and the solves' diagonal
// block.
__host__ __device__ inline int bdf_scratch_doubles(const DNet &n) {
  const int slots = n.rhs.n_slot > n.gy.n_slot ? n.rhs.n_slot : n.gy.n_slot;
  const int rhs = n.nr + (slots > 0 ? slots : 1);
  const int la = la_scratch_doubles(n.ns);
  return rhs > la ? rhs : la;
}

// Per-workgroup view of one cell's work.
struct CellCtx {
  const DNet *n;
  double *kg;      // rate coefficients (slot, global)
  double *Jg;      // Jacobian values (slot, global)
  double *tailp;   // Jacobian tail partials (slot, global)
  double *M;       // Newton matrix / LU (slot, global)
  int *piv;        // pivots (slot, global)
  int *perm;       // row permutation of the factorisation (slot, global)
  double *D;       // difference array [NDROW][ns] (slot, global)
  int lda;
  double *rs, *part, *scr, *tmp, *red;   // LDS: rate block + slots | LU panel | solve block
  int *redi, *ipiv;
  int cnt[ST_N];   // per-cell counters (identical on every thread)
  int lu_info = 0; // 0, or 1 + the first exactly-zero pivot of the last factorisation
  // temperature-coupled mode: the cell's conditions (cond[0] unused), its
  // heat capacity, background temperature and relaxation rate, the
  // log-prefactor override, and the Jacobian's T column, T row and corner
  // (slot, global, after the pattern values)
  const double *cond = nullptr;
  int nc = 1;
  double cv = 1.0, Tb = 0.0, lam = 0.0;
  const double *la_over = nullptr;
  double *Jaux = nullptr;
  // Newton matrix held as a swept sparse front and a dense Schur tail
  // (front_factor / front_solve) instead of one dense LU
  bool front = false;
};

template <int NT>
__device__ __forceinline__ double wg_rms(const double *x, double mul, const double *scale, int n,
                                         double *red) {
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += NT) {
    const double v = mul * x[i] / scale[i];
    s += v * v;
  }
  return sqrt(wg_sum<NT>(s, red) / n);
}

template <int NT>
__device__ __forceinline__ bool wg_any(bool b, double *red) {
  return wg_sum<NT>(b ? 1.0 : 0.0, red) > 0.0;
}

// f = S R(y) with the cell's coefficients; y and f in LDS.
template <int NT>
__device__ __forceinline__ void cell_rhs(CellCtx &cx, const double *y, double *f) {
  const DNet &n = *cx.n;
  constexpr int U = 4;
  for (int j0 = threadIdx.x; j0 < n.nr; j0 += U * NT) {
    uint32_t pr[U];
    double kv[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int j = j0 + u * NT;
      pr[u] = j < n.nr ? n.rpair[j] : 0u;
      kv[u] = j < n.nr ? cx.kg[j] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int j = j0 + u * NT;
      if (j < n.nr) cx.rs[j] = reaction_rate(pr[u], kv[u], y);
    }
  }
  __syncthreads();
  segsum_chunks<NT, LAYOUT_SELL, false, false>(n.rhs, cx.rs, y, cx.part, f);
  __syncthreads();
  segsum_finish<NT, false>(n.rhs, cx.part, f);
  __syncthreads();
  cx.cnt[ST_RHS]++;
}

// Jacobian values on the pattern at y (LDS) into the slot.
template <int NT>
__device__ __forceinline__ void cell_jac(CellCtx &cx, const double *y) {
  const DNet &n = *cx.n;
  runsum_partials<NT>(n.jtail, cx.kg, y, cx.tailp);
  __syncthreads();
  constexpr int EU = 4;
  for (int e0 = threadIdx.x; e0 < n.nnz_j; e0 += EU * NT) {
    uint32_t h0[EU], h1[EU], td[EU];
#pragma unroll
    for (int u = 0; u < EU; ++u) {
      const int e = e0 + u * NT;
      const bool ok = e < n.nnz_j;
      h0[u] = ok ? n.jhead0[e] : 2047u << 16;
      h1[u] = ok ? n.jhead1[e] : 2047u << 16;
      td[u] = ok ? n.jtaildesc[e] : 0u;
    }
#pragma unroll
    for (int u = 0; u < EU; ++u) {
      const int e = e0 + u * NT;
      if (e < n.nnz_j) {
        double acc = term(h0[u], cx.kg, y);
        acc = __dadd_rn(acc, term(h1[u], cx.kg, y));
        const int q0 = int(td[u] >> 8), nq = int(td[u] & 255u);
        for (int q = 0; q < nq; ++q) acc = __dadd_rn(acc, cx.tailp[q0 + q]);
        cx.Jg[e] = acc;
      }
    }
  }
  __syncthreads();
  cx.cnt[ST_JAC]++;
}

// M = I - c J from the pattern values, then its factors: the sparse front
// and Schur tail when cx.front, else the dense row-major LU (lda).
template <int NT>
__device__ __forceinline__ void cell_factor(CellCtx &cx, double c) {
  const DNet &n = *cx.n;
  if (cx.front) {
    cx.lu_info = front_factor<NT>(n, n.fr, cx.Jg, nullptr, c, cx.M, cx.piv, cx.perm, cx.scr,
                                  cx.red, cx.redi, cx.ipiv);
    cx.cnt[ST_LU]++;
    return;
  }
  const int ns = n.ns, lda = cx.lda;
  for (int e = threadIdx.x; e < ns * lda; e += NT) {
    const int i = e / lda, a = e - i * lda;
    cx.M[e] = (i == a) ? 1.0 : 0.0;
  }
  __syncthreads();
  constexpr int EU = 4;
  for (int e0 = threadIdx.x; e0 < n.nnz_j; e0 += EU * NT) {
    int ri[EU], ci[EU];
    double jv[EU];
#pragma unroll
    for (int u = 0; u < EU; ++u) {
      const int e = e0 + u * NT;
      const bool ok = e < n.nnz_j;
      ri[u] = ok ? n.jent_row[e] : 0;
      ci[u] = ok ? n.jent_col[e] : 0;
      jv[u] = ok ? cx.Jg[e] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < EU; ++u)
      if (e0 + u * NT < n.nnz_j)
        cx.M[size_t(ri[u]) * lda + ci[u]] = (ri[u] == ci[u] ? 1.0 : 0.0) - c * jv[u];
  }
  __syncthreads();
  cx.lu_info = wg_lu<NT>(cx.M, lda, ns, cx.piv, cx.perm, cx.scr, cx.red, cx.redi, cx.ipiv);
  cx.cnt[ST_LU]++;
}

// ---------------------------------------------- temperature as a state
// State (n_1..n_ns, T); the coefficients follow the state's T and
// dT/dt = (sum_j heat_j R_j) / c_v - lambda (T - T_b) (codes that solve
// temperature and abundances together, Sec. 5).

// f = (S R(y), dT/dt), coefficients recomputed at T = y[ns]; y, f in LDS.
template <int NT>
__device__ __forceinline__ void cell_rhs_th(CellCtx &cx, const double *y, double *f) {
  const DNet &n = *cx.n;
  const int ns = n.ns;
  const double T = y[ns];
  const Env env = env_with_T(cx.cond, cx.nc, T);
  const double *heat = n.heat;
  double hsum = 0.0;
  for_rx<NT>(n, cx.la_over, env, [&](int j, double kj, const Rx &r) {
    const double rj = reaction_rate(r.pair, kj, y);
    cx.rs[j] = rj;
    if (heat) hsum += heat[j] * rj;
  });
  __syncthreads();
  segsum_chunks<NT, LAYOUT_SELL, false, false>(n.rhs, cx.rs, y, cx.part, f);
  __syncthreads();
  segsum_finish<NT, false>(n.rhs, cx.part, f);
  const double q = wg_sum<NT>(hsum, cx.red);
  if (threadIdx.x == 0) f[ns] = q / cx.cv - cx.lam * (T - cx.Tb);
  __syncthreads();
  cx.cnt[ST_RHS]++;
}

// Jacobian at y (LDS) with the coefficients at T = y[ns]: pattern values
// into the slot (as cell_jac, with the coefficients refreshed in the slot),
// then the T column sum_j S_ij R_j dln k_j/dT, the T row
// sum_{slots of a} heat_j dR_j/dn_a / c_v and the corner
// sum_j heat_j R_j dln k_j/dT / c_v - lambda into cx.Jaux.
template <int NT>
__device__ __forceinline__ void cell_jac_th(CellCtx &cx, const double *y) {
  const DNet &n = *cx.n;
  const int ns = n.ns;
  const double T = y[ns];
  const Env env = env_with_T(cx.cond, cx.nc, T);
  const double *heat = n.heat;
  double csum = 0.0;
  for_rx<NT>(n, cx.la_over, env, [&](int j, double kj, const Rx &r) {
    cx.kg[j] = kj;
    const double w = reaction_rate(r.pair, kj, y) * rate_dlnk_dT(r, env.invT);
    cx.rs[j] = w;
    if (heat) csum += heat[j] * w;
  });
  __syncthreads();
  segsum_chunks<NT, LAYOUT_SELL, false, false>(n.rhs, cx.rs, y, cx.part, cx.Jaux);
  __syncthreads();
  segsum_finish<NT, false>(n.rhs, cx.part, cx.Jaux);
  __syncthreads();
  for (int j = threadIdx.x; j < n.nr; j += NT) cx.rs[j] = heat ? cx.kg[j] * heat[j] / cx.cv : 0.0;
  __syncthreads();
  segsum_chunks<NT, LAYOUT_SELL, false, true>(n.gy, cx.rs, y, cx.part, cx.Jaux + ns);
  __syncthreads();
  segsum_finish<NT, false>(n.gy, cx.part, cx.Jaux + ns);
  const double corner = wg_sum<NT>(csum, cx.red) / cx.cv - cx.lam;
  if (threadIdx.x == 0) cx.Jaux[2 * ns] = corner;
  __syncthreads();
  cell_jac<NT>(cx, y);   // pattern values with the refreshed coefficients
}

// M = I - c J over the coupled state (ns + 1), then its factors: the
// sparse front of the coupled state's plan when cx.front, else one LU.
template <int NT>
__device__ __forceinline__ void cell_factor_th(CellCtx &cx, double c) {
  const DNet &n = *cx.n;
  if (cx.front) {
    cx.lu_info = front_factor<NT>(n, n.fr_th, cx.Jg, cx.Jaux, c, cx.M, cx.piv, cx.perm, cx.scr,
                                  cx.red, cx.redi, cx.ipiv);
    cx.cnt[ST_LU]++;
    return;
  }
  const int ns = n.ns, nv = ns + 1, lda = cx.lda;
  for (int e = threadIdx.x; e < nv * lda; e += NT) {
    const int i = e / lda, a = e - i * lda;
    cx.M[e] = (i == a) ? 1.0 : 0.0;
  }
  __syncthreads();
  for (int e = threadIdx.x; e < n.nnz_j; e += NT) {
    const int ri = n.jent_row[e], ci = n.jent_col[e];
    cx.M[size_t(ri) * lda + ci] = (ri == ci ? 1.0 : 0.0) - c * cx.Jg[e];
  }
  for (int i = threadIdx.x; i < ns; i += NT) {
    cx.M[size_t(i) * lda + ns] = -c * cx.Jaux[i];
    cx.M[size_t(ns) * lda + i] = -c * cx.Jaux[ns + i];
  }
  if (threadIdx.x == 0) cx.M[size_t(ns) * lda + ns] = 1.0 - c * cx.Jaux[2 * ns];
  __syncthreads();
  cx.lu_info = wg_lu<NT>(cx.M, lda, nv, cx.piv, cx.perm, cx.scr, cx.red, cx.redi, cx.ipiv);
  cx.cnt[ST_LU]++;
}

template <int NT, bool TH>
__device__ __forceinline__ void cell_rhs_any(CellCtx &cx, const double *y, double *f) {
  if (TH) cell_rhs_th<NT>(cx, y, f);
  else cell_rhs<NT>(cx, y, f);
}

template <int NT, bool TH>
__device__ __forceinline__ void cell_jac_any(CellCtx &cx, const double *y) {
  if (TH) cell_jac_th<NT>(cx, y);
  else cell_jac<NT>(cx, y);
}

template <int NT, bool TH>
__device__ __forceinline__ void cell_factor_any(CellCtx &cx, double c) {
  if (TH) cell_factor_th<NT>(cx, c);
  else cell_factor<NT>(cx, c);
}

// x = M^-1 x (or M^-T x) with the factors of cell_factor_any; x in LDS,
// cx.tmp and cx.scr as scratch.
template <int NT, bool TH>
__device__ __forceinline__ void cell_solve(CellCtx &cx, double *x, bool trans) {
  if (cx.front)
    front_solve<NT>(TH ? cx.n->fr_th : cx.n->fr, cx.M, cx.perm, x, cx.tmp, trans, cx.scr);
  else
    wg_solve<NT>(cx.M, cx.lda, cx.n->ns + (TH ? 1 : 0), cx.perm, x, cx.tmp, trans, cx.scr);
}

// Resampling matrix for a step change by `factor` (Shampine & Reichelt
// 1997): RU = R(factor) U with R(f)_{ij} = prod_{m=1..i} (m - 1 - f j)/m
// for j >= 1, R_{0j} = 1, R_{i0} = 0 (i > 0), and U = R(1); (q+1)^2
// entries with row stride QMAX+1 in LDS (cx.red + 16), formed by thread 0.
template <int NT>
__device__ __forceinline__ const double *resample_matrix(CellCtx &cx, int q, double factor) {
  constexpr int W = QMAX + 1;
  double *RU = cx.red + 16, *R = RU + W * W, *U = R + W * W;   // LDS
  if (threadIdx.x == 0) {
    for (int j = 0; j <= q; ++j) {
      R[j] = 1.0;
      U[j] = 1.0;
    }
    for (int i = 1; i <= q; ++i) {
      R[i * W] = 0.0;
      U[i * W] = 0.0;
      for (int j = 1; j <= q; ++j) {
        R[i * W + j] = R[(i - 1) * W + j] * ((i - 1 - factor * j) / i);
        U[i * W + j] = U[(i - 1) * W + j] * ((i - 1 - 1.0 * j) / i);
      }
    }
    for (int i = 0; i <= q; ++i)
      for (int j = 0; j <= q; ++j) {
        double s = 0.0;
        for (int m = 0; m <= q; ++m) s += R[i * W + m] * U[m * W + j];
        RU[i * W + j] = s;
      }
  }
  __syncthreads();
  return RU;
}

// Rows 0..q of a difference array X (global, row stride ns) times RU:
// X <- RU^T X (the resampling itself) or, with ADJ, X <- RU X (its
// transpose, for adjoint variables).
template <int NT, bool ADJ>
__device__ __forceinline__ void apply_resample(const double *RU, double *X, int q, int ns) {
  constexpr int W = QMAX + 1;
  for (int x = threadIdx.x; x < ns; x += NT) {
    double old[QMAX + 1];
#pragma unroll
    for (int i = 0; i <= QMAX; ++i) old[i] = i <= q ? X[size_t(i) * ns + x] : 0.0;
#pragma unroll
    for (int kk = 0; kk <= QMAX; ++kk) {
      if (kk > q) break;
      double s = 0.0;
#pragma unroll
      for (int i = 0; i <= QMAX; ++i)
        if (i <= q) s += (ADJ ? RU[kk * W + i] : RU[i * W + kk]) * old[i];
      X[size_t(kk) * ns + x] = s;
    }
  }
  __syncthreads();
}

// Resample D[0..q] for a step change by `factor`: D <- (R(factor) U)^T D.
template <int NT>
__device__ __forceinline__ void rescale_diffs(CellCtx &cx, int q, double factor, int ns) {
  apply_resample<NT, false>(resample_matrix<NT>(cx, q, factor), cx.D, q, ns);
}

// Accepted step of order q with corrector increment d (LDS):
// D_{q+2} = d - D_{q+1}, D_{q+1} = d, D_i += D_{i+1} for i = q..0.
template <int NT>
__device__ __forceinline__ void update_diffs(CellCtx &cx, int q, const double *d, int ns) {
  for (int x = threadIdx.x; x < ns; x += NT) {
    double *Dx = cx.D + x;
    Dx[size_t(q + 2) * ns] = d[x] - Dx[size_t(q + 1) * ns];
    Dx[size_t(q + 1) * ns] = d[x];
    for (int i = q; i >= 0; --i) Dx[size_t(i) * ns] += Dx[size_t(i + 1) * ns];
  }
  __syncthreads();
}

// Predictor y_pred = sum_{m<=q} D_m, error weights atol + rtol |y_pred| and
// psi = sum_{m=1..q} gamma_m D_m / alpha_q, into LDS.
template <int NT>
__device__ __forceinline__ void predict(const CellCtx &cx, int q, double rtol, double atol, int ns,
                                        double *yp, double *scl, double *psi) {
  double gam_m[QMAX + 1];
#pragma unroll
  for (int m = 0; m <= QMAX; ++m) gam_m[m] = bdf_gamma(m);
  const double alph_q = bdf_gamma(q);
  for (int x = threadIdx.x; x < ns; x += NT) {
    double s = 0.0;
    for (int m = 0; m <= q; ++m) s += cx.D[size_t(m) * ns + x];
    yp[x] = s;
    scl[x] = atol + rtol * fabs(s);
    double p = 0.0;
    for (int m = 1; m <= q; ++m) p += gam_m[m] * cx.D[size_t(m) * ns + x];
    psi[x] = p / alph_q;
  }
  __syncthreads();
}

}  // namespace ac
