// Batched stiff integrator for gfx950: variable-order (1..5) BDF in
// backward-difference form with a simplified Newton corrector on the
// Newton matrix I - c J: a sparse front swept in levels and the dense Schur
// tail factored on the FP64 matrix cores (devfront.h), or one dense LU.
//
// The paper integrates every cell with DLSODES (Sec. 3) and precomputes the
// rate coefficients outside the solver; here one persistent workgroup
// integrates one cell at a time, pulling cell indices from a device queue
// so cells with many steps do not hold up the others. The coefficients are
// computed once per cell; every RHS, Jacobian, factorisation and solve of
// the cell then runs inside the same workgroup. Per-slot state (Newton
// matrix, Jacobian values, difference array, coefficients) lives in a
// global workspace slot; vectors of one cell live in LDS.
//
// Step, order and Newton rules (identical on the CPU oracle):
//   gamma_q = sum_{m<=q} 1/m, alpha_q = gamma_q, error constant 1/(q+1)
//   corrector d - c f(y_pred + d) + psi = 0, c = h/alpha_q,
//     psi = sum_{m=1..q} gamma_m D_m / alpha_q; simplified Newton with
//     M = I - c J, <= 4 iterations, convergence-rate test with tolerance
//     max(10 eps/rtol, min(0.03, sqrt(rtol)))
//   Newton failure: refresh J at y_pred once per attempt, then halve h
//   error test: RMS of d/(atol + rtol|y_new|)/(q+1) <= 1; step factor
//     safety * err^(-1/(q+1)) in [0.2, 10], safety = 0.9*9/(8 + iterations)
//   order change after q+1 equal steps, to the best of q-1, q, q+1
//   M = I - c_M J kept while |c/c_M - 1| <= 0.3, refactored when c moves
//   further or J is refreshed (J only on Newton failure); with c != c_M
//   each Newton correction is scaled by 2/(1 + c/c_M) (the matrix-reuse
//   rule of the LSODE family, to which the paper's DLSODES belongs).
#include "devstep.h"

namespace ac {

__device__ __forceinline__ void tape_put(const TapeView &tv, int64_t cell, int &len, int type,
                                         int q, double val) {
  if (!tv.ev) return;
  if (threadIdx.x == 0 && len < tv.cap) {
    AcEvent *e = tv.ev + cell * tv.cap + len;
    e->type = type;
    e->q = q;
    e->val = val;
  }
  ++len;
}

// TH: temperature-coupled mode, the state is (n_1..n_ns, T) and therm
// holds (c_v, T_b, lambda) per cell; otherwise T is held at the cell's
// conditions. ns below is the length of the state vector. FR: the Newton
// matrix is factored with the sparse front (a separate instance, so that
// the dense path keeps its own register allocation).
template <int NT, bool TH, bool FR>
__global__ __launch_bounds__(NT) void k_bdf(DNet n, const double *__restrict__ la_over,
                                            int64_t n_cells, double *__restrict__ y,
                                            const double *__restrict__ T,
                                            const double *__restrict__ therm, BdfParams P,
                                            CellOut out, TapeView tv, WsView W,
                                            unsigned *queue) {
  extern __shared__ double sm[];
  const int ns = n.ns + (TH ? 1 : 0), nr = n.nr;
  double *f = sm, *yn = f + ns, *dd = yn + ns, *psi = dd + ns, *scl = psi + ns, *yp = scl + ns,
         *dy = yp + ns, *tmp = dy + ns, *scr = tmp + ns;
  double *rs = scr, *part = scr + nr;        // RHS use of the scratch region
  double *red = scr + bdf_scratch_doubles(n);
  int *redi = reinterpret_cast<int *>(red + 16 + 3 * (QMAX + 1) * (QMAX + 1));
  int *ipiv = redi + 16;
  __shared__ int64_t s_cell;

  const size_t slot = blockIdx.x;
  CellCtx cx;
  cx.n = &n;
  cx.kg = W.k + slot * W.k_stride;
  cx.Jg = W.J + slot * W.j_stride;
  cx.tailp = W.tail + slot * W.tail_stride;
  cx.M = W.M + slot * W.m_stride;
  cx.piv = W.piv + slot * W.piv_stride;
  cx.perm = cx.piv + ns;
  cx.D = W.D + slot * W.d_stride;
  cx.lda = W.lda;
  cx.rs = rs;
  cx.part = part;
  cx.scr = scr;
  cx.tmp = tmp;
  cx.red = red;
  cx.redi = redi;
  cx.ipiv = ipiv;
  cx.nc = n.n_cond;
  cx.la_over = la_over;
  cx.Jaux = cx.Jg + n.nnz_j;
  cx.front = FR;
  const double rtol = P.rtol, atol = P.atol, t_end = P.t_end;
  const double tol = P.newton_tol > 0.0
                         ? P.newton_tol
                         : fmax(10.0 * 2.220446049250313e-16 / rtol, fmin(0.03, sqrt(rtol)));

  for (int64_t iter = 0;; ++iter) {
    if (threadIdx.x == 0) {
      int64_t pos = queue ? int64_t(atomicAdd(queue, 1u)) : int64_t(blockIdx.x) + iter * gridDim.x;
      // progress for the host: a system-scope store to the pinned word
      if (W.progress && pos < n_cells)
        __hip_atomic_store(W.progress, unsigned(pos + 1), __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_SYSTEM);
      s_cell = (P.order && pos < n_cells) ? int64_t(P.order[pos]) : pos;
    }
    __syncthreads();
    const int64_t cell = s_cell;
    __syncthreads();
    if (cell >= n_cells) break;

    for (int i = 0; i < ST_N; ++i) cx.cnt[i] = 0;
    int tlen = 0;
    double *ycell = y + cell * ns;
    bool bad = false;
    for (int i = threadIdx.x; i < ns; i += NT) {
      const double v = ycell[i];
      if (!(isfinite(v) && v >= 0.0)) bad = true;
    }
    bad = wg_any<NT>(bad, red) || !cell_env_ok(T, cell, n.n_cond);
    if (TH) {
      const double *th = therm + cell * 3, Tc = ycell[n.ns];
      bad = bad || !(Tc > 0.0 && isfinite(th[0]) && th[0] > 0.0 && isfinite(th[1]) &&
                     th[1] > 0.0 && isfinite(th[2]) && th[2] >= 0.0);
      cx.cond = T + cell * n.n_cond;
      cx.cv = th[0];
      cx.Tb = th[1];
      cx.lam = th[2];
    }
    int status = AC_CELL_OK, q = 1, steps = 0;
    const bool run = !bad && t_end > 0.0;
    if (bad) status = AC_CELL_BADINPUT;
    if (run) {
      if (!TH) {
        const Env env = cell_env(T, cell, n.n_cond);
        for_reactions<NT>(n, la_over, env, [&](int j, double kj, uint32_t) { cx.kg[j] = kj; });
      }
      for (int x = threadIdx.x; x < ns; x += NT) {
        const double v = ycell[x];
        yn[x] = v;
        cx.D[x] = v;
        for (int m = 1; m < NDROW; ++m) cx.D[size_t(m) * ns + x] = 0.0;
      }
      __syncthreads();
      cell_rhs_any<NT, TH>(cx, yn, f);
      // first step (Hairer, Norsett & Wanner, Sec. II.4, order 1)
      double h;
      if (P.h0 > 0.0) {
        h = fmin(P.h0, t_end);
      } else {
        for (int x = threadIdx.x; x < ns; x += NT) scl[x] = atol + rtol * fabs(yn[x]);
        __syncthreads();
        const double d0 = wg_rms<NT>(yn, 1.0, scl, ns, red);
        const double d1 = wg_rms<NT>(f, 1.0, scl, ns, red);
        double h0 = (d0 < 1e-5 || d1 < 1e-5) ? 1e-6 : 0.01 * d0 / d1;
        if (h0 > t_end) h0 = t_end;
        for (int x = threadIdx.x; x < ns; x += NT) yp[x] = yn[x] + h0 * f[x];
        __syncthreads();
        cell_rhs_any<NT, TH>(cx, yp, dy);
        for (int x = threadIdx.x; x < ns; x += NT) dy[x] -= f[x];
        __syncthreads();
        const double d2 = wg_rms<NT>(dy, 1.0, scl, ns, red) / h0;
        const double h1 = (d1 <= 1e-15 && d2 <= 1e-15) ? fmax(1e-6, h0 * 1e-3)
                                                         : pow(0.01 / fmax(d1, d2), 1.0 / 2.0);
        h = fmin(fmin(100.0 * h0, h1), t_end);
      }
      tape_put(tv, cell, tlen, EV_INIT, 1, h);
      for (int x = threadIdx.x; x < ns; x += NT) cx.D[size_t(ns) + x] = h * f[x];
      __syncthreads();
      cell_jac_any<NT, TH>(cx, yn);

      int n_equal = 0;
      // why the last attempt was rejected, the status if h falls below h_min
      int last_fail = AC_CELL_HMIN;
      bool lu_valid = false;
      double cM = 0.0;   // c of the factored Newton matrix
      double t = 0.0, h_abs = h;
      while (t < t_end) {
        if (steps >= P.max_steps) {
          status = AC_CELL_MAXSTEPS;
          break;
        }
        const double hmin = 10.0 * (nextafter(t, INFINITY) - t);
        bool jac_fresh = false;
        int n_iter = 0;
        double t_new = t, en = 0.0, safety = 0.0;
        bool failed = false;
        for (;;) {   // attempts
          if (h_abs < hmin) {
            status = last_fail;
            failed = true;
            break;
          }
          t_new = t + h_abs;
          if (t_new > t_end) {
            t_new = t_end;
            const double factor = (t_new - t) / h_abs;
            rescale_diffs<NT>(cx, q, factor, ns);
            tape_put(tv, cell, tlen, EV_RESCALE, q, factor);
            n_equal = 0;
          }
          h = t_new - t;
          h_abs = h;
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
          const double c = h / alph_q;
          bool conv = false, nonfin = false;
          for (;;) {
            if (!lu_valid || fabs(c / cM - 1.0) > 0.3) {
              cell_factor_any<NT, TH>(cx, c);
              lu_valid = true;
              cM = c;
            }
            const double corr = c == cM ? 1.0 : 2.0 / (1.0 + c / cM);
            // simplified Newton
            for (int x = threadIdx.x; x < ns; x += NT) {
              yn[x] = yp[x];
              dd[x] = 0.0;
            }
            __syncthreads();
            double prev = 0.0;
            int it;
            for (it = 0; it < NEWTON_MAXITER; ++it) {
              cell_rhs_any<NT, TH>(cx, yn, f);
              bool nonfinite = false;
              for (int x = threadIdx.x; x < ns; x += NT)
                if (!isfinite(f[x])) nonfinite = true;
              nonfin = wg_any<NT>(nonfinite, red);
              if (nonfin) break;
              for (int x = threadIdx.x; x < ns; x += NT) dy[x] = c * f[x] - psi[x] - dd[x];
              __syncthreads();
              cell_solve<NT, TH>(cx, dy, false);
              if (corr != 1.0) {
                for (int x = threadIdx.x; x < ns; x += NT) dy[x] *= corr;
                __syncthreads();
              }
              const double dn = wg_rms<NT>(dy, 1.0, scl, ns, red);
              double rate = 0.0;
              if (it > 0) {
                rate = dn / prev;
                if (rate >= 1.0 || pow(rate, double(NEWTON_MAXITER - it)) / (1.0 - rate) * dn > tol)
                  break;
              }
              for (int x = threadIdx.x; x < ns; x += NT) {
                yn[x] += dy[x];
                dd[x] += dy[x];
              }
              __syncthreads();
              if (dn == 0.0 || (it > 0 && rate / (1.0 - rate) * dn < tol)) {
                conv = true;
                break;
              }
              prev = dn;
            }
            n_iter = it + 1;
            cx.cnt[ST_NEWTON] += it < NEWTON_MAXITER ? it + 1 : NEWTON_MAXITER;
            if (conv || jac_fresh) break;
            cell_jac_any<NT, TH>(cx, yp);
            jac_fresh = true;
            lu_valid = false;
          }
          if (!conv) {
            last_fail = cx.lu_info ? AC_CELL_SINGULAR : nonfin ? AC_CELL_NONFINITE
                                                               : AC_CELL_NEWTON_FAIL;
            h_abs *= 0.5;
            rescale_diffs<NT>(cx, q, 0.5, ns);
            tape_put(tv, cell, tlen, EV_RESCALE, q, 0.5);
            n_equal = 0;
            cx.cnt[ST_REJ_NEWTON]++;
            continue;
          }
          safety = 0.9 * (2 * NEWTON_MAXITER + 1) / (2 * NEWTON_MAXITER + n_iter);
          for (int x = threadIdx.x; x < ns; x += NT) scl[x] = atol + rtol * fabs(yn[x]);
          __syncthreads();
          en = wg_rms<NT>(dd, bdf_errc(q), scl, ns, red);
          if (en > 1.0) {
            last_fail = AC_CELL_HMIN;
            const double factor = fmax(MIN_FACTOR, safety * pow_neg(en, 1.0 / (q + 1)));
            h_abs *= factor;
            rescale_diffs<NT>(cx, q, factor, ns);
            tape_put(tv, cell, tlen, EV_RESCALE, q, factor);
            n_equal = 0;
            cx.cnt[ST_REJ_ERR]++;
            continue;
          }
          break;
        }
        if (failed) break;
        // accepted
        t = t_new;
        ++steps;
        tape_put(tv, cell, tlen, EV_STEP, q, h);
        for (int x = threadIdx.x; x < ns; x += NT) {
          double *Dx = cx.D + x;
          Dx[size_t(q + 2) * ns] = dd[x] - Dx[size_t(q + 1) * ns];
          Dx[size_t(q + 1) * ns] = dd[x];
          for (int i = q; i >= 0; --i) Dx[size_t(i) * ns] += Dx[size_t(i + 1) * ns];
        }
        __syncthreads();
        ++n_equal;
        if (n_equal < q + 1) continue;
        const double em = q > 1 ? wg_rms<NT>(cx.D + size_t(q) * ns, bdf_errc(q - 1), scl, ns, red) : INFINITY;
        const double ep = q < P.q_max ? wg_rms<NT>(cx.D + size_t(q + 2) * ns, bdf_errc(q + 1), scl, ns, red) : INFINITY;
        const double fac[3] = {pow_neg(em, 1.0 / q), pow_neg(en, 1.0 / (q + 1)),
                               pow_neg(ep, 1.0 / (q + 2))};
        int best = 0;
        for (int i = 1; i < 3; ++i)
          if (fac[i] > fac[best]) best = i;
        q += best - 1;
        const double factor = fmin(MAX_FACTOR, safety * fac[best]);
        h_abs *= factor;
        rescale_diffs<NT>(cx, q, factor, ns);
        tape_put(tv, cell, tlen, EV_RESCALE, q, factor);
        n_equal = 0;
      }
      for (int x = threadIdx.x; x < ns; x += NT) ycell[x] = cx.D[x];
      __syncthreads();
    }
    if (threadIdx.x == 0) {
      if (out.status) out.status[cell] = status;
      if (out.stats) {
        int *st = out.stats + cell * ST_N;
        for (int i = 0; i < ST_N; ++i) st[i] = cx.cnt[i];
        st[ST_STEPS] = steps;
        st[ST_QLAST] = run ? q : 0;
      }
      if (tv.len) tv.len[cell] = tlen > tv.cap ? -1 : tlen;
    }
    __syncthreads();
  }
}

// The integrator's Newton systems on their own: matrix m is I - c[m] J_m
// with J_m's pattern values at jvals + m nnz_j; b [n_mat][ns] is solved in
// place, plainly or transposed. Workgroup g uses slot g and takes the
// matrices g, g + grid, ...
template <int NT, bool FR>
__global__ __launch_bounds__(NT) void k_newton(DNet n, int64_t n_mat, const double *__restrict__ jvals,
                                               const double *__restrict__ c, double *__restrict__ b,
                                               int trans, WsView W, int32_t *__restrict__ info) {
  extern __shared__ double sm[];
  const int ns = n.ns;
  double *x = sm, *tmp = x + ns, *scr = tmp + ns;
  double *red = scr + bdf_scratch_doubles(n);
  int *redi = reinterpret_cast<int *>(red + 16 + 3 * (QMAX + 1) * (QMAX + 1));
  int *ipiv = redi + 16;
  const size_t slot = blockIdx.x;
  CellCtx cx;
  cx.n = &n;
  cx.M = W.M + slot * W.m_stride;
  cx.piv = W.piv + slot * W.piv_stride;
  cx.perm = cx.piv + ns;
  cx.lda = W.lda;
  cx.scr = scr;
  cx.tmp = tmp;
  cx.red = red;
  cx.redi = redi;
  cx.ipiv = ipiv;
  cx.front = FR;
  for (int64_t m = blockIdx.x; m < n_mat; m += gridDim.x) {
    cx.Jg = const_cast<double *>(jvals) + m * n.nnz_j;
    cell_factor<NT>(cx, c[m]);
    for (int i = threadIdx.x; i < ns; i += NT) x[i] = b[m * ns + i];
    __syncthreads();
    cell_solve<NT, false>(cx, x, trans != 0);
    for (int i = threadIdx.x; i < ns; i += NT) b[m * ns + i] = x[i];
    if (threadIdx.x == 0 && info) info[m] = cx.lu_info;
    __syncthreads();
  }
}

hipError_t launch_newton(const DNet &n, int64_t n_mat, const double *jvals, const double *c,
                         double *b, int trans, bool front, const WsView &W, int slots,
                         int32_t *info, hipStream_t st) {
  if (n_mat == 0) return hipSuccess;
  const size_t lds = bdf_lds_bytes(n);
  auto kern = front ? k_newton<BDF_NT, true> : k_newton<BDF_NT, false>;
  if (lds > 65536) hipFuncSetAttribute(reinterpret_cast<const void *>(kern),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, int(lds));
  const int g = int(n_mat < slots ? n_mat : slots);
  hipLaunchKernelGGL(kern, dim3(g), dim3(BDF_NT), lds, st, n, n_mat, jvals, c, b, trans, W, info);
  return hipGetLastError();
}

__global__ void k_reset_queue(unsigned *q, unsigned *progress) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    *q = 0u;
    if (progress) __hip_atomic_store(progress, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
  }
}

// ------------------------------------------------------- standalone LU

template <int NT>
__global__ __launch_bounds__(NT) void k_lu_factor(int n, int lda, int64_t nmat, double *A,
                                                  int *piv, int *info) {
  extern __shared__ double sm[];
  __shared__ double red[NT / 64];
  __shared__ int redi[NT / 64];
  __shared__ int ipiv[9 * PW + 2];
  for (int64_t m = blockIdx.x; m < nmat; m += gridDim.x) {
    int *pm = piv + size_t(m) * n;
    const int inf = wg_lu<NT>(A + size_t(m) * n * lda, lda, n, pm, nullptr, sm, red, redi, ipiv);
    if (threadIdx.x == 0 && info) info[m] = inf;
    __syncthreads();
  }
}

template <int NT>
__global__ __launch_bounds__(NT) void k_lu_solve(int n, int lda, int64_t nmat, const double *LU,
                                                 const int *piv, double *b, int trans) {
  extern __shared__ double sm[];
  double *x = sm, *tmp = sm + n, *blk = tmp + n;
  int *perm = reinterpret_cast<int *>(blk + 3 * SB * SBP);
  for (int64_t m = blockIdx.x; m < nmat; m += gridDim.x) {
    const int *pv = piv + size_t(m) * n;
    if (threadIdx.x == 0) {
      for (int i = 0; i < n; ++i) perm[i] = i;
      for (int k = 0; k < n; ++k) {
        const int p = pv[k], t = perm[k];
        perm[k] = perm[p];
        perm[p] = t;
      }
    }
    double *bm = b + size_t(m) * n;
    for (int i = threadIdx.x; i < n; i += NT) x[i] = bm[i];
    __syncthreads();
    wg_solve<NT>(LU + size_t(m) * n * lda, lda, n, perm, x, tmp, trans != 0, blk);
    for (int i = threadIdx.x; i < n; i += NT) bm[i] = x[i];
    __syncthreads();
  }
}

// ---------------------------------------------------------------- launch

// LDS of the integrator and adjoint kernels: 8 state vectors (room for the
// temperature of the coupled mode), the shared scratch region, reductions.
size_t bdf_lds_bytes(const DNet &n) {
  return sizeof(double) * (size_t(8) * (n.ns + 1) + bdf_scratch_doubles(n) + 16 +
                           3 * (QMAX + 1) * (QMAX + 1)) +
         sizeof(int) * (16 + 9 * PW + 2);
}

int bdf_resident_blocks(const DNet &n) {
  const size_t lds = bdf_lds_bytes(n);
  if (lds > 65536) hipFuncSetAttribute(reinterpret_cast<const void *>(k_bdf<BDF_NT, false, false>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, int(lds));
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_bdf<BDF_NT, false, false>, BDF_NT, lds) !=
          hipSuccess || per_cu <= 0)
    per_cu = 1;
  int dev = 0, cus = 0;
  hipGetDevice(&dev);
  hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  return per_cu * (cus > 0 ? cus : 256);
}

hipError_t launch_bdf(const DNet &n, const double *la, int64_t n_cells, double *y, const double *T,
                      const double *therm, const BdfParams &P, const CellOut &out,
                      const TapeView &tv, const WsView &W, unsigned *queue, int grid,
                      hipStream_t st) {
  if (n_cells == 0) return hipSuccess;
  const size_t lds = bdf_lds_bytes(n);
  auto kern = therm ? (use_front_th(n, P) ? k_bdf<BDF_NT, true, true> : k_bdf<BDF_NT, true, false>)
                    : use_front(n, P) ? k_bdf<BDF_NT, false, true> : k_bdf<BDF_NT, false, false>;
  if (lds > 65536) hipFuncSetAttribute(reinterpret_cast<const void *>(kern),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, int(lds));
  if (queue) hipLaunchKernelGGL(k_reset_queue, dim3(1), dim3(64), 0, st, queue, W.progress);
  const int g = int(n_cells < grid ? n_cells : grid);
  hipLaunchKernelGGL(kern, dim3(g), dim3(BDF_NT), lds, st, n, la, n_cells, y, T, therm, P, out, tv,
                     W, queue);
  return hipGetLastError();
}

hipError_t launch_reset_queue(unsigned *queue, hipStream_t st) {
  if (!queue) return hipSuccess;
  hipLaunchKernelGGL(k_reset_queue, dim3(1), dim3(64), 0, st, queue, nullptr);
  return hipGetLastError();
}

hipError_t launch_lu_factor(int n, int lda, int64_t nmat, double *A, int *piv, int *info,
                            hipStream_t st) {
  if (nmat == 0) return hipSuccess;
  const int g = int(nmat < 4096 ? nmat : 4096);
  const size_t lds = sizeof(double) * size_t(la_scratch_doubles(n));
  if (lds > 65536) hipFuncSetAttribute(reinterpret_cast<const void *>(k_lu_factor<BDF_NT>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, int(lds));
  hipLaunchKernelGGL(k_lu_factor<BDF_NT>, dim3(g), dim3(BDF_NT), lds, st, n, lda, nmat, A, piv, info);
  return hipGetLastError();
}

hipError_t launch_lu_solve(int n, int lda, int64_t nmat, const double *LU, const int *piv,
                           double *b, int trans, hipStream_t st) {
  if (nmat == 0) return hipSuccess;
  const int g = int(nmat < 4096 ? nmat : 4096);
  const size_t lds = sizeof(double) * (size_t(2) * n + 3 * SB * SBP) + sizeof(int) * size_t(n);
  if (lds > 65536) hipFuncSetAttribute(reinterpret_cast<const void *>(k_lu_solve<BDF_NT>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, int(lds));
  hipLaunchKernelGGL(k_lu_solve<BDF_NT>, dim3(g), dim3(BDF_NT), lds, st, n, lda, nmat, LU, piv, b,
                     trans);
  return hipGetLastError();
}

}  // namespace ac
