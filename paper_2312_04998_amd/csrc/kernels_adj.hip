// Discrete adjoint of the batched BDF integrator for gfx950.
//
// The map differentiated is the integrator's own step sequence (orders,
// step sizes and every resampling of the difference array, as recorded in
// its tape) with each corrector equation solved exactly: step sizes and
// orders are constants, and every accepted step satisfies
//
//     G(d; D, p) = d - c f(y_pred(D) + d, p) + psi(D) = 0,   c = h / alpha_q,
//
// so by the implicit function theorem, with y = y_pred + d and
// M = I - c J(y), a cotangent dbar of d gives w = M^{-T} dbar and
//
//     ybar_pred = c J(y)^T w,   psibar = -w,   pbar_j = c R_j(y) (S^T w)_j
//
// for p = log alpha (dR_j / d log alpha_j = R_j). The difference-array
// operations (update after a step, resampling) are linear with recorded
// coefficients and are transposed directly. The first step D_1 = h0 f(y0)
// contributes h0 J(y0)^T Dbar_1 to dL/dy0 and h0 R_j (S^T Dbar_1)_j.
//
// One persistent workgroup handles one cell at a time (device queue). It
// replays the tape forward once with converged correctors, keeping the
// difference array every A.every accepted steps (the replay of a segment
// depends only on its checkpoint, so a recomputed segment repeats the first
// pass bit for bit); the reverse sweep then
// walks the segments backwards, recomputing each segment forward from its
// checkpoint (storing the converged y of every step) before reversing it.
// Each reverse step refactors M at the converged y and does one transposed
// solve and one VJP. The per-cell dL/dlog alpha rows are summed over cells
// in cell order by a separate reduction, so the result does not depend on
// which workgroup took which cell.
#include "devstep.h"

namespace ac {

// LDS vectors of one cell (ns doubles each).
struct AdjVecs {
  double *f, *yn, *dd, *psi, *scl, *yp, *dy;
};

// Converged corrector for a recorded step (q, h): Newton on G(d) = 0 until
// the update is at rounding level, then D advances. The Newton matrix
// carries over from the previous step with the integrator's reuse rule
// (refactored with the same Jacobian once |c/cM - 1| > 0.3, corrections
// scaled by 2/(1 + c/cM) in between) and J is refreshed at the current
// iterate whenever the contraction is slow; cM is the c of the factored
// matrix, 0 when there is none (J is then formed at y_pred).
// Every checkpointed segment starts from cM = 0, so a segment's replay
// depends only on its checkpoint and is bitwise repeatable. The converged
// y is left in v.yn. Stopping rules are the oracle's replay rules.
template <int NT>
__device__ __forceinline__ void replay_step(CellCtx &cx, const AdjVecs &v, int q, double h,
                                            double rtol, double atol, int ns, double &cM) {
  predict<NT>(cx, q, rtol, atol, ns, v.yp, v.scl, v.psi);
  const double c = h / bdf_gamma(q);
  for (int x = threadIdx.x; x < ns; x += NT) v.dd[x] = 0.0;
  __syncthreads();
  if (cM == 0.0) cell_jac<NT>(cx, v.yp);
  if (cM == 0.0 || fabs(c / cM - 1.0) > 0.3) {
    cell_factor<NT>(cx, c);
    cM = c;
  }
  double prev = INFINITY;
  bool refresh = false;
  for (int it = 0; it < 60; ++it) {
    for (int x = threadIdx.x; x < ns; x += NT) v.yn[x] = v.yp[x] + v.dd[x];
    __syncthreads();
    if (refresh) {
      cell_jac<NT>(cx, v.yn);
      cell_factor<NT>(cx, c);
      cM = c;
      refresh = false;
    }
    cell_rhs<NT>(cx, v.yn, v.f);
    cx.cnt[ST_NEWTON]++;
    for (int x = threadIdx.x; x < ns; x += NT) v.dy[x] = -(v.dd[x] - c * v.f[x] + v.psi[x]);
    __syncthreads();
    cell_solve<NT, false>(cx, v.dy, false);
    if (c != cM) {
      const double corr = 2.0 / (1.0 + c / cM);
      for (int x = threadIdx.x; x < ns; x += NT) v.dy[x] *= corr;
      __syncthreads();
    }
    const double dn = wg_rms<NT>(v.dy, 1.0, v.scl, ns, cx.red);
    for (int x = threadIdx.x; x < ns; x += NT) v.dd[x] += v.dy[x];
    __syncthreads();
    if (dn <= 1e-10) break;                       // converged
    if (dn <= 1e-7 && dn > 0.5 * prev) break;     // at rounding level
    if (dn > 0.1 * prev) refresh = true;          // slow: Jacobian at the iterate
    prev = dn;
  }
  for (int x = threadIdx.x; x < ns; x += NT) v.yn[x] = v.yp[x] + v.dd[x];
  __syncthreads();
  update_diffs<NT>(cx, q, v.dd, ns);
}

// u = J(y)^T w (LDS) and, when grow is set, grow_j += scale R_j(y) (S^T w)_j
// (one thread per reaction, so the per-cell row is accumulated in a fixed
// order). y, w, u in LDS; uses the scratch region for k_j (S^T w)_j.
template <int NT>
__device__ __forceinline__ void cell_vjp(CellCtx &cx, const double *y, const double *w, double *u,
                                         double *grow, double scale) {
  const DNet &n = *cx.n;
  double *kw = cx.rs, *part = cx.part;
  constexpr int U = 4;
  for (int j0 = threadIdx.x; j0 < n.nr; j0 += U * NT) {
    uint4 col[U];
    uint32_t pr[U];
    double kv[U];
#pragma unroll
    for (int u2 = 0; u2 < U; ++u2) {
      const int j = j0 + u2 * NT;
      const bool ok = j < n.nr;
      col[u2] = ok ? n.rxpack[2 * n.nr + j] : make_uint4(~0u, ~0u, ~0u, ~0u);
      pr[u2] = ok ? n.rpair[j] : 0u;
      kv[u2] = ok ? cx.kg[j] : 0.0;
    }
#pragma unroll
    for (int u2 = 0; u2 < U; ++u2) {
      const int j = j0 + u2 * NT;
      if (j >= n.nr) continue;
      const uint32_t w4[4] = {col[u2].x, col[u2].y, col[u2].z, col[u2].w};
      double sw = 0.0;
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const uint32_t hw = (w4[q >> 1] >> (16 * (q & 1))) & 0xFFFFu;
        if (hw != 0xFFFFu) {
          const int coef = int32_t(hw << 16) >> 27;
          sw += double(coef) * w[hw & 2047u];
        }
      }
      kw[j] = kv[u2] * sw;
      if (grow) grow[j] += scale * (reaction_rate(pr[u2], kv[u2], y) * sw);
    }
  }
  __syncthreads();
  segsum_chunks<NT, LAYOUT_SELL, false>(n.gy, kw, y, part, u);
  __syncthreads();
  segsum_finish<NT, false>(n.gy, part, u);
  __syncthreads();
}

// Reverse of an accepted step (q, h) whose converged y is in v.yn; Db is
// the slot's adjoint difference array (global).
template <int NT>
__device__ __forceinline__ void reverse_step(CellCtx &cx, const AdjVecs &v, double *Db, int q,
                                             double h, int ns, double *grow) {
  const double alph_q = bdf_gamma(q), c = h / alph_q;
  // transpose of the difference update: dbar = sum_{i<=q+2} Db_i,
  // Db_m <- sum_{i<=m} Db_i (m <= q), Db_{q+1} <- -Db_{q+2}, Db_{q+2} <- 0
  for (int x = threadIdx.x; x < ns; x += NT) {
    double *B = Db + x;
    double run = 0.0;
    for (int m = 0; m <= q; ++m) {
      run += B[size_t(m) * ns];
      B[size_t(m) * ns] = run;
    }
    const double b1 = B[size_t(q + 1) * ns], b2 = B[size_t(q + 2) * ns];
    v.dy[x] = run + b1 + b2;
    B[size_t(q + 1) * ns] = -b2;
    B[size_t(q + 2) * ns] = 0.0;
  }
  __syncthreads();
  // w = M(y)^{-T} dbar with M refactored at the converged y
  cell_jac<NT>(cx, v.yn);
  cell_factor<NT>(cx, c);
  cell_solve<NT, false>(cx, v.dy, true);
  cell_vjp<NT>(cx, v.yn, v.dy, v.f, grow, c);
  double gam_m[QMAX + 1];
#pragma unroll
  for (int m = 0; m <= QMAX; ++m) gam_m[m] = bdf_gamma(m);
  for (int x = threadIdx.x; x < ns; x += NT) {
    const double u = c * v.f[x], w = v.dy[x];
    for (int m = 0; m <= q; ++m) Db[size_t(m) * ns + x] += u - (gam_m[m] / alph_q) * w;
  }
  __syncthreads();
}

template <int NT, bool FR>
__global__ __launch_bounds__(NT) void k_adj(DNet n, const double *__restrict__ la_over,
                                            int64_t n_cells, AdjIO io, BdfParams P, WsView W,
                                            AdjView A, unsigned *queue) {
  extern __shared__ double sm[];
  const int ns = n.ns, nr = n.nr;
  double *f = sm, *yn = f + ns, *dd = yn + ns, *psi = dd + ns, *scl = psi + ns, *yp = scl + ns,
         *dy = yp + ns, *tmp = dy + ns, *scr = tmp + ns;
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
  cx.rs = scr;
  cx.part = scr + nr;
  cx.scr = scr;
  cx.tmp = tmp;
  cx.red = red;
  cx.redi = redi;
  cx.ipiv = ipiv;
  cx.front = FR;
  double *Db = A.Db + slot * A.db_stride;
  double *ck = A.ck + slot * A.ck_stride;
  int *ckev = A.ckev + slot * A.ckev_stride;
  double *segY = A.segY + slot * A.segy_stride;
  const AdjVecs v{f, yn, dd, psi, scl, yp, dy};
  const size_t dsz = size_t(NDROW) * ns;

  for (int64_t iter = 0;; ++iter) {
    if (threadIdx.x == 0)
      s_cell = queue ? int64_t(atomicAdd(queue, 1u)) : int64_t(blockIdx.x) + iter * gridDim.x;
    __syncthreads();
    const int64_t cell = s_cell;
    __syncthreads();
    if (cell >= n_cells) break;

    for (int i = 0; i < ST_N; ++i) cx.cnt[i] = 0;
    const double *y0 = io.y0 + cell * ns;
    const AcEvent *ev = io.ev + cell * io.cap;
    const int nev = io.len[cell];
    double *grow = io.g_cells ? io.g_cells + cell * nr : nullptr;
    bool bad = false;
    for (int i = threadIdx.x; i < ns; i += NT) {
      const double y = y0[i];
      if (!(isfinite(y) && y >= 0.0)) bad = true;
    }
    bad = wg_any<NT>(bad, red) || !cell_env_ok(io.T, cell, n.n_cond);
    // a tape that overflowed, or holds an order outside 1..QMAX, is not replayed
    bool badtape = nev < 0 || nev > io.cap;
    if (!badtape) {
      for (int e = threadIdx.x; e < nev; e += NT) {
        const AcEvent E = ev[e];
        if ((E.type == EV_STEP || E.type == EV_RESCALE) && (E.q < 1 || E.q > QMAX)) badtape = true;
      }
      badtape = wg_any<NT>(badtape, red);
    }
    int status = bad ? AC_CELL_BADINPUT : (badtape ? AC_CELL_TAPE : AC_CELL_OK);
    if (grow)
      for (int j = threadIdx.x; j < nr; j += NT) grow[j] = 0.0;
    for (int x = threadIdx.x; x < ns; x += NT) {
      Db[x] = io.lam ? io.lam[cell * ns + x] : 0.0;
      for (int m = 1; m < NDROW; ++m) Db[size_t(m) * ns + x] = 0.0;
    }
    __syncthreads();
    if (status == AC_CELL_OK && nev > 0) {
      const Env env = cell_env(io.T, cell, n.n_cond);
      for_reactions<NT>(n, la_over, env, [&](int j, double kj, uint32_t) { cx.kg[j] = kj; });
      for (int x = threadIdx.x; x < ns; x += NT) {
        cx.D[x] = y0[x];
        for (int m = 1; m < NDROW; ++m) cx.D[size_t(m) * ns + x] = 0.0;
      }
      __syncthreads();
      // forward replay with checkpoints every A.every accepted steps
      const int every = A.every;
      int nck = 0, nstep = 0;   // nck <= cap / every + 1 <= A.ckcap since nstep <= nev <= cap
      double cM = 0.0;
      for (int e = 0; e < nev; ++e) {
        const AcEvent E = ev[e];
        if (E.type == EV_STEP) {
          if (nstep % every == 0) {
            double *dst = ck + size_t(nck) * dsz;
            for (size_t i = threadIdx.x; i < dsz; i += NT) dst[i] = cx.D[i];
            if (threadIdx.x == 0) ckev[nck] = e;
            ++nck;
            cM = 0.0;
          }
          replay_step<NT>(cx, v, E.q, E.val, P.rtol, P.atol, ns, cM);
          if (A.all_states && io.gy0)   // nstep < nev <= cap = segcap
            for (int x = threadIdx.x; x < ns; x += NT) segY[size_t(nstep) * ns + x] = yn[x];
          ++nstep;
        } else if (E.type == EV_RESCALE) {
          rescale_diffs<NT>(cx, E.q, E.val, ns);
        } else if (E.type == EV_INIT) {
          for (int x = threadIdx.x; x < ns; x += NT) yn[x] = y0[x];
          __syncthreads();
          cell_rhs<NT>(cx, yn, f);
          for (int x = threadIdx.x; x < ns; x += NT) cx.D[size_t(ns) + x] = E.val * f[x];
          __syncthreads();
        }
      }
      if (io.y_final)
        for (int x = threadIdx.x; x < ns; x += NT) io.y_final[cell * ns + x] = cx.D[x];
      __syncthreads();
      // reverse sweep, one checkpointed segment at a time (skipped when only
      // the replayed state is asked for)
      int e_end = io.gy0 ? nev : 0;
      for (int s = io.gy0 ? nck - 1 : -1; s >= 0; --s) {
        const int e0 = ckev[s];
        int i = 0;
        const double *sy = segY;
        if (A.all_states) {
          // the forward pass kept them: segment s is steps s*every ...
          sy = segY + size_t(s) * every * ns;
          i = s + 1 < nck ? every : nstep - s * every;
        } else {
          const double *src = ck + size_t(s) * dsz;
          for (size_t k = threadIdx.x; k < dsz; k += NT) cx.D[k] = src[k];
          __syncthreads();
          double cM = 0.0;
          for (int e = e0; e < e_end; ++e) {
            const AcEvent E = ev[e];
            if (E.type == EV_STEP) {
              replay_step<NT>(cx, v, E.q, E.val, P.rtol, P.atol, ns, cM);
              for (int x = threadIdx.x; x < ns; x += NT) segY[size_t(i) * ns + x] = yn[x];
              ++i;
            } else if (E.type == EV_RESCALE) {
              rescale_diffs<NT>(cx, E.q, E.val, ns);
            }
          }
        }
        __syncthreads();
        for (int e = e_end - 1; e >= e0; --e) {
          const AcEvent E = ev[e];
          if (E.type == EV_STEP) {
            --i;
            for (int x = threadIdx.x; x < ns; x += NT) yn[x] = sy[size_t(i) * ns + x];
            __syncthreads();
            reverse_step<NT>(cx, v, Db, E.q, E.val, ns, grow);
            cx.cnt[ST_STEPS]++;
          } else if (E.type == EV_RESCALE) {
            apply_resample<NT, true>(resample_matrix<NT>(cx, E.q, E.val), Db, E.q, ns);
          }
        }
        e_end = e0;
      }
      // events before the first accepted step: resamplings and the start
      for (int e = e_end - 1; io.gy0 && e >= 0; --e) {
        const AcEvent E = ev[e];
        if (E.type == EV_RESCALE) {
          apply_resample<NT, true>(resample_matrix<NT>(cx, E.q, E.val), Db, E.q, ns);
        } else if (E.type == EV_INIT) {
          // D_1 = h0 f(y0): dL/dy0 += h0 J(y0)^T Db_1, pbar += h0 R (S^T Db_1)
          for (int x = threadIdx.x; x < ns; x += NT) {
            yn[x] = y0[x];
            dy[x] = Db[size_t(ns) + x];
          }
          __syncthreads();
          cell_vjp<NT>(cx, yn, dy, f, grow, E.val);
          for (int x = threadIdx.x; x < ns; x += NT) {
            Db[x] += E.val * f[x];
            Db[size_t(ns) + x] = 0.0;
          }
          __syncthreads();
        }
      }
    } else if (io.y_final) {
      for (int x = threadIdx.x; x < ns; x += NT) io.y_final[cell * ns + x] = y0[x];
    }
    if (io.gy0)
      for (int x = threadIdx.x; x < ns; x += NT) io.gy0[cell * ns + x] = Db[x];
    if (threadIdx.x == 0 && io.status) io.status[cell] = status;
    if (threadIdx.x == 0 && io.stats) {
      int *st = io.stats + cell * ST_N;
      for (int i = 0; i < ST_N; ++i) st[i] = cx.cnt[i];
    }
    __syncthreads();
  }
}

hipError_t launch_adjoint(const DNet &n, const double *la, int64_t n_cells, const AdjIO &io,
                          const BdfParams &P, const WsView &W, const AdjView &A, unsigned *queue,
                          int grid, hipStream_t st) {
  if (n_cells == 0) return hipSuccess;
  const size_t lds = bdf_lds_bytes(n);
  auto kern = use_front(n, P) ? k_adj<BDF_NT, true> : k_adj<BDF_NT, false>;
  if (lds > 65536) hipFuncSetAttribute(reinterpret_cast<const void *>(kern),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, int(lds));
  hipError_t e = launch_reset_queue(queue, st);
  if (e != hipSuccess) return e;
  const int g = int(n_cells < grid ? n_cells : grid);
  hipLaunchKernelGGL(kern, dim3(g), dim3(BDF_NT), lds, st, n, la, n_cells, io, P, W, A, queue);
  return hipGetLastError();
}

}  // namespace ac
