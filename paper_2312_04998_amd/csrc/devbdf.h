// Integrator data shared by the host API and the BDF kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "../../include/astrochem.h"
#include "devnet.h"

namespace ac {

constexpr int BDF_NT = 512;   // threads per integrator workgroup (8 wavefronts)

// per-cell counters, same order as the public ac_stat enum
enum { ST_STEPS = 0, ST_REJ_ERR, ST_REJ_NEWTON, ST_NEWTON, ST_JAC, ST_LU, ST_RHS, ST_QLAST, ST_N };
enum { EV_INIT = 1, EV_RESCALE = 2, EV_STEP = 3 };

struct AcEvent {
  int32_t type, q;
  double val;
};

struct BdfParams {
  double rtol, atol, h0, t_end;
  int q_max, max_steps;
  double newton_tol;   // <= 0: max(10 eps/rtol, min(0.03, sqrt(rtol)))
  const int32_t *order = nullptr;   // queue position -> cell, or null (index order)
  int linear_solver = 0;   // AC_LINSOLVE_*
};

struct CellOut {
  int32_t *status;   // [n_cells] or null
  int32_t *stats;    // [n_cells][ST_N] or null
};

struct TapeView {
  AcEvent *ev;       // [n_cells][cap] or null
  int32_t *len;      // [n_cells] or null
  int cap;
};

// Global workspace slots (one per resident workgroup).
struct WsView {
  double *M, *J, *tail, *D, *k;
  int *piv;         // per slot: pivots [ns] then the row permutation [ns]
  size_t m_stride, j_stride, tail_stride, d_stride, k_stride, piv_stride;
  int lda;
  unsigned *progress;   // pinned host word: 1 + the last cell taken (or null)
};

// Discrete adjoint: per-slot buffers (checkpoints every `every` accepted
// steps, the converged states of one segment or of the whole tape, the
// adjoint difference array). CK_EVERY is the default interval.
constexpr int CK_EVERY = 64;

struct AdjView {
  double *Db, *ck, *segY;
  int *ckev;
  size_t db_stride, ck_stride, segy_stride, ckev_stride;
  int ckcap;        // checkpoints per slot
  int every;        // accepted steps between checkpoints
  int segcap;       // converged states per slot: every, or every step of a tape
  int all_states;   // 1: the forward pass keeps every state, so no segment is recomputed
};

struct AdjIO {
  const AcEvent *ev;      // [n_cells][cap]
  const int32_t *len;     // [n_cells]
  int cap;
  const double *y0, *T, *lam;   // [n_cells][ns], [n_cells], [n_cells][ns]
  double *y_final;        // [n_cells][ns] or null (replayed y(t_end))
  double *gy0;            // [n_cells][ns]
  double *g_cells;        // [n_cells][nr] or null
  int32_t *status;        // [n_cells] or null
  int32_t *stats;         // [n_cells][ST_N] or null
};

size_t bdf_lds_bytes(const DNet &n);
// Whether the integrator and the adjoint factor with the sparse front (the
// plan has one and the options ask for AUTO); selects the kernel instance.
inline bool use_front(const DNet &n, const BdfParams &P) {
  return P.linear_solver == AC_LINSOLVE_AUTO && n.fr.n == n.ns && n.fr.n1 > 0;
}
// The same for the temperature-coupled state (species + T).
inline bool use_front_th(const DNet &n, const BdfParams &P) {
  return P.linear_solver == AC_LINSOLVE_AUTO && n.fr_th.n == n.ns + 1 && n.fr_th.n1 > 0 &&
         n.fr_th.tcol_dst != nullptr;
}
int bdf_resident_blocks(const DNet &n);
// therm non-null selects the temperature-coupled mode (state ns + 1 per
// cell, therm [n_cells][3] = (c_v, T_b, lambda)).
hipError_t launch_bdf(const DNet &n, const double *la, int64_t n_cells, double *y, const double *T,
                      const double *therm, const BdfParams &P, const CellOut &out,
                      const TapeView &tv, const WsView &W, unsigned *queue, int grid,
                      hipStream_t st);
hipError_t launch_reset_queue(unsigned *queue, hipStream_t st);
// Newton systems (I - c J) x = b (or transposed) with the integrator's
// factorisation, one matrix per workspace slot at a time; info [n_mat] or
// null gets 0 or 1 + a zero pivot's position.
hipError_t launch_newton(const DNet &n, int64_t n_mat, const double *jvals, const double *c,
                         double *b, int trans, bool front, const WsView &W, int slots,
                         int32_t *info, hipStream_t st);
hipError_t launch_adjoint(const DNet &n, const double *la, int64_t n_cells, const AdjIO &io,
                          const BdfParams &P, const WsView &W, const AdjView &A, unsigned *queue,
                          int grid, hipStream_t st);
// out = (acc ? out : 0) + the rows in row order (chunks of rows summed one
// after another equal one pass over all rows).
hipError_t launch_sum_rows(const double *part, int64_t rows, int nr, double *out, bool acc,
                           hipStream_t st);
hipError_t launch_lu_factor(int n, int lda, int64_t nmat, double *A, int *piv, int *info,
                            hipStream_t st);
hipError_t launch_lu_solve(int n, int lda, int64_t nmat, const double *LU, const int *piv,
                           double *b, int trans, hipStream_t st);

}  // namespace ac
