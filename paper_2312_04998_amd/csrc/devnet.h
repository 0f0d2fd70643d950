// Device views of a network, passed by value to kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "../../include/astrochem.h"

namespace ac {

constexpr int LAYOUT_CSR = 0, LAYOUT_SELL = 1, LAYOUT_COO = 2, LAYOUT_RUNS = 3, LAYOUT_CCS = 4;
constexpr int RUN_ITEMS = 32;   // items per run of the equal-run partition

struct DSched {
  int n_seg, n_chunk, n_item, n_slot, n_multi;
  const int32_t *seg_out, *seg_chunk, *chunk_ptr, *chunk_dst, *multi_out, *multi_slot;
  const uint32_t *items;
  int sell_c, n_slice;
  const int32_t *slice_ptr, *sell_chunk, *sell_len, *sell_dst;
  const uint32_t *sell_items;
  const int32_t *coo_out;
  int n_run, n_rslot;
  const uint4 *run_items;      // interleaved per 64-run block (see runsum_partials)
  const uint32_t *run_mask;
  const int32_t *run_slot, *seg_run;
};

// Plan of the integrator's Newton solve: sparse front swept in levels, dense
// Schur tail (frontlu.h). n = 0: no plan.
struct DFront {
  int n, n1, n2, lda2, vofs, nv, n_lev;
  const int32_t *perm, *lev_ptr, *row_ptr, *col, *rsplit, *vdiag, *cptr, *crow, *cidx, *csplit;
  const int32_t *asm_dst, *tg_ptr, *tgt, *op_ptr;
  const int2 *ops;
  const int32_t *gseg;   // [4 (n + 1)] pieces of each output of the solves' four gathers
  const int2 *gpc;       // entry range of every piece
  int gbase[5];          // first piece of each gather
  // temperature-coupled plan only: destinations of the T column, T row, corner
  const int32_t *tcol_dst, *trow_dst;
  int corner_dst;
};

struct DNet {
  int ns, nr, nnz_j, layout, block;
  int n_cond;                  // doubles of per-cell conditions: 1 (T) or AC_NCOND
  const double *log_alpha, *beta, *gamma;
  const uint32_t *rpair;       // reactant a | b << 16 (0xFFFF none)
  const uint4 *rxpack;         // planes of nr words: (la, beta) | (gamma, rpair) | S column
  const int32_t *s_col_ptr, *s_row, *s_cval;   // CCS of S
  DSched rhs, jac, gy, jtail;
  const uint32_t *jhead0, *jhead1, *jtaildesc;
  const int32_t *jent_row, *jent_col;   // row and column of every pattern entry
  const double *heat;          // [nr] energy per reaction event (temperature-coupled mode) or null
  DFront fr;                   // Newton-solve plan of the species state
  DFront fr_th;                // and of the temperature-coupled state (species + T)
};

// Launchers (kernels_chem.hip). All enqueue on `stream`; return hipError_t.
hipError_t launch_rates(const DNet &n, const double *log_alpha, int64_t n_cells, const double *T,
                        double *k, hipStream_t stream);
hipError_t launch_rhs(const DNet &n, const double *log_alpha, int64_t n_cells, const double *y,
                      const double *T, const double *k, double *dydt, hipStream_t stream);
hipError_t launch_jac(const DNet &n, const double *log_alpha, int64_t n_cells, const double *y,
                      const double *T, double *jvals, hipStream_t stream);
hipError_t launch_rhs_jac(const DNet &n, const double *log_alpha, int64_t n_cells, const double *y,
                          const double *T, double *dydt, double *jvals, hipStream_t stream);
hipError_t launch_vjp(const DNet &n, const double *log_alpha, int64_t n_cells, const double *y,
                      const double *T, const double *v, double *gy, double *g_logalpha,
                      double *part, int part_rows, hipStream_t stream);
size_t rhs_lds_bytes(const DNet &n);

// Temperature-coupled mode (kernels_thermal.hip): state [n_cells][ns + 1],
// therm [n_cells][3] = (c_v, T_b, lambda); the Jacobian's values per cell
// are the pattern values, the T column, the T row and the corner.
hipError_t launch_rhs_thermal(const DNet &n, const double *la, int64_t n_cells, const double *y,
                              const double *cond, const double *therm, double *dydt,
                              hipStream_t stream);
hipError_t launch_jac_thermal(const DNet &n, const double *la, int64_t n_cells, const double *y,
                              const double *cond, const double *therm, double *jvals,
                              hipStream_t stream);

// Allocation-free VJP: partial-sum rows held in a device array of the
// library (static_scratch.hip), VJP_STATIC_ROWS rows of at most
// VJP_STATIC_NR reactions. *ptr gets this device's copy (looked up on the
// first call on each device).
constexpr int VJP_STATIC_ROWS = 512;
constexpr int VJP_STATIC_NR = 8192;
hipError_t vjp_static_scratch(double **ptr);

}  // namespace ac
