/* astrochem: stoichiometry-matrix chemistry on MI355X (gfx950).
 *
 * C ABI of libastrochem.so. For many independent cells that share one
 * reaction network it evaluates the chemical time derivative
 *
 *     dn/dt = S R(n, T),   R_j = k_j(T) * prod_{a in reactants(j)} n_a,
 *     k_j(T) = alpha_j (T/300)^beta_j exp(-gamma_j / T),
 *
 * where S is the integer stoichiometry matrix (species x reactions; entry
 * (i, j) is how much species i changes in reaction j -- the matrix form of
 * Motoyama et al., Sec. 2.1, eq. matrix-form), its Jacobian S dR/dn,
 * vector-Jacobian products, a batched stiff BDF integrator and its discrete
 * adjoint.
 *
 * Conventions shared by every entry point:
 *  - Per-cell arrays are DEVICE pointers owned by the caller, laid out cell
 *    by cell ([n_cells][n_species], each cell contiguous, species in the
 *    natural order of the network description). Orderings chosen at network
 *    creation only change the traversal inside the kernels.
 *  - The argument named T is the per-cell conditions array: [n_cells]
 *    temperatures [K] for a network whose reactions all follow the modified
 *    Arrhenius law (rate_law NULL at creation), else [n_cells][AC_NCOND]
 *    rows (T [K], A_V [mag], zeta/zeta_0, G_0), see ac_rate_law.
 *  - Work is enqueued on `stream` (a hipStream_t; NULL is the null stream)
 *    and the call returns without synchronising. Argument errors are found
 *    on the host before anything is enqueued.
 *  - Every call returns an ac_status. No exception or abort crosses the ABI.
 *    ac_last_error() gives a message for the last failure on the calling
 *    thread.
 *  - Network handles are immutable after creation and may be shared by
 *    threads; calls that use a network's internal reduction buffer
 *    (ac_vjp with g_logalpha) must not overlap on one network.
 *  - All arithmetic is IEEE FP64 with denormals kept.
 */
#ifndef ASTROCHEM_H
#define ASTROCHEM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef void *ac_stream; /* a hipStream_t */

typedef enum {
  AC_OK = 0,
  AC_EINVAL = 1,        /* bad argument (null pointer, size, index out of range, option) */
  AC_ENOMEM = 2,        /* host or device allocation failed */
  AC_EHIP = 3,          /* a HIP runtime call failed */
  AC_EUNBALANCED = 4,   /* a reaction does not conserve elements/charge (check requested) */
  AC_ECAPACITY = 5,     /* more cells than the workspace was created for */
  AC_ELIMIT = 6         /* network exceeds a compiled limit (see AC_MAX_*) */
} ac_status;

/* Per-cell outcome of the integrator. */
typedef enum {
  AC_CELL_OK = 0,
  AC_CELL_MAXSTEPS = 1,   /* step budget exhausted before t_end */
  AC_CELL_HMIN = 2,       /* step size fell below 10 ulp(t) after error-test rejections */
  AC_CELL_BADINPUT = 3,   /* T <= 0 or not finite, or an initial density < 0 or not finite */
  AC_CELL_TAPE = 4,       /* adjoint: the cell's tape overflowed or is malformed */
  AC_CELL_NEWTON_FAIL = 5,/* step size fell below 10 ulp(t): the corrector iteration kept
                             failing to converge (on finite values) */
  AC_CELL_SINGULAR = 6,   /* ... the last Newton matrix had an exactly zero pivot */
  AC_CELL_NONFINITE = 7   /* ... the RHS kept producing non-finite values */
} ac_cell_status;

/* Storage of S used by the RHS kernel (Sec. 2.2 compares COO, CCS, CRS and
 * SELL on CPUs). Rows are split into chunks of at most `chunk` nonzeros so
 * that heavy species rows are shared by many lanes. */
typedef enum {
  AC_LAYOUT_CSR = 0,   /* row chunks with contiguous nonzeros (CRS) */
  AC_LAYOUT_SELL = 1,  /* sliced ELLPACK over row chunks: slices of sell_c chunks,
                          nonzero k of every chunk of a slice stored together, chunks
                          sorted by length within windows of sell_sigma (SELL-C-sigma) */
  AC_LAYOUT_COO = 2,   /* coordinate triplets, scattered with LDS atomics
                          (summation order not reproducible run to run) */
  AC_LAYOUT_RUNS = 3,  /* CRS nonzeros cut into equal runs of 32 per lane
                          whatever the row lengths (merge-style partition); a
                          32-bit mask per run marks row starts, each row adds
                          its run partials in order */
  AC_LAYOUT_CCS = 4    /* column by column: each reaction scatters S_ij R_j
                          into its species with LDS atomics (order not
                          reproducible run to run) */
} ac_layout;

/* Order in which species rows are traversed (Sec. 3 reorders rows by their
 * number of nonzeros). */
typedef enum {
  AC_ORDER_NATURAL = 0,
  AC_ORDER_NNZ_DESC = 1,  /* most nonzeros first, ties in natural order */
  AC_ORDER_RCM = 2        /* reverse Cuthill-McKee on the species graph of S S^T */
} ac_ordering;

/* Rate laws. The coefficients depend on local conditions: temperature,
 * cosmic-ray ionisation rate and FUV intensity (Sec. 3). With per-cell
 * conditions (T, A_V, zeta/zeta_0, G_0):
 *   AC_LAW_KOOIJ   k = alpha (T/300)^beta exp(-gamma/T)         (modified Arrhenius)
 *   AC_LAW_CRP     k = alpha zeta/zeta_0                        (direct cosmic-ray ionisation;
 *                                                                beta, gamma unused)
 *   AC_LAW_CRPHOT  k = alpha (T/300)^beta gamma zeta/zeta_0 / (1 - AC_GRAIN_ALBEDO)
 *                                                               (cosmic-ray induced photons;
 *                                                                gamma: efficiency, > 0)
 *   AC_LAW_PHOTO   k = alpha G_0 exp(-gamma A_V)                (interstellar FUV; beta unused)
 * Every law is linear in alpha, so d k / d ln alpha = k for all of them. */
typedef enum { AC_LAW_KOOIJ = 0, AC_LAW_CRP = 1, AC_LAW_CRPHOT = 2, AC_LAW_PHOTO = 3 } ac_rate_law;
#define AC_NCOND 4
#define AC_GRAIN_ALBEDO 0.6

#define AC_MAX_SPECIES 2047
#define AC_MAX_REACTIONS 65536
#define AC_MAX_REACTANTS 2
#define AC_MAX_PRODUCTS 4

typedef struct {
  int32_t n_species;
  int32_t n_reactions;
  const int32_t *reactants;  /* host [n_reactions][2]: species index or -1; A + A listed twice;
                                at least one reactant per reaction */
  const int32_t *products;   /* host [n_reactions][4]: species index or -1 */
  const double *alpha;       /* host [n_reactions], > 0 */
  const double *beta;        /* host [n_reactions] */
  const double *gamma;       /* host [n_reactions] */
  const int8_t *composition; /* host [n_species][n_elem] element/charge counts, or NULL */
  int32_t n_elem;
  int32_t check_balance;     /* nonzero: fail with AC_EUNBALANCED unless E S = 0 exactly */
  int32_t layout;            /* ac_layout */
  int32_t ordering;          /* ac_ordering */
  int32_t chunk;             /* max nonzeros per row chunk; 0 = default (32) */
  int32_t sell_c;            /* SELL slice width in chunks: 0 or 64 (one wavefront) */
  int32_t sell_sigma;        /* SELL sorting window in chunks; 0 = default (whole matrix) */
  int32_t block;             /* threads per workgroup of the one-cell chemistry kernels:
                                256, 512 or 1024; 0 = per kernel, 1024 when its LDS
                                leaves room for one workgroup per CU, else 512 (the
                                two-cells-per-pass kernels always run 1024) */
  const int8_t *rate_law;    /* host [n_reactions] ac_rate_law codes, or NULL (every reaction
                                AC_LAW_KOOIJ, per-cell conditions = T only) */
  const double *heat;        /* host [n_reactions] energy released per reaction event [erg]
                                (exothermic > 0) for the temperature-coupled calls, or NULL
                                (no chemical heating) */
} ac_net_desc;

typedef struct ac_net ac_net;

/* Builds a network (Sec. 2.1: S from the reactant/product lists, net
 * entries only, so a catalyst A in A + B -> A + C has S = 0 but still enters
 * R and the Jacobian) together with its row storage, traversal order, the
 * symbolic pattern of the Jacobian and the per-entry contribution lists, and
 * uploads them to the current device. All arrays are copied. Without a
 * visible device the handle is host-only: the queries below work and every
 * kernel entry point returns AC_EHIP. */
ac_status ac_net_create(const ac_net_desc *desc, ac_net **out);
ac_status ac_net_destroy(ac_net *net);

/* Sizes: nonzeros of S, nonzeros of the Jacobian pattern, Jacobian
 * contribution terms, row chunks of the RHS storage. Any pointer may be NULL. */
ac_status ac_net_info(const ac_net *net, int64_t *nnz_s, int64_t *nnz_j, int64_t *n_contrib,
                      int64_t *n_chunks);

/* Host copies of S in CSR (natural species rows, reactions ascending) and of
 * the Jacobian pattern (CSR, natural rows, columns ascending). Output arrays
 * are caller-owned host memory of the sizes ac_net_info reports. */
ac_status ac_net_stoich(const ac_net *net, int32_t *row_ptr /*n_species+1*/,
                        int32_t *reaction /*nnz_s*/, int32_t *value /*nnz_s*/);
ac_status ac_net_jac_pattern(const ac_net *net, int32_t *row_ptr /*n_species+1*/,
                             int32_t *col /*nnz_j*/);
/* Traversal order of species rows (perm[k] = species visited k-th). */
ac_status ac_net_row_order(const ac_net *net, int32_t *perm /*n_species*/);
/* Plan of the integrator's Newton solve (AC_LINSOLVE_AUTO, built with the
 * network from the Jacobian pattern): the number of front species swept
 * sparsely, the sweep levels, the stored sparse values and sweep updates per
 * factorisation, the order of the species (order[p] = species at position
 * p, the front first, then the densely factored tail), and the modelled
 * cost of a factorisation and its solves relative to one dense LU of the
 * whole matrix (< 1 means the plan is expected to be faster). The front is
 * chosen by the minimum-degree order of the pattern, as in the sparse solve
 * of DLSODES (Sec. 3). n_front = 0: the front would not repay its fixed
 * latency (small networks), and AUTO factors the whole matrix densely. Any
 * output may be NULL. */
ac_status ac_net_front_info(const ac_net *net, int32_t *n_front, int32_t *n_levels,
                            int64_t *n_values, int64_t *n_updates, double *cost_ratio,
                            int32_t *order /*n_species*/);

/* Host-side storage builder for any small integer matrix given densely
 * (row-major n_rows x n_cols), exposing the formats of Sec. 2.2 with
 * 0-based indices:
 *   AC_FMT_COO: val, idx = column, idx2 = row, in row-major order
 *   AC_FMT_CCS: val, idx = row, ptr = column pointers (n_cols+1)
 *   AC_FMT_CRS: val, idx = column, ptr = row pointers (n_rows+1)
 *   AC_FMT_SELL: slices of `width` rows (no splitting, no sorting); inside a
 *     slice nonzero k of every row is stored before nonzero k+1; short rows
 *     are padded with value 0 and a valid column; ptr = slice lengths
 *     (n_slices), idx = column.
 * *n_val is the capacity of val/idx/idx2 on entry and the count on return
 * (AC_EINVAL if too small). */
enum { AC_FMT_COO = 0, AC_FMT_CCS = 1, AC_FMT_CRS = 2, AC_FMT_SELL = 3 };
ac_status ac_sparse_format(int32_t n_rows, int32_t n_cols, const int32_t *dense, int32_t fmt,
                           int32_t width, int64_t *n_val, int32_t *val, int32_t *idx,
                           int32_t *idx2, int32_t *ptr);

/* ---------------------------------------------------------------- kernels
 * log_alpha: optional DEVICE [n_reactions] override of ln(alpha) (for
 * differentiation); NULL uses the network's own coefficients. */

/* k[c][j] = the coefficient of reaction j by its rate law at cell c's
 * conditions (alpha_j (T_c/300)^beta_j exp(-gamma_j/T_c) for the default
 * law), the coefficients the paper precomputes outside the stiff solver
 * (Sec. 3). k: [n_cells][n_reactions]. */
ac_status ac_rates(const ac_net *net, const double *log_alpha, int64_t n_cells, const double *T,
                   double *k, ac_stream stream);

/* dydt = S R(y, T) per cell (eq. matrix-form), coefficients computed on the
 * fly. y, dydt: [n_cells][n_species]; T: [n_cells]. */
ac_status ac_rhs(const ac_net *net, const double *log_alpha, int64_t n_cells, const double *y,
                 const double *T, double *dydt, ac_stream stream);

/* Same with precomputed coefficients k [n_cells][n_reactions]. */
ac_status ac_rhs_k(const ac_net *net, int64_t n_cells, const double *k, const double *y,
                   double *dydt, ac_stream stream);

/* Jacobian values on the fixed pattern (ac_net_jac_pattern):
 * jvals[c][e] = d(dydt_i)/d(y_a) for pattern entry e = (i, a).
 * jvals: [n_cells][nnz_j]. */
ac_status ac_jac(const ac_net *net, const double *log_alpha, int64_t n_cells, const double *y,
                 const double *T, double *jvals, ac_stream stream);

/* ac_rhs and ac_jac in one call (eq. matrix-form and its Jacobian, Sec.
 * 2.1): dydt [n_cells][n_species] and jvals [n_cells][nnz_j], DEVICE,
 * written; bit-identical to the two calls. With the SELL layout
 * one kernel computes the coefficients once per cell for both (the
 * Newton step needs both at the same state); otherwise it issues the two
 * launches. Errors as ac_rhs / ac_jac. */
ac_status ac_rhs_jac(const ac_net *net, const double *log_alpha, int64_t n_cells, const double *y,
                     const double *T, double *dydt, double *jvals, ac_stream stream);

/* Vector-Jacobian products for cotangents v [n_cells][n_species]:
 *   gy[c][a] = sum_i v[c][i] J_ia                            (gy may be NULL)
 *   g_logalpha[j] = sum_c sum_i v[c][i] d(dydt_i)/d(ln alpha_j)
 *                 = sum_c R_cj (S^T v_c)_j                     (may be NULL)
 * The cell sum is formed in a fixed order (reproducible bit for bit). */
ac_status ac_vjp(const ac_net *net, const double *log_alpha, int64_t n_cells, const double *y,
                 const double *T, const double *v, double *gy, double *g_logalpha,
                 ac_stream stream);

/* ac_vjp for callers that cannot allocate device memory: code recorded
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc. Same arguments and results as ac_vjp (bit for bit: same
 * kernels, same fixed grid), but the per-workgroup partial sums of
 * g_logalpha live in a scratch array the library holds on each GPU for the
 * life of the process (512 rows of at most 8192 reactions, 32 MiB), not in
 * the network's buffer. The call allocates nothing. Every call on one GPU
 * shares that GPU's array: calls that overlap on one GPU (on different
 * streams or threads) race and must be serialised by the caller.
 * AC_ELIMIT when g_logalpha is requested for a network of more than 8192
 * reactions. */
ac_status ac_vjp_static(const ac_net *net, const double *log_alpha, int64_t n_cells,
                        const double *y, const double *T, const double *v, double *gy,
                        double *g_logalpha, ac_stream stream);

/* ------------------------------------------- temperature as a state
 * Codes that solve temperature and abundances together within the stiff
 * solver (Sec. 5) make T part of the state. Per cell the state is
 * (n_1..n_ns, T): y and dydt are [n_cells][n_species + 1]; the rate
 * coefficients follow the state's T (the T column of the conditions array
 * is not read; A_V, zeta and G_0 are) and
 *     dT/dt = (sum_j heat_j R_j) / c_v - lambda (T - T_b)
 * with therm [n_cells][3] = (c_v [erg cm^-3 K^-1] > 0, T_b [K] > 0,
 * lambda [1/s] >= 0) per cell and heat_j from the network description.
 * ac_jac_thermal writes per cell nnz_j + 2 n_species + 1 values: the
 * pattern values (as ac_jac, at the state's T), the T column
 * d(dn_i/dt)/dT = sum_j S_ij R_j d ln k_j/dT, the T row
 * d(dT/dt)/dn_a = sum_j heat_j dR_j/dn_a / c_v, and the corner
 * d(dT/dt)/dT. All pointers DEVICE; errors as ac_rhs. */
ac_status ac_rhs_thermal(const ac_net *net, const double *log_alpha, int64_t n_cells,
                         const double *y, const double *T, const double *therm, double *dydt,
                         ac_stream stream);
ac_status ac_jac_thermal(const ac_net *net, const double *log_alpha, int64_t n_cells,
                         const double *y, const double *T, const double *therm, double *jvals,
                         ac_stream stream);

/* ------------------------------------------------ batched dense LU
 * The Newton matrices of the implicit integrator are dense n x n (n =
 * species), one per cell. A: [n_mat][n][lda] row-major DEVICE array,
 * factored in place as P A = L U with unit lower L (partial pivoting, whole
 * rows swapped, piv[k] = row exchanged with row k at step k); info[m] = 0 or
 * 1 + index of the first exactly-zero pivot (info may be NULL). lda >= n;
 * n <= 1024 (AC_ELIMIT otherwise: a panel column lives in one workgroup's
 * registers, two rows per thread). Errors: AC_EINVAL for bad sizes or NULL
 * arrays with n_mat > 0, AC_EHIP for a failed launch. */
ac_status ac_lu_factor(int32_t n, int32_t lda, int64_t n_mat, double *A, int32_t *piv,
                       int32_t *info, ac_stream stream);
/* Solves A x = b (trans = 0) or A^T x = b (trans = 1) in place in b
 * [n_mat][n] with the factors of ac_lu_factor. */
ac_status ac_lu_solve(int32_t n, int32_t lda, int64_t n_mat, const double *LU,
                      const int32_t *piv, double *b, int32_t trans, ac_stream stream);

/* ---------------------------------------------------------- integrator
 * Variable-order (1..q_max <= 5) BDF in backward-difference form with a
 * simplified Newton corrector on the matrix I - c J, factored as chosen by
 * ac_integ_opts.linear_solver (see ac_linear_solver) (the paper
 * integrates every cell with the BDF code DLSODES, Sec. 3, and keeps T fixed
 * during the chemistry update, Sec. 5). Rules, identical in the CPU oracle:
 * error test on RMS(d / (atol + rtol |y|)) / (q+1) <= 1; step factor
 * 0.9*9/(8+iters) * err^(-1/(q+1)) clamped to [0.2, 10]; order change to
 * the best of q-1, q, q+1 after q+1 equal steps; at most 4 Newton
 * iterations with a rate test; J refreshed once per attempt on Newton
 * failure, then h halved; M = I - c_M J kept while |c/c_M - 1| <= 0.3 and
 * refactored beyond that or after a refresh of J, Newton corrections scaled
 * by 2/(1 + c/c_M) in between (the LSODE-family matrix-reuse rule). */
typedef struct {
  double rtol;        /* > 0 */
  double atol;        /* >= 0, in units of y */
  double h0;          /* first step [s]; <= 0 selects it (Hairer-Norsett-Wanner) */
  int32_t q_max;      /* 1..5; 1 is adaptive backward Euler */
  int32_t max_steps;  /* accepted-step budget per cell */
  int32_t adj_recompute; /* adjoint only: 1 recomputes every segment from its
                            checkpoint; 0 keeps every converged state of the
                            forward replay instead when the workspace reserved
                            room for them (see ac_ws_reserve_adjoint) */
  int32_t checkpoint_every; /* adjoint and replay: accepted steps between
                            checkpoints; 0 = 64; must equal the interval the
                            workspace reserved for */
  double newton_tol;     /* corrector convergence tolerance in the weighted RMS
                            norm; <= 0 selects max(10 eps/rtol, min(0.03, sqrt(rtol))) */
  const int32_t *cell_order; /* ac_integrate and ac_integrate_thermal: DEVICE
                            [n_cells], the order in which the persistent
                            workgroups take the cells (a permutation of
                            0..n_cells-1; cells expected to take longest first
                            shorten the run's tail), or NULL for index order.
                            Each cell's results do not depend on it. Not
                            checked: a repeated index integrates that cell
                            twice, concurrently. */
  int32_t linear_solver; /* ac_linear_solver: how the Newton matrix is factored */
} ac_integ_opts;

/* Newton solves of the integrator and the adjoint. DLSODES, the integrator
 * of the paper (Sec. 3), factors the sparse Newton matrix under a
 * minimum-degree order without pivoting. AUTO does that for the species the
 * order eliminates first (a Gauss-Jordan sweep of that sparse front, in
 * levels of independent pivots, chosen by structure at network build) and
 * factors the Schur complement left over by the remaining, densely coupled
 * species with partial pivoting on the matrix cores. DENSE factors the whole
 * matrix with partial pivoting. The temperature-coupled mode has its own
 * plan, over the species and T: its full temperature row and column end in
 * the dense tail. */
typedef enum { AC_LINSOLVE_AUTO = 0, AC_LINSOLVE_DENSE = 1 } ac_linear_solver;

/* Per-cell counters written by the integrator ([n_cells][AC_NSTAT]). */
enum { AC_STAT_STEPS = 0, AC_STAT_REJECT_ERR, AC_STAT_REJECT_NEWTON, AC_STAT_NEWTON_ITERS,
       AC_STAT_JAC, AC_STAT_LU, AC_STAT_RHS, AC_STAT_Q_LAST, AC_NSTAT };

/* Step-sequence record for replay and the adjoint: INIT (val = first step),
 * RESCALE (difference array resampled for order q by factor val), STEP
 * (accepted step of order q and size val). */
typedef struct {
  int32_t type;       /* 1 INIT, 2 RESCALE, 3 STEP */
  int32_t q;
  double val;
} ac_event;

typedef struct ac_ws ac_ws;

/* Integrator workspace: one slot (Newton matrix, Jacobian values,
 * difference array, coefficients: about 8 n^2 + 8 nnz_j + 64 n + 8 n_r
 * bytes) per resident workgroup. n_slots = 0 uses every workgroup that
 * fits on the device at once. All integrator scratch is allocated here. */
ac_status ac_ws_create(const ac_net *net, int32_t n_slots, ac_ws **out);
ac_status ac_ws_destroy(ac_ws *ws);
ac_status ac_ws_info(const ac_ws *ws, int32_t *n_slots, int64_t *bytes);

/* Progress of a running ac_integrate or ac_integrate_thermal on this
 * workspace: *cells_taken = 1 + the index of the last cell a workgroup took
 * from the device queue (cells done or in progress; workgroups report in
 * whatever order they take cells, so the count can briefly step back by a
 * few), or the last call's final count once it ends. The integrator
 * writes it to a pinned host word of the workspace; this call only reads
 * that word, so it returns at once while the integration runs. For
 * progress reports of long integrations. */
ac_status ac_ws_progress(ac_ws *ws, int64_t *cells_taken);

/* Room for the discrete adjoint and the replay, allocated here (with a
 * device synchronisation; any earlier reservation is released) so that
 * ac_integrate_adjoint and ac_replay allocate nothing:
 *   max_tape          longest tape (events) the calls will pass (tape_cap)
 *   checkpoint_every  accepted steps between checkpoints; 0 = 64; the calls
 *                     must use the same interval
 *   keep_states       1: also room for every converged state of a max_tape
 *                     replay per slot, when that comes to at most 32 GiB over
 *                     all slots (max_tape n_species 8 bytes per slot), so the
 *                     reverse sweep reads them instead of recomputing segments
 *   max_cells         cells whose per-cell dL/dlog alpha rows the workspace
 *                     holds, so the summed gradient needs no caller buffer
 *                     (longer calls run in chunks of max_cells); 0 = none
 * Per slot: (max_tape / checkpoint_every + 1) 64 n_species bytes of
 * checkpoints, 8 n_species bytes of adjoint state and checkpoint_every (or,
 * keeping states, max_tape) 8 n_species bytes of converged states; plus
 * 8 n_reactions max_cells bytes of rows. */
typedef struct {
  int32_t max_tape;
  int32_t checkpoint_every;
  int32_t keep_states;
  int32_t max_cells;
} ac_adj_reserve;
ac_status ac_ws_reserve_adjoint(ac_ws *ws, const ac_adj_reserve *r);
/* What the workspace reserved (zeros when nothing): the longest tape, the
 * checkpoint interval, whether every state is kept, the gradient rows. */
ac_status ac_ws_adjoint_info(const ac_ws *ws, int32_t *max_tape, int32_t *checkpoint_every,
                             int32_t *keeps_states, int32_t *max_cells);

/* Integrates dy/dt = S R(y) from t = 0 to t_end for every cell, T held
 * fixed per cell. y [n_cells][n_species] DEVICE, overwritten with y(t_end)
 * (cells with AC_CELL_BADINPUT are left untouched); T [n_cells] DEVICE.
 * cell_status [n_cells] and cell_stats [n_cells][AC_NSTAT] DEVICE (either
 * may be NULL). tape [n_cells][tape_cap] and tape_len [n_cells] DEVICE
 * record the step sequence when tape is not NULL (tape_len = -1 when a
 * cell needs more than tape_cap events). Cells are handed to the
 * workspace's persistent workgroups through a device queue; one workspace
 * serves one stream at a time. */
ac_status ac_integrate(ac_ws *ws, const double *log_alpha, int64_t n_cells, double *y,
                       const double *T, double t_end, const ac_integ_opts *opts,
                       int32_t *cell_status, int32_t *cell_stats, ac_event *tape,
                       int32_t tape_cap, int32_t *tape_len, ac_stream stream);

/* The integrator with temperature as a state (see ac_rhs_thermal): y
 * [n_cells][n_species + 1] (DEVICE, in/out; initial T > 0 in the last
 * entry), conditions T and therm [n_cells][3] as there. The Newton matrix is
 * (n_species + 1)^2 with the T column and row; the coefficients are
 * recomputed at every RHS and Jacobian evaluation. Same rules, options and
 * per-cell outputs as ac_integrate (no tape: the adjoint covers the
 * fixed-temperature integrator). AC_CELL_BADINPUT also for T <= 0 or bad
 * therm values. */
ac_status ac_integrate_thermal(ac_ws *ws, const double *log_alpha, int64_t n_cells, double *y,
                               const double *T, const double *therm, double t_end,
                               const ac_integ_opts *opts, int32_t *cell_status,
                               int32_t *cell_stats, ac_stream stream);

/* The integrator's Newton systems on their own (the corrector of the BDF
 * code DLSODES, Sec. 3): for matrix m, M = I - c[m] J_m with J_m given by
 * its values on the network's Jacobian pattern, solves M x = b (trans = 0)
 * or M^T x = b (trans = 1). jvals: DEVICE [n_mat][nnz_j] (ac_jac's layout);
 * c: DEVICE [n_mat]; b: DEVICE [n_mat][n_species], overwritten by x; info:
 * DEVICE [n_mat] or NULL, 0 or 1 + the position of an exactly zero pivot
 * (x is then not finite). linear_solver as ac_integ_opts.linear_solver. The
 * workspace's slots hold the factors, one matrix per slot at a time, so
 * calls on one workspace must not overlap with each other or with an
 * integration. */
ac_status ac_newton_solve(ac_ws *ws, int64_t n_mat, const double *jvals, const double *c,
                          double *b, int32_t trans, int32_t linear_solver, int32_t *info,
                          ac_stream stream);

/* Same integrator, one cell per kernel launch, one workgroup, launches
 * issued back to back from the host: the unbatched baseline. */
ac_status ac_integrate_plain(ac_ws *ws, const double *log_alpha, int64_t n_cells, double *y,
                             const double *T, double t_end, const ac_integ_opts *opts,
                             int32_t *cell_status, int32_t *cell_stats, ac_stream stream);

/* Discrete adjoint of ac_integrate for L = sum_c <lambda_c, y_c(t_end)>.
 * The map differentiated is the recorded step sequence (tape, tape_len as
 * written by ac_integrate with the same y0, T, log_alpha and tolerances)
 * with step sizes and orders held fixed and every corrector equation
 * d - c f(y_pred + d) + psi = 0 solved to convergence, so each accepted
 * step is differentiated through the implicit function theorem: one
 * transposed solve with M = I - c J(y_{n+1}), refactored at the converged
 * state, and one vector-Jacobian product per step. The tape is replayed
 * forward once, keeping the difference array every checkpoint_every accepted
 * steps (and every converged state when the workspace has room), and the
 * reverse sweep reads the kept states or recomputes each segment from its
 * checkpoint. Not in the paper; the forward method is Sec. 3's BDF
 * integration of eq. matrix-form.
 *   y0, lambda [n_cells][n_species], T [n_cells]    DEVICE, read
 *   tape [n_cells][tape_cap], tape_len [n_cells]    DEVICE, read
 *   y_final [n_cells][n_species] DEVICE or NULL: the replayed y(t_end)
 *   dL_dy0 [n_cells][n_species] DEVICE, written
 *   g_cells [n_cells][n_reactions] DEVICE or NULL: per-cell dL/dlog alpha
 *   dL_dlogalpha [n_reactions] DEVICE or NULL: the sum over cells in cell
 *     order (bitwise reproducible), from g_cells when given, else from the
 *     workspace's rows max_cells cells at a time (same bits)
 *   cell_status [n_cells] DEVICE or NULL: AC_CELL_OK, AC_CELL_BADINPUT
 *     (dL_dy0 = lambda, no parameter terms) or AC_CELL_TAPE (tape_len < 0,
 *     > tape_cap, or an order outside 1..5; dL_dy0 = lambda).
 *   cell_stats [n_cells][AC_NSTAT] DEVICE or NULL: steps reversed, Newton
 *     iterations of the replays, Jacobians, factorisations and RHS
 *     evaluations (the rejection and order fields are 0).
 * Only rtol, atol, adj_recompute and checkpoint_every of opts are used (the
 * tolerances scale the replay's convergence test). Nothing is allocated:
 * the workspace must hold an adjoint reservation (ac_ws_reserve_adjoint)
 * with max_tape >= tape_cap and the same checkpoint interval, and gradient
 * rows when dL_dlogalpha is asked for without g_cells; otherwise
 * AC_ECAPACITY. Errors: AC_EINVAL for bad sizes or NULL required arrays,
 * AC_EHIP for launch failures. */
ac_status ac_integrate_adjoint(ac_ws *ws, const double *log_alpha, int64_t n_cells,
                               const double *y0, const double *T, const ac_integ_opts *opts,
                               const ac_event *tape, int32_t tape_cap, const int32_t *tape_len,
                               const double *lambda, double *y_final, double *dL_dy0,
                               double *g_cells, double *dL_dlogalpha, int32_t *cell_status,
                               int32_t *cell_stats, ac_stream stream);

/* The forward half of ac_integrate_adjoint alone: replays a recorded step
 * sequence (as written by ac_integrate) from y0 with every corrector
 * equation solved to convergence and writes the replayed y(t_end) to
 * y_final [n_cells][n_species] (DEVICE). Step sizes, orders and
 * resamplings come from the tape, so the result is a smooth function of y0
 * and log_alpha (what finite differences of the adjoint's map need).
 * cell_status / cell_stats as for ac_integrate_adjoint (either may be
 * NULL). Errors: AC_EINVAL for bad sizes or NULL required arrays. */
ac_status ac_replay(ac_ws *ws, const double *log_alpha, int64_t n_cells, const double *y0,
                    const double *T, const ac_integ_opts *opts, const ac_event *tape,
                    int32_t tape_cap, const int32_t *tape_len, double *y_final,
                    int32_t *cell_status, int32_t *cell_stats, ac_stream stream);

/* Status text and the calling thread's last error message (incl. HIP's). *//* Status text and the calling thread's last error message (incl. HIP's). */
const char *ac_status_string(ac_status s);
int ac_last_error(char *buf, size_t n);

#ifdef __cplusplus
}
#endif
#endif
