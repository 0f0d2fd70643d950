/* Oracle for the stoichiometry-matrix chemistry path -- TEST INFRASTRUCTURE.
 *
 * A plain, slow, obviously correct FP64 CPU implementation of what the GPU
 * library computes. Only the test-suite, the smoke check and the benchmark's
 * CPU-baseline leg may load it. It shares no code, header, table or helper
 * with the GPU library.
 *
 * Every array is row-major, cell-major for per-cell data ([n_cells][...]).
 * Reactant and product slots hold species indices or -1 for "empty"; a
 * repeated reactant (A + A) is listed twice.
 */
#ifndef ASTROCHEM_ORACLE_H
#define ASTROCHEM_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
  int n_species;
  int n_reactions;
  const int *reactants;   /* [n_reactions][2] */
  const int *products;    /* [n_reactions][4] */
  const double *alpha;    /* [n_reactions] */
  const double *beta;     /* [n_reactions] */
  const double *gamma;    /* [n_reactions] */
  const signed char *law; /* [n_reactions] ORC_LAW_*, or NULL: every reaction ORC_LAW_KOOIJ */
  int n_cond;             /* doubles of per-cell conditions: 1 (T) or ORC_NCOND (T, A_V,
                             zeta/zeta_0, G_0); 0 is taken as 1 */
  const double *heat;     /* [n_reactions] energy released per reaction event [erg] for the
                             temperature-coupled mode, or NULL (no chemical heating) */
} orc_net;

/* Rate laws (the coefficients depend on the temperature, the cosmic-ray
 * ionisation rate and the FUV intensity, Sec. 3). Per-cell conditions
 * cond[c] = (T [K], A_V [mag], zeta/zeta_0, G_0):
 *   KOOIJ   k = alpha (T/300)^beta exp(-gamma/T)
 *   CRP     k = alpha zeta/zeta_0                       (direct cosmic-ray ionisation)
 *   CRPHOT  k = alpha (T/300)^beta gamma zeta/zeta_0 / (1 - omega), omega = 0.6
 *                                                       (cosmic-ray induced photons)
 *   PHOTO   k = alpha G_0 exp(-gamma A_V)               (interstellar FUV field) */
enum { ORC_LAW_KOOIJ = 0, ORC_LAW_CRP = 1, ORC_LAW_CRPHOT = 2, ORC_LAW_PHOTO = 3 };
#define ORC_NCOND 4
#define ORC_GRAIN_ALBEDO 0.6

/* Threads used by the per-cell loops (cells are independent). */
void orc_set_threads(int n);
int  orc_get_threads(void);

/* Dense stoichiometry matrix S[i][j] = (#i among products) - (#i among
 * reactants) of reaction j (the matrix form of the rate equations, Sec. 2.1). */
void orc_stoich(const orc_net *net, int *S);

/* k[c][j] by the reaction's rate law at the cell's conditions. Every "T"
 * argument below is the per-cell conditions array, n_cond doubles per cell
 * (just T for an all-KOOIJ network). */
void orc_rate_coeffs(const orc_net *net, long n_cells, const double *T, double *k);

/* r[c][j] = k_j * product of the reactant densities. */
void orc_rates(const orc_net *net, long n_cells, const double *y, const double *T, double *r);

/* dydt = S r, accumulated reaction by reaction: the rate is subtracted from
 * every reactant and added to every product. absterm (may be NULL) collects
 * the sum of |terms| per species, the scale of the rounding error. */
void orc_rhs(const orc_net *net, long n_cells, const double *y, const double *T,
             double *dydt, double *absterm);
void orc_rhs_k(const orc_net *net, long n_cells, const double *k, const double *y,
               double *dydt, double *absterm);

/* Dense Jacobian J[c][i][a] = d(dydt_i)/d(y_a) and the |term| sums absJ
 * (may be NULL). */
void orc_jac_dense(const orc_net *net, long n_cells, const double *y, const double *T,
                   double *J, double *absJ);

/* The Jacobian's values on a given CSR pattern (row_ptr[n_species+1],
 * col[nnz] ascending per row): jvals[c][e] = J_{row(e), col[e]} as
 * S dR/dn with the net stoichiometry (orc_jac_dense uses the gross
 * bookkeeping; the two agree up to rounding). Returns 1 if a nonzero term
 * falls outside the pattern, else 0. */
int orc_jac_pattern(const orc_net *net, long n_cells, const double *y, const double *T,
                    const int *row_ptr, const int *col, double *jvals);

/* Vector-Jacobian products for cotangent v[c][i]:
 *   gy[c][a]     = sum_i v_i J_ia                        (may be NULL)
 *   glog[c][j]   = sum_i v_i d(dydt_i)/d(log alpha_j) = r_j (S^T v)_j
 *                                                          (may be NULL) */
void orc_vjp(const orc_net *net, long n_cells, const double *y, const double *T,
             const double *v, double *gy, double *glog);

/* LU with partial pivoting, in place on a row-major n x n matrix:
 * P A = L U with unit lower L. piv[k] is the row swapped with row k at
 * step k. Returns 0, or k+1 if the k-th pivot is exactly zero. */
int  orc_lu_factor(int n, double *A, int *piv);
void orc_lu_solve(int n, const double *LU, const int *piv, double *b);    /* A x = b   */
void orc_lu_solve_t(int n, const double *LU, const int *piv, double *b);  /* A^T x = b */

/* ---------------------------------------------------------------- BDF */

/* Cell outcomes. When the step size falls below h_min the code names why
 * the last attempt was rejected: the error test (HMIN), a Newton iteration
 * that did not converge on finite values (NEWTON_FAIL), an exactly
 * singular Newton matrix (SINGULAR) or a non-finite RHS (NONFINITE). */
enum { ORC_OK = 0, ORC_MAXSTEPS = 1, ORC_HMIN = 2, ORC_BADINPUT = 3, ORC_NEWTON_FAIL = 5,
       ORC_SINGULAR = 6, ORC_NONFINITE = 7 };
enum { ORC_EV_INIT = 1, ORC_EV_RESCALE = 2, ORC_EV_STEP = 3 };

typedef struct {
  double rtol, atol;
  double h0;        /* first step; <= 0 selects it automatically */
  int q_max;        /* 1..5; 1 is adaptive backward Euler */
  int max_steps;
  double newton_tol; /* corrector tolerance (weighted RMS); <= 0: max(10 eps/rtol, min(0.03, sqrt(rtol))) */
} orc_bdf_opts;

typedef struct {
  int type;         /* ORC_EV_* */
  int q;            /* order the event applies to */
  double val;       /* INIT: h0; RESCALE: factor; STEP: h */
} orc_event;

/* Per-cell counters written to stats[c][ORC_NSTAT]. */
enum { ORC_ST_STEPS = 0, ORC_ST_REJECT_ERR, ORC_ST_REJECT_NEWTON, ORC_ST_NEWTON_IT,
       ORC_ST_JAC, ORC_ST_LU, ORC_ST_RHS, ORC_ST_QLAST, ORC_NSTAT };

/* Integrates dy/dt = S r(y) from t = 0 to t_end for every cell, with the
 * rate coefficients held at the cell's temperature. y is overwritten.
 * status[c] gets ORC_*; stats (may be NULL) gets counters; tape (may be
 * NULL) records the step sequence, up to tape_cap events per cell, with the
 * count (or -1 on overflow) in tape_len[c]. */
void orc_bdf(const orc_net *net, const orc_bdf_opts *opt, long n_cells, double *y,
             const double *T, double t_end, int *status, int *stats,
             orc_event *tape, int tape_cap, int *tape_len);

/* Temperature as a state variable (codes that solve temperature and
 * abundances together, Sec. 5): per cell the state is (n_1..n_ns, T),
 * [n_cells][n_species + 1], the coefficients follow the state's T (cond[0]
 * is ignored, the other conditions are used), and
 *   dT/dt = (sum_j heat_j R_j) / c_v - lambda (T - T_b),
 * therm[c] = (c_v [erg cm^-3 K^-1], T_b [K], lambda [1/s]).
 * orc_jac_thermal writes the dense (ns+1) x (ns+1) Jacobian per cell;
 * orc_bdf_thermal integrates the coupled system with the BDF above. */
void orc_rhs_thermal(const orc_net *net, long n_cells, const double *y, const double *cond,
                     const double *therm, double *dydt, double *absterm);
void orc_jac_thermal(const orc_net *net, long n_cells, const double *y, const double *cond,
                     const double *therm, double *J);
void orc_bdf_thermal(const orc_net *net, const orc_bdf_opts *opt, long n_cells, double *y,
                     const double *cond, const double *therm, double t_end, int *status,
                     int *stats);

/* Replays a recorded step sequence with the corrector solved to convergence
 * and propagates n_dir forward sensitivities. Direction d perturbs the
 * initial state by dy0[c][d][:] (NULL: zero) and log alpha by
 * dlogalpha[d][:] (NULL: zero). Outputs y_out[c][:] and s_out[c][d][:]. */
void orc_bdf_replay(const orc_net *net, const orc_bdf_opts *opt, long n_cells,
                    const double *y0, const double *T,
                    const orc_event *tape, int tape_cap, const int *tape_len,
                    int n_dir, const double *dy0, const double *dlogalpha,
                    double *y_out, double *s_out);

#ifdef __cplusplus
}
#endif
#endif
