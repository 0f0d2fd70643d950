/* Oracle for the stoichiometry-matrix chemistry path -- TEST INFRASTRUCTURE.
 *
 * Plain FP64 loops, one cell at a time (cells are independent, so the outer
 * loop over cells may run on several threads, like the paper's domain
 * decomposition in Sec. 3). No blocking, fusion or reordering: every
 * function follows the definition it cites, so it can be checked by eye.
 *
 * Only tests, the smoke check and the benchmark's CPU-baseline leg use this
 * file. It shares nothing with the GPU library.
 */
#include "oracle.h"

#include <float.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define NRS 2   /* reactant slots per reaction */
#define NPS 4   /* product slots per reaction  */

static int g_threads = 1;
void orc_set_threads(int n) { g_threads = n > 0 ? n : 1; }
int orc_get_threads(void) { return g_threads; }

static void *xcalloc(size_t n, size_t sz) {
  void *p = calloc(n ? n : 1, sz);
  if (!p) abort();
  return p;
}

/* ------------------------------------------------------------------ S */

/* Sec. 2.1, eq. (matrix-form): alpha_ij is how much species i changes in
 * reaction j -- negative for reactants, positive for products. */
void orc_stoich(const orc_net *net, int *S) {
  const int ns = net->n_species, nr = net->n_reactions;
  memset(S, 0, sizeof(int) * (size_t)ns * (size_t)nr);
  for (int j = 0; j < nr; ++j) {
    for (int s = 0; s < NRS; ++s) {
      int a = net->reactants[j * NRS + s];
      if (a >= 0) S[(size_t)a * nr + j] -= 1;
    }
    for (int s = 0; s < NPS; ++s) {
      int p = net->products[j * NPS + s];
      if (p >= 0) S[(size_t)p * nr + j] += 1;
    }
  }
}

/* ------------------------------------------------------- rates and RHS */

static int n_cond(const orc_net *net) { return net->n_cond > 1 ? net->n_cond : 1; }

/* Rate coefficient of reaction j at a cell's conditions c = (T, A_V,
 * zeta/zeta_0, G_0), held fixed during the chemistry update (the
 * coefficients are precomputed outside the stiff solver and depend on the
 * temperature, the cosmic-ray ionisation rate and the FUV intensity, Sec.
 * 3; temperature is constant during the update, Sec. 5). The default law
 * is the modified Arrhenius (Kooij) form. */
static double rate_coeff(const orc_net *net, int j, const double *c) {
  const int law = net->law ? net->law[j] : ORC_LAW_KOOIJ;
  const double T = c[0];
  switch (law) {
    case ORC_LAW_CRP:
      return net->alpha[j] * c[2];
    case ORC_LAW_CRPHOT:
      return net->alpha[j] * pow(T / 300.0, net->beta[j]) * net->gamma[j] * c[2] /
             (1.0 - ORC_GRAIN_ALBEDO);
    case ORC_LAW_PHOTO:
      return net->alpha[j] * c[3] * exp(-net->gamma[j] * c[1]);
    default:
      return net->alpha[j] * pow(T / 300.0, net->beta[j]) * exp(-net->gamma[j] / T);
  }
}

static void cell_rate_coeffs(const orc_net *net, const double *c, double *k) {
  for (int j = 0; j < net->n_reactions; ++j) k[j] = rate_coeff(net, j, c);
}

/* R_j of eq. (matrix-form): the coefficient times the density of every
 * reactant, so 2A -> B proceeds at k n_A^2 (Sec. 2.1 example). */
static double reaction_rate(const orc_net *net, const double *k, const double *y, int j) {
  double r = k[j];
  for (int s = 0; s < NRS; ++s) {
    int a = net->reactants[j * NRS + s];
    if (a >= 0) r *= y[a];
  }
  return r;
}

/* dn/dt = S R (eq. matrix-form), taken reaction by reaction (column order,
 * the traversal of the CCS listing in Sec. 2.2): each reaction's rate is
 * subtracted from its reactants and added to its products. */
static void cell_rhs_k(const orc_net *net, const double *k, const double *y, double *dydt,
                       double *absterm) {
  const int ns = net->n_species, nr = net->n_reactions;
  for (int i = 0; i < ns; ++i) dydt[i] = 0.0;
  if (absterm)
    for (int i = 0; i < ns; ++i) absterm[i] = 0.0;
  for (int j = 0; j < nr; ++j) {
    double r = reaction_rate(net, k, y, j);
    for (int s = 0; s < NRS; ++s) {
      int a = net->reactants[j * NRS + s];
      if (a < 0) continue;
      dydt[a] -= r;
      if (absterm) absterm[a] += fabs(r);
    }
    for (int s = 0; s < NPS; ++s) {
      int p = net->products[j * NPS + s];
      if (p < 0) continue;
      dydt[p] += r;
      if (absterm) absterm[p] += fabs(r);
    }
  }
}

void orc_rate_coeffs(const orc_net *net, long n_cells, const double *T, double *k) {
  const int nr = net->n_reactions;
#pragma omp parallel for num_threads(g_threads) schedule(static)
  for (long c = 0; c < n_cells; ++c) cell_rate_coeffs(net, T + (size_t)c * n_cond(net), k + (size_t)c * nr);
}

void orc_rates(const orc_net *net, long n_cells, const double *y, const double *T, double *r) {
  const int ns = net->n_species, nr = net->n_reactions;
#pragma omp parallel num_threads(g_threads)
  {
    double *k = xcalloc((size_t)nr, sizeof(double));
#pragma omp for schedule(static)
    for (long c = 0; c < n_cells; ++c) {
      cell_rate_coeffs(net, T + (size_t)c * n_cond(net), k);
      for (int j = 0; j < nr; ++j)
        r[(size_t)c * nr + j] = reaction_rate(net, k, y + (size_t)c * ns, j);
    }
    free(k);
  }
}

void orc_rhs(const orc_net *net, long n_cells, const double *y, const double *T, double *dydt,
             double *absterm) {
  const int ns = net->n_species, nr = net->n_reactions;
#pragma omp parallel num_threads(g_threads)
  {
    double *k = xcalloc((size_t)nr, sizeof(double));
#pragma omp for schedule(static)
    for (long c = 0; c < n_cells; ++c) {
      cell_rate_coeffs(net, T + (size_t)c * n_cond(net), k);
      cell_rhs_k(net, k, y + (size_t)c * ns, dydt + (size_t)c * ns,
                 absterm ? absterm + (size_t)c * ns : NULL);
    }
    free(k);
  }
}

void orc_rhs_k(const orc_net *net, long n_cells, const double *k, const double *y, double *dydt,
               double *absterm) {
  const int ns = net->n_species, nr = net->n_reactions;
#pragma omp parallel for num_threads(g_threads) schedule(static)
  for (long c = 0; c < n_cells; ++c)
    cell_rhs_k(net, k + (size_t)c * nr, y + (size_t)c * ns, dydt + (size_t)c * ns,
               absterm ? absterm + (size_t)c * ns : NULL);
}

/* --------------------------------------------------------- Jacobian */

/* Partial derivative of R_j with respect to the reactant in slot s: the
 * coefficient times the densities of the *other* reactant slots (for
 * A + A each slot gives k n_A, together 2 k n_A). */
static double rate_slot_derivative(const orc_net *net, const double *k, const double *y, int j,
                                   int s) {
  double d = k[j];
  for (int t = 0; t < NRS; ++t) {
    if (t == s) continue;
    int b = net->reactants[j * NRS + t];
    if (b >= 0) d *= y[b];
  }
  return d;
}

/* J_ia = sum_j S_ij dR_j/dn_a, accumulated with the same reactant/product
 * bookkeeping as the RHS. */
static void cell_jac(const orc_net *net, const double *k, const double *y, double *J,
                     double *absJ) {
  const int ns = net->n_species, nr = net->n_reactions;
  memset(J, 0, sizeof(double) * (size_t)ns * ns);
  if (absJ) memset(absJ, 0, sizeof(double) * (size_t)ns * ns);
  for (int j = 0; j < nr; ++j) {
    for (int s = 0; s < NRS; ++s) {
      int a = net->reactants[j * NRS + s];
      if (a < 0) continue;
      double d = rate_slot_derivative(net, k, y, j, s);
      for (int t = 0; t < NRS; ++t) {
        int b = net->reactants[j * NRS + t];
        if (b < 0) continue;
        J[(size_t)b * ns + a] -= d;
        if (absJ) absJ[(size_t)b * ns + a] += fabs(d);
      }
      for (int t = 0; t < NPS; ++t) {
        int p = net->products[j * NPS + t];
        if (p < 0) continue;
        J[(size_t)p * ns + a] += d;
        if (absJ) absJ[(size_t)p * ns + a] += fabs(d);
      }
    }
  }
}

void orc_jac_dense(const orc_net *net, long n_cells, const double *y, const double *T, double *J,
                   double *absJ) {
  const int ns = net->n_species, nr = net->n_reactions;
  const size_t nn = (size_t)ns * ns;
#pragma omp parallel num_threads(g_threads)
  {
    double *k = xcalloc((size_t)nr, sizeof(double));
#pragma omp for schedule(static)
    for (long c = 0; c < n_cells; ++c) {
      cell_rate_coeffs(net, T + (size_t)c * n_cond(net), k);
      cell_jac(net, k, y + (size_t)c * ns, J + (size_t)c * nn, absJ ? absJ + (size_t)c * nn : NULL);
    }
    free(k);
  }
}

/* The Jacobian on a given sparsity pattern (CSR: row_ptr[ns+1], col[nnz],
 * columns ascending within a row), as the matrix product of eq.
 * (matrix-form) differentiated: J = S dR/dn with the net stoichiometry, so
 * a catalyst (in and out of the same reaction) adds nothing to its own row.
 * Reaction by reaction, every reactant slot's derivative times each net
 * entry of the reaction's column of S goes to its entry. A term outside the
 * pattern is an error (returns 1). */
static int pattern_index(const int *row_ptr, const int *col, int i, int a) {
  int lo = row_ptr[i], hi = row_ptr[i + 1];
  while (lo < hi) {
    int mid = (lo + hi) / 2;
    if (col[mid] < a) lo = mid + 1;
    else hi = mid;
  }
  return (lo < row_ptr[i + 1] && col[lo] == a) ? lo : -1;
}

/* Net column of S for reaction j: species and coefficients, zeros dropped. */
static int net_column(const orc_net *net, int j, int *sp, int *coef) {
  int m = 0;
  for (int t = 0; t < NRS + NPS; ++t) {
    int x = t < NRS ? net->reactants[j * NRS + t] : net->products[j * NPS + t - NRS];
    if (x < 0) continue;
    int q = 0;
    while (q < m && sp[q] != x) ++q;
    if (q == m) {
      sp[m] = x;
      coef[m] = 0;
      ++m;
    }
    coef[q] += t < NRS ? -1 : 1;
  }
  return m;
}

/* One term of the pattern Jacobian: reaction j's derivative in reactant
 * slot s, times coef, goes to entry e. */
typedef struct {
  int j, s, e, coef;
} pat_term;

/* The terms of S dR/dn on the pattern, reaction by reaction (the order in
 * which every entry receives them); NULL with *bad = 1 if a term falls
 * outside the pattern. */
static pat_term *pattern_terms(const orc_net *net, const int *row_ptr, const int *col, int *nt,
                               int *bad) {
  const int nr = net->n_reactions;
  pat_term *t = xcalloc((size_t)nr * NRS * (NRS + NPS), sizeof(pat_term));
  int m = 0;
  *bad = 0;
  for (int j = 0; j < nr; ++j) {
    int sp[NRS + NPS], coef[NRS + NPS];
    const int nc = net_column(net, j, sp, coef);
    for (int s = 0; s < NRS; ++s) {
      int a = net->reactants[j * NRS + s];
      if (a < 0) continue;
      for (int q = 0; q < nc; ++q) {
        if (coef[q] == 0) continue;
        int e = pattern_index(row_ptr, col, sp[q], a);
        if (e < 0) {
          *bad = 1;
          free(t);
          return NULL;
        }
        t[m].j = j;
        t[m].s = s;
        t[m].e = e;
        t[m].coef = coef[q];
        ++m;
      }
    }
  }
  *nt = m;
  return t;
}

int orc_jac_pattern(const orc_net *net, long n_cells, const double *y, const double *T,
                    const int *row_ptr, const int *col, double *jvals) {
  const int ns = net->n_species, nr = net->n_reactions;
  const size_t nnz = (size_t)row_ptr[ns];
  int nt = 0, bad = 0;
  pat_term *t = pattern_terms(net, row_ptr, col, &nt, &bad);
  if (bad) return 1;
#pragma omp parallel num_threads(g_threads)
  {
    double *k = xcalloc((size_t)nr, sizeof(double));
#pragma omp for schedule(static)
    for (long c = 0; c < n_cells; ++c) {
      const double *yc = y + (size_t)c * ns;
      double *jv = jvals + (size_t)c * nnz;
      cell_rate_coeffs(net, T + (size_t)c * n_cond(net), k);
      memset(jv, 0, sizeof(double) * nnz);
      for (int q = 0; q < nt; ++q)
        jv[t[q].e] += t[q].coef * rate_slot_derivative(net, k, yc, t[q].j, t[q].s);
    }
    free(k);
  }
  free(t);
  return 0;
}

/* ------------------------------------------- temperature as a state
 *
 * Codes that solve temperature and abundances together in the stiff
 * solver (Sec. 5) add T to the state. Here the gas heats by the energy the
 * reactions release and relaxes towards a background temperature:
 *   dT/dt = (sum_j heat_j R_j) / c_v - lambda (T - T_b),
 * heat_j [erg] per reaction event, per-cell c_v [erg cm^-3 K^-1], T_b [K]
 * and lambda [1/s] (therm[c] = (c_v, T_b, lambda)). The coefficients follow
 * the state's T, so the Jacobian gains a T column through dk/dT and a T
 * row through the heating term. */

/* d ln k_j / dT at the cell's conditions (rate laws of rate_coeff). */
static double rate_dlog_dT(const orc_net *net, int j, double T) {
  const int law = net->law ? net->law[j] : ORC_LAW_KOOIJ;
  switch (law) {
    case ORC_LAW_CRP:
    case ORC_LAW_PHOTO:
      return 0.0;
    case ORC_LAW_CRPHOT:
      return net->beta[j] / T;
    default:
      return (net->beta[j] + net->gamma[j] / T) / T;
  }
}

/* Conditions with the state's temperature in place of cond[0]. */
static void cond_at(const orc_net *net, const double *cond, double T, double *out) {
  for (int i = 0; i < n_cond(net); ++i) out[i] = cond[i];
  out[0] = T;
}

static void cell_rhs_thermal(const orc_net *net, const double *cond, const double *therm,
                             const double *y, double *k, double *f, double *absterm) {
  const int ns = net->n_species, nr = net->n_reactions;
  double c[ORC_NCOND];
  cond_at(net, cond, y[ns], c);
  cell_rate_coeffs(net, c, k);
  cell_rhs_k(net, k, y, f, absterm);
  double q = 0.0, qa = 0.0;
  if (net->heat)
    for (int j = 0; j < nr; ++j) {
      double h = net->heat[j] * reaction_rate(net, k, y, j);
      q += h;
      qa += fabs(h);
    }
  f[ns] = q / therm[0] - therm[2] * (y[ns] - therm[1]);
  if (absterm) absterm[ns] = qa / therm[0] + fabs(therm[2] * (y[ns] - therm[1]));
}

/* Dense (ns+1) x (ns+1) Jacobian of the coupled system, row-major. */
static void cell_jac_thermal(const orc_net *net, const double *cond, const double *therm,
                             const double *y, double *k, double *Jn, double *Jb) {
  const int ns = net->n_species, nr = net->n_reactions, n = ns + 1;
  const double T = y[ns];
  double c[ORC_NCOND];
  cond_at(net, cond, T, c);
  cell_rate_coeffs(net, c, k);
  cell_jac(net, k, y, Jb, NULL);
  for (int i = 0; i < ns; ++i) {
    for (int a = 0; a < ns; ++a) Jn[(size_t)i * n + a] = Jb[(size_t)i * ns + a];
    Jn[(size_t)i * n + ns] = 0.0;
  }
  for (int a = 0; a <= ns; ++a) Jn[(size_t)ns * n + a] = 0.0;
  /* T column: d(dn_i/dt)/dT = sum_j S_ij R_j dln k_j/dT, same bookkeeping */
  for (int j = 0; j < nr; ++j) {
    const double dr = reaction_rate(net, k, y, j) * rate_dlog_dT(net, j, T);
    for (int s = 0; s < NRS; ++s) {
      int a = net->reactants[j * NRS + s];
      if (a >= 0) Jn[(size_t)a * n + ns] -= dr;
    }
    for (int s = 0; s < NPS; ++s) {
      int p = net->products[j * NPS + s];
      if (p >= 0) Jn[(size_t)p * n + ns] += dr;
    }
    if (net->heat) {
      /* T row: heating through every reactant density, and through T */
      const double hj = net->heat[j] / therm[0];
      for (int s = 0; s < NRS; ++s) {
        int a = net->reactants[j * NRS + s];
        if (a >= 0) Jn[(size_t)ns * n + a] += hj * rate_slot_derivative(net, k, y, j, s);
      }
      Jn[(size_t)ns * n + ns] += hj * dr;
    }
  }
  Jn[(size_t)ns * n + ns] -= therm[2];
}

void orc_rhs_thermal(const orc_net *net, long n_cells, const double *y, const double *cond,
                     const double *therm, double *dydt, double *absterm) {
  const int n = net->n_species + 1, nr = net->n_reactions;
#pragma omp parallel num_threads(g_threads)
  {
    double *k = xcalloc((size_t)nr, sizeof(double));
#pragma omp for schedule(static)
    for (long c = 0; c < n_cells; ++c)
      cell_rhs_thermal(net, cond + (size_t)c * n_cond(net), therm + (size_t)c * 3,
                       y + (size_t)c * n, k, dydt + (size_t)c * n,
                       absterm ? absterm + (size_t)c * n : NULL);
    free(k);
  }
}

void orc_jac_thermal(const orc_net *net, long n_cells, const double *y, const double *cond,
                     const double *therm, double *J) {
  const int ns = net->n_species, n = ns + 1, nr = net->n_reactions;
#pragma omp parallel num_threads(g_threads)
  {
    double *k = xcalloc((size_t)nr, sizeof(double));
    double *Jb = xcalloc((size_t)ns * ns, sizeof(double));
#pragma omp for schedule(static)
    for (long c = 0; c < n_cells; ++c)
      cell_jac_thermal(net, cond + (size_t)c * n_cond(net), therm + (size_t)c * 3,
                       y + (size_t)c * n, k, J + (size_t)c * n * n, Jb);
    free(k);
    free(Jb);
  }
}

/* ------------------------------------------------------------- VJP */

/* (S^T v)_j: the net change of <v, n> per unit of reaction j. */
static double stoich_dot(const orc_net *net, const double *v, int j) {
  double w = 0.0;
  for (int s = 0; s < NRS; ++s) {
    int a = net->reactants[j * NRS + s];
    if (a >= 0) w -= v[a];
  }
  for (int s = 0; s < NPS; ++s) {
    int p = net->products[j * NPS + s];
    if (p >= 0) w += v[p];
  }
  return w;
}

/* gy = J^T v and d<v, dydt>/d(log alpha_j) = R_j (S^T v)_j, because
 * dR_j/d(log alpha_j) = R_j. */
static void cell_vjp(const orc_net *net, const double *k, const double *y, const double *v,
                     double *gy, double *glog) {
  const int ns = net->n_species, nr = net->n_reactions;
  if (gy)
    for (int a = 0; a < ns; ++a) gy[a] = 0.0;
  for (int j = 0; j < nr; ++j) {
    double w = stoich_dot(net, v, j);
    if (glog) glog[j] = reaction_rate(net, k, y, j) * w;
    if (!gy) continue;
    for (int s = 0; s < NRS; ++s) {
      int a = net->reactants[j * NRS + s];
      if (a >= 0) gy[a] += rate_slot_derivative(net, k, y, j, s) * w;
    }
  }
}

void orc_vjp(const orc_net *net, long n_cells, const double *y, const double *T, const double *v,
             double *gy, double *glog) {
  const int ns = net->n_species, nr = net->n_reactions;
#pragma omp parallel num_threads(g_threads)
  {
    double *k = xcalloc((size_t)nr, sizeof(double));
#pragma omp for schedule(static)
    for (long c = 0; c < n_cells; ++c) {
      cell_rate_coeffs(net, T + (size_t)c * n_cond(net), k);
      cell_vjp(net, k, y + (size_t)c * ns, v + (size_t)c * ns, gy ? gy + (size_t)c * ns : NULL,
               glog ? glog + (size_t)c * nr : NULL);
    }
    free(k);
  }
}

/* ------------------------------------------------------------------ LU */

/* Doolittle elimination with partial (row) pivoting; whole rows are swapped
 * so that P A = L U holds for the final factors. The row update is an
 * element-wise loop, so the AVX2 clone (picked at load time where the CPU
 * has it) rounds every element exactly as the plain one does: no
 * contraction, no reassociation. */
__attribute__((target_clones("avx2", "default")))
int orc_lu_factor(int n, double *A, int *piv) {
  int info = 0;
  for (int k = 0; k < n; ++k) {
    int p = k;
    double amax = fabs(A[(size_t)k * n + k]);
    for (int i = k + 1; i < n; ++i) {
      double v = fabs(A[(size_t)i * n + k]);
      if (v > amax) {
        amax = v;
        p = i;
      }
    }
    piv[k] = p;
    if (p != k)
      for (int j = 0; j < n; ++j) {
        double t = A[(size_t)k * n + j];
        A[(size_t)k * n + j] = A[(size_t)p * n + j];
        A[(size_t)p * n + j] = t;
      }
    double pivot = A[(size_t)k * n + k];
    if (pivot == 0.0) {
      if (!info) info = k + 1;
      continue;
    }
    for (int i = k + 1; i < n; ++i) {
      double l = A[(size_t)i * n + k] / pivot;
      A[(size_t)i * n + k] = l;
      for (int j = k + 1; j < n; ++j) A[(size_t)i * n + j] -= l * A[(size_t)k * n + j];
    }
  }
  return info;
}

void orc_lu_solve(int n, const double *LU, const int *piv, double *b) {
  for (int k = 0; k < n; ++k)
    if (piv[k] != k) {
      double t = b[k];
      b[k] = b[piv[k]];
      b[piv[k]] = t;
    }
  for (int i = 0; i < n; ++i) {
    double s = b[i];
    for (int j = 0; j < i; ++j) s -= LU[(size_t)i * n + j] * b[j];
    b[i] = s;
  }
  for (int i = n - 1; i >= 0; --i) {
    double s = b[i];
    for (int j = i + 1; j < n; ++j) s -= LU[(size_t)i * n + j] * b[j];
    b[i] = s / LU[(size_t)i * n + i];
  }
}

/* A^T x = b with A = P^T L U, i.e. A^T = U^T L^T P. */
void orc_lu_solve_t(int n, const double *LU, const int *piv, double *b) {
  for (int i = 0; i < n; ++i) {
    double s = b[i];
    for (int j = 0; j < i; ++j) s -= LU[(size_t)j * n + i] * b[j];
    b[i] = s / LU[(size_t)i * n + i];
  }
  for (int i = n - 1; i >= 0; --i) {
    double s = b[i];
    for (int j = i + 1; j < n; ++j) s -= LU[(size_t)j * n + i] * b[j];
    b[i] = s;
  }
  for (int k = n - 1; k >= 0; --k)
    if (piv[k] != k) {
      double t = b[k];
      b[k] = b[piv[k]];
      b[piv[k]] = t;
    }
}

/* ----------------------------------------------------------------- BDF
 *
 * The paper integrates with DLSODES, a variable-order BDF code (Sec. 3),
 * without giving its internals. This is the fixed-leading-coefficient BDF
 * of orders 1..5 in backward-difference form of Shampine & Reichelt (1997,
 * "The MATLAB ODE Suite", with the NDF constants kappa set to zero), with
 * the step-selection, order-selection and Newton rules fixed as follows:
 *
 *   gamma_q = sum_{m=1..q} 1/m, alpha_q = gamma_q, error constant 1/(q+1)
 *   corrector: d - c f(y_pred + d) + psi = 0, c = h/alpha_q,
 *              psi = sum_{m=1..q} gamma_m D_m / alpha_q,
 *              simplified Newton with M = I - c J, at most 4 iterations,
 *              convergence-rate test, tolerance max(10 eps/rtol,
 *              min(0.03, sqrt(rtol)))
 *   Newton failure: refresh J at y_pred once per attempt, then halve h
 *   error test: RMS of d/(atol + rtol |y|) / (q+1) <= 1
 *   step factor: safety * err^(-1/(q+1)) in [0.2, 10],
 *                safety = 0.9 (2*4+1)/(2*4 + newton iterations)
 *   order change after q+1 equal steps, to the best of q-1, q, q+1
 *   M = I - c_M J is kept while |c / c_M - 1| <= 0.3 and refactored when
 *   c moves further, or after J is refreshed (J only on Newton failure);
 *   with c != c_M every Newton correction is scaled by 2 / (1 + c / c_M).
 *   This is the matrix-reuse rule of the LSODE family the paper uses
 *   (DLSODES, Sec. 3), which the paper itself does not spell out.
 */

#define QMAX 5
#define NDROW (QMAX + 3)
#define NEWTON_MAXITER 4
#define MIN_FACTOR 0.2
#define MAX_FACTOR 10.0

typedef struct {
  double gam[NDROW];   /* gamma_q */
  double alph[NDROW];  /* alpha_q */
  double errc[NDROW];  /* error constants */
} bdf_consts;

static void bdf_constants(bdf_consts *k) {
  k->gam[0] = 0.0;
  for (int q = 1; q < NDROW; ++q) k->gam[q] = k->gam[q - 1] + 1.0 / q;
  for (int q = 0; q < NDROW; ++q) {
    k->alph[q] = k->gam[q];
    k->errc[q] = 1.0 / (q + 1);
  }
}

static double rms_scaled(int n, const double *x, double mul, const double *scale) {
  double s = 0.0;
  for (int i = 0; i < n; ++i) {
    double v = mul * x[i] / scale[i];
    s += v * v;
  }
  return sqrt(s / n);
}

/* Resample the difference array when the step changes by `factor`
 * (Shampine & Reichelt 1997): D[0..q] <- (R(factor) U)^T D[0..q] with
 * R(f)_{ij} = prod_{m=1..i} (m - 1 - f j)/m for j >= 1, R_{0j} = 1, R_{i0} = 0 (i>0),
 * and U = R(1). */
static void rescale_diffs(int n, int q, double factor, double *D) {
  double R[NDROW][NDROW], U[NDROW][NDROW], RU[NDROW][NDROW];
  for (int j = 0; j <= q; ++j) {
    R[0][j] = 1.0;
    U[0][j] = 1.0;
  }
  for (int i = 1; i <= q; ++i) {
    R[i][0] = 0.0;
    U[i][0] = 0.0;
    for (int j = 1; j <= q; ++j) {
      R[i][j] = R[i - 1][j] * ((i - 1 - factor * j) / i);
      U[i][j] = U[i - 1][j] * ((i - 1 - 1.0 * j) / i);
    }
  }
  for (int i = 0; i <= q; ++i)
    for (int j = 0; j <= q; ++j) {
      double s = 0.0;
      for (int m = 0; m <= q; ++m) s += R[i][m] * U[m][j];
      RU[i][j] = s;
    }
  double *tmp = xcalloc((size_t)(q + 1) * n, sizeof(double));
  for (int kk = 0; kk <= q; ++kk)
    for (int x = 0; x < n; ++x) {
      double s = 0.0;
      for (int i = 0; i <= q; ++i) s += RU[i][kk] * D[(size_t)i * n + x];
      tmp[(size_t)kk * n + x] = s;
    }
  memcpy(D, tmp, sizeof(double) * (size_t)(q + 1) * n);
  free(tmp);
}

/* Accept a step of order q with corrector increment d. */
static void update_diffs(int n, int q, const double *d, double *D) {
  for (int x = 0; x < n; ++x) {
    D[(size_t)(q + 2) * n + x] = d[x] - D[(size_t)(q + 1) * n + x];
    D[(size_t)(q + 1) * n + x] = d[x];
  }
  for (int i = q; i >= 0; --i)
    for (int x = 0; x < n; ++x) D[(size_t)i * n + x] += D[(size_t)(i + 1) * n + x];
}

static int all_finite(int n, const double *x) {
  for (int i = 0; i < n; ++i)
    if (!isfinite(x[i])) return 0;
  return 1;
}

static double pow_neg(double x, double e) { /* x^(-e), with 0 -> inf */
  if (x == 0.0) return INFINITY;
  return pow(x, -e);
}

typedef struct {
  const orc_net *net;
  double *k;
  int n;
  int *st;
  const double *cond;    /* temperature-coupled mode: the cell's conditions, */
  const double *therm;   /* (c_v, T_b, lambda), or NULL for T held fixed */
  double *Jb;            /* ns x ns scratch of the coupled Jacobian */
} cell_ctx;

static void F(cell_ctx *cx, const double *y, double *f) {
  if (cx->therm)
    cell_rhs_thermal(cx->net, cx->cond, cx->therm, y, cx->k, f, NULL);
  else
    cell_rhs_k(cx->net, cx->k, y, f, NULL);
  if (cx->st) cx->st[ORC_ST_RHS]++;
}

/* The Jacobian of F, n x n. */
static void JF(cell_ctx *cx, const double *y, double *J) {
  if (cx->therm)
    cell_jac_thermal(cx->net, cx->cond, cx->therm, y, cx->k, J, cx->Jb);
  else
    cell_jac(cx->net, cx->k, y, J, NULL);
}

static void build_newton_matrix(int n, double c, const double *J, double *M) {
  for (int i = 0; i < n; ++i)
    for (int a = 0; a < n; ++a) M[(size_t)i * n + a] = (i == a ? 1.0 : 0.0) - c * J[(size_t)i * n + a];
}

/* Simplified Newton on the corrector equation with M factored at c_M;
 * returns 1 if converged. */
static int newton(cell_ctx *cx, const double *ypred, double c, double cM, const double *psi,
                  const double *LU, const int *piv, const double *scale, double tol, double *ynew,
                  double *d, double *f, double *dy, int *n_iter, int *nonfinite) {
  const double corr = (c == cM) ? 1.0 : 2.0 / (1.0 + c / cM);
  const int n = cx->n;
  memcpy(ynew, ypred, sizeof(double) * n);
  for (int i = 0; i < n; ++i) d[i] = 0.0;
  double prev = 0.0;
  int conv = 0, it;
  *nonfinite = 0;
  for (it = 0; it < NEWTON_MAXITER; ++it) {
    F(cx, ynew, f);
    if (!all_finite(n, f)) {
      *nonfinite = 1;
      break;
    }
    for (int i = 0; i < n; ++i) dy[i] = c * f[i] - psi[i] - d[i];
    orc_lu_solve(n, LU, piv, dy);
    if (corr != 1.0)
      for (int i = 0; i < n; ++i) dy[i] *= corr;
    double dn = rms_scaled(n, dy, 1.0, scale);
    double rate = 0.0;
    if (it > 0) {
      rate = dn / prev;
      if (rate >= 1.0 || pow(rate, NEWTON_MAXITER - it) / (1.0 - rate) * dn > tol) break;
    }
    for (int i = 0; i < n; ++i) {
      ynew[i] += dy[i];
      d[i] += dy[i];
    }
    if (dn == 0.0 || (it > 0 && rate / (1.0 - rate) * dn < tol)) {
      conv = 1;
      break;
    }
    prev = dn;
  }
  *n_iter = it + 1;
  if (cx->st) cx->st[ORC_ST_NEWTON_IT] += (it < NEWTON_MAXITER ? it + 1 : NEWTON_MAXITER);
  return conv;
}

/* First step from the starting-step algorithm of Hairer, Norsett & Wanner
 * (Solving ODEs I, Sec. II.4) for an order-1 method. */
static double initial_step(cell_ctx *cx, const double *y0, const double *f0, double rtol,
                           double atol, double t_end) {
  const int n = cx->n;
  double *scale = xcalloc((size_t)n, sizeof(double));
  double *y1 = xcalloc((size_t)n, sizeof(double));
  double *f1 = xcalloc((size_t)n, sizeof(double));
  for (int i = 0; i < n; ++i) scale[i] = atol + rtol * fabs(y0[i]);
  double d0 = rms_scaled(n, y0, 1.0, scale);
  double d1 = rms_scaled(n, f0, 1.0, scale);
  double h0 = (d0 < 1e-5 || d1 < 1e-5) ? 1e-6 : 0.01 * d0 / d1;
  if (h0 > t_end) h0 = t_end;
  for (int i = 0; i < n; ++i) y1[i] = y0[i] + h0 * f0[i];
  F(cx, y1, f1);
  for (int i = 0; i < n; ++i) f1[i] -= f0[i];
  double d2 = rms_scaled(n, f1, 1.0, scale) / h0;
  double h1;
  if (d1 <= 1e-15 && d2 <= 1e-15)
    h1 = fmax(1e-6, h0 * 1e-3);
  else
    h1 = pow(0.01 / fmax(d1, d2), 1.0 / 2.0);
  free(scale);
  free(y1);
  free(f1);
  double h = fmin(100.0 * h0, h1);
  return fmin(h, t_end);
}

typedef struct {
  orc_event *ev;
  int cap, len, overflow;
} tape_w;

static void tape_put(tape_w *t, int type, int q, double val) {
  if (!t->ev) return;
  if (t->len >= t->cap) {
    t->overflow = 1;
    return;
  }
  t->ev[t->len].type = type;
  t->ev[t->len].q = q;
  t->ev[t->len].val = val;
  t->len++;
}

static int valid_input(int n, const double *y, const double *cond, int nc) {
  if (!(isfinite(cond[0]) && cond[0] > 0.0)) return 0;
  for (int i = 1; i < nc; ++i)
    if (!(isfinite(cond[i]) && cond[i] >= 0.0)) return 0;
  for (int i = 0; i < n; ++i)
    if (!(isfinite(y[i]) && y[i] >= 0.0)) return 0;
  return 1;
}

static int bdf_cell(const orc_net *net, const orc_bdf_opts *o, double *y, const double *cond,
                    const double *therm, double t_end, int *st, tape_w *tw) {
  const int ns = net->n_species, nr = net->n_reactions, n = ns + (therm ? 1 : 0);
  if (!valid_input(ns, y, cond, n_cond(net))) return ORC_BADINPUT;
  if (therm && !(isfinite(y[ns]) && y[ns] > 0.0 && therm[0] > 0.0 && isfinite(therm[0]) &&
                 therm[1] > 0.0 && isfinite(therm[1]) && therm[2] >= 0.0 && isfinite(therm[2])))
    return ORC_BADINPUT;
  if (!(t_end > 0.0)) return ORC_OK;
  bdf_consts K;
  bdf_constants(&K);
  const int qmax = o->q_max;
  const double rtol = o->rtol, atol = o->atol;
  const double tol = o->newton_tol > 0.0 ? o->newton_tol
                                         : fmax(10.0 * DBL_EPSILON / rtol, fmin(0.03, sqrt(rtol)));

  double *k = xcalloc((size_t)nr, sizeof(double));
  double *D = xcalloc((size_t)NDROW * n, sizeof(double));
  double *J = xcalloc((size_t)n * n, sizeof(double));
  double *LU = xcalloc((size_t)n * n, sizeof(double));
  int *piv = xcalloc((size_t)n, sizeof(int));
  double *ypred = xcalloc((size_t)n, sizeof(double));
  double *psi = xcalloc((size_t)n, sizeof(double));
  double *scale = xcalloc((size_t)n, sizeof(double));
  double *ynew = xcalloc((size_t)n, sizeof(double));
  double *d = xcalloc((size_t)n, sizeof(double));
  double *f = xcalloc((size_t)n, sizeof(double));
  double *dy = xcalloc((size_t)n, sizeof(double));
  double *Jb = therm ? xcalloc((size_t)ns * ns, sizeof(double)) : NULL;

  if (!therm) cell_rate_coeffs(net, cond, k);
  cell_ctx cx = {net, k, n, st, cond, therm, Jb};
  F(&cx, y, f);
  double h = o->h0 > 0.0 ? fmin(o->h0, t_end) : initial_step(&cx, y, f, rtol, atol, t_end);
  tape_put(tw, ORC_EV_INIT, 1, h);
  for (int x = 0; x < n; ++x) {
    D[x] = y[x];
    D[n + x] = h * f[x];
  }
  JF(&cx, y, J);
  if (st) st[ORC_ST_JAC]++;

  int status = ORC_OK, q = 1, n_equal = 0, lu_valid = 0, steps = 0;
  /* why the last attempt was rejected, reported if h falls below h_min:
   * the error test, a Newton failure with finite values, a non-finite RHS,
   * or an exactly singular Newton matrix */
  int last_fail = ORC_HMIN, lu_info = 0;
  double cM = 0.0;
  double t = 0.0, h_abs = h;
  while (t < t_end) {
    if (steps >= o->max_steps) {
      status = ORC_MAXSTEPS;
      break;
    }
    const double hmin = 10.0 * (nextafter(t, INFINITY) - t);
    int jac_fresh = 0, n_iter = 0, nonfin = 0;
    double t_new = t, en = 0.0, safety = 0.0;
    for (;;) { /* attempts */
      if (h_abs < hmin) {
        status = last_fail;
        goto done;
      }
      t_new = t + h_abs;
      if (t_new > t_end) {
        t_new = t_end;
        double factor = (t_new - t) / h_abs;
        rescale_diffs(n, q, factor, D);
        tape_put(tw, ORC_EV_RESCALE, q, factor);
        n_equal = 0;
      }
      h = t_new - t;
      h_abs = h;
      for (int x = 0; x < n; ++x) {
        double s = 0.0;
        for (int m = 0; m <= q; ++m) s += D[(size_t)m * n + x];
        ypred[x] = s;
        scale[x] = atol + rtol * fabs(s);
        double p = 0.0;
        for (int m = 1; m <= q; ++m) p += K.gam[m] * D[(size_t)m * n + x];
        psi[x] = p / K.alph[q];
      }
      const double c = h / K.alph[q];
      int conv = 0;
      for (;;) {
        if (!lu_valid || fabs(c / cM - 1.0) > 0.3) {
          build_newton_matrix(n, c, J, LU);
          lu_info = orc_lu_factor(n, LU, piv);
          if (st) st[ORC_ST_LU]++;
          lu_valid = 1;
          cM = c;
        }
        conv = newton(&cx, ypred, c, cM, psi, LU, piv, scale, tol, ynew, d, f, dy, &n_iter,
                      &nonfin);
        if (conv || jac_fresh) break;
        JF(&cx, ypred, J);
        if (st) st[ORC_ST_JAC]++;
        jac_fresh = 1;
        lu_valid = 0;
      }
      if (!conv) {
        last_fail = lu_info ? ORC_SINGULAR : nonfin ? ORC_NONFINITE : ORC_NEWTON_FAIL;
        h_abs *= 0.5;
        rescale_diffs(n, q, 0.5, D);
        tape_put(tw, ORC_EV_RESCALE, q, 0.5);
        n_equal = 0;
        if (st) st[ORC_ST_REJECT_NEWTON]++;
        continue;
      }
      safety = 0.9 * (2 * NEWTON_MAXITER + 1) / (2 * NEWTON_MAXITER + n_iter);
      for (int x = 0; x < n; ++x) scale[x] = atol + rtol * fabs(ynew[x]);
      en = rms_scaled(n, d, K.errc[q], scale);
      if (en > 1.0) {
        last_fail = ORC_HMIN;
        double factor = fmax(MIN_FACTOR, safety * pow_neg(en, 1.0 / (q + 1)));
        h_abs *= factor;
        rescale_diffs(n, q, factor, D);
        tape_put(tw, ORC_EV_RESCALE, q, factor);
        n_equal = 0;
        if (st) st[ORC_ST_REJECT_ERR]++;
        continue;
      }
      break;
    }
    /* accepted */
    t = t_new;
    steps++;
    tape_put(tw, ORC_EV_STEP, q, h);
    update_diffs(n, q, d, D);
    n_equal++;
    if (n_equal < q + 1) continue;
    double em = q > 1 ? rms_scaled(n, D + (size_t)q * n, K.errc[q - 1], scale) : INFINITY;
    double ep = q < qmax ? rms_scaled(n, D + (size_t)(q + 2) * n, K.errc[q + 1], scale) : INFINITY;
    double fac[3] = {pow_neg(em, 1.0 / q), pow_neg(en, 1.0 / (q + 1)), pow_neg(ep, 1.0 / (q + 2))};
    int best = 0;
    for (int i = 1; i < 3; ++i)
      if (fac[i] > fac[best]) best = i;
    q += best - 1;
    double factor = fmin(MAX_FACTOR, safety * fac[best]);
    h_abs *= factor;
    rescale_diffs(n, q, factor, D);
    tape_put(tw, ORC_EV_RESCALE, q, factor);
    n_equal = 0;
  }
done:
  memcpy(y, D, sizeof(double) * n);
  if (st) {
    st[ORC_ST_STEPS] = steps;
    st[ORC_ST_QLAST] = q;
  }
  free(k); free(D); free(J); free(LU); free(piv); free(ypred); free(psi);
  free(scale); free(ynew); free(d); free(f); free(dy); free(Jb);
  return status;
}

void orc_bdf(const orc_net *net, const orc_bdf_opts *opt, long n_cells, double *y,
             const double *T, double t_end, int *status, int *stats, orc_event *tape, int tape_cap,
             int *tape_len) {
  const int ns = net->n_species;
#pragma omp parallel for num_threads(g_threads) schedule(dynamic, 1)
  for (long c = 0; c < n_cells; ++c) {
    int *st = stats ? stats + (size_t)c * ORC_NSTAT : NULL;
    if (st) memset(st, 0, sizeof(int) * ORC_NSTAT);
    tape_w tw = {tape ? tape + (size_t)c * tape_cap : NULL, tape_cap, 0, 0};
    int s = bdf_cell(net, opt, y + (size_t)c * ns, T + (size_t)c * n_cond(net), NULL, t_end, st,
                     &tw);
    if (status) status[c] = s;
    if (tape_len) tape_len[c] = tw.overflow ? -1 : tw.len;
  }
}

void orc_bdf_thermal(const orc_net *net, const orc_bdf_opts *opt, long n_cells, double *y,
                     const double *cond, const double *therm, double t_end, int *status,
                     int *stats) {
  const int n = net->n_species + 1;
#pragma omp parallel for num_threads(g_threads) schedule(dynamic, 1)
  for (long c = 0; c < n_cells; ++c) {
    int *st = stats ? stats + (size_t)c * ORC_NSTAT : NULL;
    if (st) memset(st, 0, sizeof(int) * ORC_NSTAT);
    tape_w tw = {NULL, 0, 0, 0};
    int s = bdf_cell(net, opt, y + (size_t)c * n, cond + (size_t)c * n_cond(net),
                     therm + (size_t)c * 3, t_end, st, &tw);
    if (status) status[c] = s;
  }
}

/* ------------------------------------------------ replay + sensitivity */

/* d(dydt)/d(log alpha) applied to direction w: sum_j w_j R_j S_:j. */
static void rhs_param_dir(const orc_net *net, const double *k, const double *y, const double *w,
                          double *out) {
  const int ns = net->n_species, nr = net->n_reactions;
  for (int i = 0; i < ns; ++i) out[i] = 0.0;
  for (int j = 0; j < nr; ++j) {
    if (w[j] == 0.0) continue;
    double r = reaction_rate(net, k, y, j) * w[j];
    for (int s = 0; s < NRS; ++s) {
      int a = net->reactants[j * NRS + s];
      if (a >= 0) out[a] -= r;
    }
    for (int s = 0; s < NPS; ++s) {
      int p = net->products[j * NPS + s];
      if (p >= 0) out[p] += r;
    }
  }
}

static void matvec(int n, const double *A, const double *x, double *out) {
  for (int i = 0; i < n; ++i) {
    double s = 0.0;
    for (int a = 0; a < n; ++a) s += A[(size_t)i * n + a] * x[a];
    out[i] = s;
  }
}

/* The step sequence (h, q and every resampling) is taken from the tape, and
 * the corrector equation is solved to convergence, so the result is a smooth
 * function of the initial state and parameters. Tangents follow from
 * differentiating each step:  (I - c J(y)) s_d = c (J(y) s_pred + f_p) - s_psi. */
static void replay_cell(const orc_net *net, const orc_bdf_opts *o, const double *y0,
                        const double *cond,
                        const orc_event *ev, int n_ev, int n_dir, const double *dy0,
                        const double *dlogalpha, double *y_out, double *s_out) {
  const int n = net->n_species, nr = net->n_reactions;
  bdf_consts K;
  bdf_constants(&K);
  double *k = xcalloc((size_t)nr, sizeof(double));
  double *D = xcalloc((size_t)NDROW * n, sizeof(double));
  double *sD = xcalloc((size_t)(n_dir > 0 ? n_dir : 1) * NDROW * n, sizeof(double));
  double *J = xcalloc((size_t)n * n, sizeof(double));
  double *LU = xcalloc((size_t)n * n, sizeof(double));
  int *piv = xcalloc((size_t)n, sizeof(int));
  double *ypred = xcalloc((size_t)n, sizeof(double));
  double *psi = xcalloc((size_t)n, sizeof(double));
  double *scale = xcalloc((size_t)n, sizeof(double));
  double *y = xcalloc((size_t)n, sizeof(double));
  double *d = xcalloc((size_t)n, sizeof(double));
  double *f = xcalloc((size_t)n, sizeof(double));
  double *g = xcalloc((size_t)n, sizeof(double));
  double *t1 = xcalloc((size_t)n, sizeof(double));
  double *t2 = xcalloc((size_t)n, sizeof(double));
  double *sd = xcalloc((size_t)n, sizeof(double));

  cell_rate_coeffs(net, cond, k);
  cell_ctx cx = {net, k, n, NULL, cond, NULL, NULL};
  memcpy(D, y0, sizeof(double) * n);
  for (int r = 0; r < n_dir; ++r)
    for (int x = 0; x < n; ++x) sD[(size_t)r * NDROW * n + x] = dy0 ? dy0[(size_t)r * n + x] : 0.0;

  for (int e = 0; e < n_ev; ++e) {
    const int q = ev[e].q;
    if (ev[e].type == ORC_EV_INIT) {
      const double h0 = ev[e].val;
      F(&cx, y0, f);
      for (int x = 0; x < n; ++x) D[n + x] = h0 * f[x];
      if (n_dir > 0) cell_jac(net, k, y0, J, NULL);
      for (int r = 0; r < n_dir; ++r) {
        double *S = sD + (size_t)r * NDROW * n;
        matvec(n, J, S, t1);
        if (dlogalpha) {
          rhs_param_dir(net, k, y0, dlogalpha + (size_t)r * nr, t2);
          for (int x = 0; x < n; ++x) t1[x] += t2[x];
        }
        for (int x = 0; x < n; ++x) S[n + x] = h0 * t1[x];
      }
    } else if (ev[e].type == ORC_EV_RESCALE) {
      rescale_diffs(n, q, ev[e].val, D);
      for (int r = 0; r < n_dir; ++r) rescale_diffs(n, q, ev[e].val, sD + (size_t)r * NDROW * n);
    } else if (ev[e].type == ORC_EV_STEP) {
      const double c = ev[e].val / K.alph[q];
      for (int x = 0; x < n; ++x) {
        double s = 0.0;
        for (int m = 0; m <= q; ++m) s += D[(size_t)m * n + x];
        ypred[x] = s;
        scale[x] = o->atol + o->rtol * fabs(s);
        double p = 0.0;
        for (int m = 1; m <= q; ++m) p += K.gam[m] * D[(size_t)m * n + x];
        psi[x] = p / K.alph[q];
        d[x] = 0.0;
      }
      /* Newton on G(d) = d - c f(y_pred + d) + psi, with the matrix
       * refreshed at the current iterate whenever the contraction is slow,
       * until the update is at rounding level. */
      double prev = INFINITY;
      int fresh = 0;
      for (int it = 0; it < 60; ++it) {
        for (int x = 0; x < n; ++x) y[x] = ypred[x] + d[x];
        if (!fresh) {
          cell_jac(net, k, y, J, NULL);
          build_newton_matrix(n, c, J, LU);
          orc_lu_factor(n, LU, piv);
          fresh = 1;
        }
        F(&cx, y, f);
        for (int x = 0; x < n; ++x) g[x] = -(d[x] - c * f[x] + psi[x]);
        orc_lu_solve(n, LU, piv, g);
        double dn = rms_scaled(n, g, 1.0, scale);
        for (int x = 0; x < n; ++x) d[x] += g[x];
        if (dn <= 1e-10) break;                               /* converged */
        if (dn <= 1e-7 && dn > 0.5 * prev) break;              /* at rounding level */
        if (dn > 0.1 * prev) fresh = 0;                        /* slow: full Newton */
        prev = dn;
      }
      for (int x = 0; x < n; ++x) y[x] = ypred[x] + d[x];
      if (n_dir > 0) {
        cell_jac(net, k, y, J, NULL);
        build_newton_matrix(n, c, J, LU);
        orc_lu_factor(n, LU, piv);
      }
      for (int r = 0; r < n_dir; ++r) {
        double *S = sD + (size_t)r * NDROW * n;
        for (int x = 0; x < n; ++x) {
          double sp = 0.0, ss = 0.0;
          for (int m = 0; m <= q; ++m) sp += S[(size_t)m * n + x];
          for (int m = 1; m <= q; ++m) ss += K.gam[m] * S[(size_t)m * n + x];
          t1[x] = sp;
          g[x] = ss / K.alph[q];
        }
        matvec(n, J, t1, t2);
        if (dlogalpha) rhs_param_dir(net, k, y, dlogalpha + (size_t)r * nr, t1);
        else
          for (int x = 0; x < n; ++x) t1[x] = 0.0;
        for (int x = 0; x < n; ++x) sd[x] = c * (t2[x] + t1[x]) - g[x];
        orc_lu_solve(n, LU, piv, sd);
        update_diffs(n, q, sd, S);
      }
      update_diffs(n, q, d, D);
    }
  }
  memcpy(y_out, D, sizeof(double) * n);
  for (int r = 0; r < n_dir; ++r)
    memcpy(s_out + (size_t)r * n, sD + (size_t)r * NDROW * n, sizeof(double) * n);
  free(k); free(D); free(sD); free(J); free(LU); free(piv); free(ypred); free(psi);
  free(scale); free(y); free(d); free(f); free(g); free(t1); free(t2); free(sd);
}

void orc_bdf_replay(const orc_net *net, const orc_bdf_opts *opt, long n_cells, const double *y0,
                    const double *T, const orc_event *tape, int tape_cap, const int *tape_len,
                    int n_dir, const double *dy0, const double *dlogalpha, double *y_out,
                    double *s_out) {
  const int ns = net->n_species;
#pragma omp parallel for num_threads(g_threads) schedule(dynamic, 1)
  for (long c = 0; c < n_cells; ++c)
    replay_cell(net, opt, y0 + (size_t)c * ns, T + (size_t)c * n_cond(net), tape + (size_t)c * tape_cap, tape_len[c],
                n_dir, dy0 ? dy0 + (size_t)c * n_dir * ns : NULL, dlogalpha,
                y_out + (size_t)c * ns, s_out ? s_out + (size_t)c * n_dir * ns : NULL);
}
