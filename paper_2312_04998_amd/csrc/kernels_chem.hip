// Rate coefficients, RHS, Jacobian and VJP kernels for gfx950.
//
// Mapping: one workgroup (four 64-wide waves) works on one cell at a time
// and strides over cells. A cell's densities are staged in LDS with a
// coalesced load; the per-reaction quantities (rates R_j for the RHS,
// coefficients k_j for the Jacobian, k_j (S^T v)_j for the VJP) are
// computed once per cell into an LDS block; the product with S is then a
// gather over precomputed term lists (rows of S, entries of the Jacobian
// pattern, reactant slots of a species), split into short chunks so heavy
// rows (H, H2, e- take part in 15-30 % of reactions) are shared by many
// lanes. Network data (a few hundred KB) stays in L2 for all cells.
#include "devnet.h"

namespace ac {

constexpr int BLOCK = 256;

// value of one packed term: coef * A[j] * (b == NONE ? 1 : y[b])
__device__ __forceinline__ double term(uint32_t it, const double *__restrict__ A,
                                       const double *__restrict__ ys) {
  const int j = int(it & 0xFFFFu);
  const int b = int((it >> 16) & 2047u);
  const int coef = int32_t(it) >> 27;
  double v = double(coef) * A[j];
  if (b != 2047) v *= ys[b];
  return v;
}

// Chunk sums of a schedule: single-chunk segments go straight to out,
// split segments leave partials in `part` for segsum_finish.
template <int LAYOUT>
__device__ __forceinline__ void segsum_chunks(const DSched &s, const double *__restrict__ A,
                                              const double *__restrict__ ys, double *part,
                                              double *__restrict__ out) {
  if (LAYOUT == LAYOUT_SELL) {
    const int npos = s.n_slice * s.sell_c;
    for (int pos = threadIdx.x; pos < npos; pos += BLOCK) {
      const int ch = s.sell_chunk[pos];
      if (ch < 0) continue;
      const int sl = pos / s.sell_c;
      const int len = s.sell_len[pos];
      const uint32_t *it = s.sell_items + s.slice_ptr[sl] + (pos - sl * s.sell_c);
      double acc = 0.0;
      for (int k = 0; k < len; ++k) acc += term(it[k * s.sell_c], A, ys);
      const int d = s.chunk_dst[ch];
      if (d >= 0) out[d] = acc;
      else part[-1 - d] = acc;
    }
  } else {
    for (int ch = threadIdx.x; ch < s.n_chunk; ch += BLOCK) {
      double acc = 0.0;
      const int e = s.chunk_ptr[ch + 1];
      for (int p = s.chunk_ptr[ch]; p < e; ++p) acc += term(s.items[p], A, ys);
      const int d = s.chunk_dst[ch];
      if (d >= 0) out[d] = acc;
      else part[-1 - d] = acc;
    }
  }
}

__device__ __forceinline__ void segsum_finish(const DSched &s, const double *part,
                                              double *__restrict__ out) {
  for (int m = threadIdx.x; m < s.n_multi; m += BLOCK) {
    const int q0 = s.multi_slot[m], q1 = s.multi_slot[m + 1];
    double acc = part[q0];
    for (int q = q0 + 1; q < q1; ++q) acc += part[q];
    out[s.multi_out[m]] = acc;
  }
}

// Full segmented sum (partials in LDS, so a barrier sits in between).
template <int LAYOUT>
__device__ __forceinline__ void segsum(const DSched &s, const double *A, const double *ys,
                                       double *part, double *out) {
  if (LAYOUT == LAYOUT_COO) {
    // scatter with LDS atomics into a per-cell accumulator (order varies)
    for (int i = threadIdx.x; i < s.n_seg; i += BLOCK) part[i] = 0.0;
    __syncthreads();
    for (int p = threadIdx.x; p < s.n_item; p += BLOCK)
      atomicAdd(&part[s.coo_out[p]], term(s.items[p], A, ys));
    __syncthreads();
    for (int i = threadIdx.x; i < s.n_seg; i += BLOCK) out[i] = part[i];
    return;
  }
  segsum_chunks<LAYOUT>(s, A, ys, part, out);
  __syncthreads();
  segsum_finish(s, part, out);
}

__device__ __forceinline__ void load_cell(const double *__restrict__ src, double *dst, int n) {
  for (int i = threadIdx.x; i < n; i += BLOCK) dst[i] = src[i];
}

// k_j = exp(ln alpha_j + beta_j ln(T/300) - gamma_j / T)
__device__ __forceinline__ double rate_coeff(const DNet &n, const double *la, int j, double L,
                                             double invT) {
  return exp(la[j] + n.beta[j] * L - n.gamma[j] * invT);
}

__device__ __forceinline__ double reaction_rate(uint32_t pair, double k, const double *ys) {
  double r = k * ys[pair & 0xFFFFu];
  const uint32_t b = pair >> 16;
  if (b != 0xFFFFu) r *= ys[b];
  return r;
}

// ------------------------------------------------------------------ rates

__global__ __launch_bounds__(BLOCK) void k_rates(DNet n, const double *__restrict__ la_over,
                                                 int64_t n_cells, const double *__restrict__ T,
                                                 double *__restrict__ k) {
  const double *la = la_over ? la_over : n.log_alpha;
  for (int64_t c = blockIdx.x; c < n_cells; c += gridDim.x) {
    const double Tc = T[c];
    const double L = log(Tc / 300.0), invT = 1.0 / Tc;
    double *kc = k + c * n.nr;
    for (int j = threadIdx.x; j < n.nr; j += BLOCK)
      __builtin_nontemporal_store(rate_coeff(n, la, j, L, invT), kc + j);
  }
}

// -------------------------------------------------------------------- RHS

template <int LAYOUT, bool PREK>
__global__ __launch_bounds__(BLOCK) void k_rhs(DNet n, const double *__restrict__ la_over,
                                               int64_t n_cells, const double *__restrict__ y,
                                               const double *__restrict__ T,
                                               const double *__restrict__ kin,
                                               double *__restrict__ dydt) {
  extern __shared__ double sm[];
  const int ns = n.ns, nr = n.nr;
  double *ys = sm;
  double *rs = sm + ns;
  double *part = rs + nr;
  const double *la = la_over ? la_over : n.log_alpha;
  for (int64_t c = blockIdx.x; c < n_cells; c += gridDim.x) {
    load_cell(y + c * ns, ys, ns);
    double L = 0.0, invT = 0.0;
    if (!PREK) {
      const double Tc = T[c];
      L = log(Tc / 300.0);
      invT = 1.0 / Tc;
    }
    __syncthreads();
    const double *kc = PREK ? kin + c * nr : nullptr;
    for (int j = threadIdx.x; j < nr; j += BLOCK) {
      const double kj = PREK ? __builtin_nontemporal_load(kc + j) : rate_coeff(n, la, j, L, invT);
      rs[j] = reaction_rate(n.rpair[j], kj, ys);
    }
    __syncthreads();
    segsum<LAYOUT>(n.rhs, rs, ys, part, dydt + c * ns);
    __syncthreads();
  }
}

// --------------------------------------------------------------- Jacobian

__global__ __launch_bounds__(BLOCK) void k_jac(DNet n, const double *__restrict__ la_over,
                                               int64_t n_cells, const double *__restrict__ y,
                                               const double *__restrict__ T,
                                               double *__restrict__ jvals) {
  extern __shared__ double sm[];
  const int ns = n.ns, nr = n.nr;
  double *ys = sm;
  double *ks = sm + ns;
  double *part = ks + nr;
  const double *la = la_over ? la_over : n.log_alpha;
  for (int64_t c = blockIdx.x; c < n_cells; c += gridDim.x) {
    load_cell(y + c * ns, ys, ns);
    const double Tc = T[c];
    const double L = log(Tc / 300.0), invT = 1.0 / Tc;
    for (int j = threadIdx.x; j < nr; j += BLOCK) ks[j] = rate_coeff(n, la, j, L, invT);
    __syncthreads();
    double *out = jvals + c * n.nnz_j;
    segsum_chunks<LAYOUT_CSR>(n.jac, ks, ys, part, out);
    __syncthreads();
    segsum_finish(n.jac, part, out);
    __syncthreads();
  }
}

// -------------------------------------------------------------------- VJP
//
// w_j = (S^T v)_j from the CCS of S; gy_a = sum over reactant slots of a of
// mult * k_j * n_other * w_j. The log-alpha gradient sum_c R_cj w_cj goes
// to a per-workgroup row of partial sums: a thread always owns the same
// reactions and a workgroup the same cells (fixed grid), so the row is
// updated without atomics, and the rows are added in workgroup order.

__global__ __launch_bounds__(BLOCK) void k_vjp(DNet n, const double *__restrict__ la_over,
                                               int64_t n_cells, const double *__restrict__ y,
                                               const double *__restrict__ T,
                                               const double *__restrict__ v,
                                               double *__restrict__ gy,
                                               double *__restrict__ part_glog) {
  extern __shared__ double sm[];
  const int ns = n.ns, nr = n.nr;
  double *ys = sm;
  double *vs = ys + ns;
  double *kw = vs + ns;
  double *part = kw + nr;
  const double *la = la_over ? la_over : n.log_alpha;
  double *prow = part_glog ? part_glog + size_t(blockIdx.x) * nr : nullptr;
  if (prow)
    for (int j = threadIdx.x; j < nr; j += BLOCK) prow[j] = 0.0;
  for (int64_t c = blockIdx.x; c < n_cells; c += gridDim.x) {
    load_cell(y + c * ns, ys, ns);
    load_cell(v + c * ns, vs, ns);
    const double Tc = T[c];
    const double L = log(Tc / 300.0), invT = 1.0 / Tc;
    __syncthreads();
    for (int j = threadIdx.x; j < nr; j += BLOCK) {
      double w = 0.0;
      const int p1 = n.s_col_ptr[j + 1];
      for (int p = n.s_col_ptr[j]; p < p1; ++p) w += double(n.s_cval[p]) * vs[n.s_row[p]];
      const double kj = rate_coeff(n, la, j, L, invT);
      kw[j] = kj * w;
      if (prow) prow[j] += reaction_rate(n.rpair[j], kj, ys) * w;
    }
    __syncthreads();
    if (gy) {
      double *out = gy + c * ns;
      segsum_chunks<LAYOUT_CSR>(n.gy, kw, ys, part, out);
      __syncthreads();
      segsum_finish(n.gy, part, out);
    }
    __syncthreads();
  }
}

__global__ __launch_bounds__(BLOCK) void k_fill(double *__restrict__ p, int64_t n, double v) {
  for (int64_t i = blockIdx.x * int64_t(BLOCK) + threadIdx.x; i < n; i += int64_t(gridDim.x) * BLOCK)
    p[i] = v;
}

__global__ __launch_bounds__(BLOCK) void k_sum_rows(const double *__restrict__ part, int rows,
                                                    int nr, double *__restrict__ out) {
  const int j = blockIdx.x * BLOCK + threadIdx.x;
  if (j >= nr) return;
  double s = 0.0;
  for (int r = 0; r < rows; ++r) s += part[size_t(r) * nr + j];
  out[j] = s;
}

// ---------------------------------------------------------------- launch

static int device_cus() {
  static int cus = 0;
  if (!cus) {
    int dev = 0;
    hipGetDevice(&dev);
    hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (cus <= 0) cus = 256;
  }
  return cus;
}

template <typename K>
static int grid_for(K kernel, size_t lds, int64_t n_cells) {
  if (lds > 65536) hipFuncSetAttribute(reinterpret_cast<const void *>(kernel),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, int(lds));
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, BLOCK, lds) != hipSuccess ||
      per_cu <= 0)
    per_cu = 1;
  const int64_t g = int64_t(per_cu) * device_cus();
  return int(n_cells < g ? n_cells : g);
}

size_t rhs_lds_bytes(const DNet &n) {
  const int extra = n.layout == LAYOUT_COO ? n.ns : n.rhs.n_slot;
  return sizeof(double) * size_t(n.ns + n.nr + (extra > 0 ? extra : 1));
}

hipError_t launch_rates(const DNet &n, const double *la, int64_t n_cells, const double *T,
                        double *k, hipStream_t st) {
  if (n_cells == 0) return hipSuccess;
  const int g = grid_for(k_rates, 0, n_cells);
  hipLaunchKernelGGL(k_rates, dim3(g), dim3(BLOCK), 0, st, n, la, n_cells, T, k);
  return hipGetLastError();
}

template <int LAYOUT, bool PREK>
static hipError_t rhs_variant(const DNet &n, const double *la, int64_t n_cells, const double *y,
                              const double *T, const double *k, double *dydt, hipStream_t st) {
  const size_t lds = rhs_lds_bytes(n);
  auto kern = k_rhs<LAYOUT, PREK>;
  const int g = grid_for(kern, lds, n_cells);
  hipLaunchKernelGGL(kern, dim3(g), dim3(BLOCK), lds, st, n, la, n_cells, y, T, k, dydt);
  return hipGetLastError();
}

hipError_t launch_rhs(const DNet &n, const double *la, int64_t n_cells, const double *y,
                      const double *T, const double *k, double *dydt, hipStream_t st) {
  if (n_cells == 0) return hipSuccess;
  if (k) {
    if (n.layout == LAYOUT_SELL) return rhs_variant<LAYOUT_SELL, true>(n, la, n_cells, y, T, k, dydt, st);
    if (n.layout == LAYOUT_COO) return rhs_variant<LAYOUT_COO, true>(n, la, n_cells, y, T, k, dydt, st);
    return rhs_variant<LAYOUT_CSR, true>(n, la, n_cells, y, T, k, dydt, st);
  }
  if (n.layout == LAYOUT_SELL) return rhs_variant<LAYOUT_SELL, false>(n, la, n_cells, y, T, k, dydt, st);
  if (n.layout == LAYOUT_COO) return rhs_variant<LAYOUT_COO, false>(n, la, n_cells, y, T, k, dydt, st);
  return rhs_variant<LAYOUT_CSR, false>(n, la, n_cells, y, T, k, dydt, st);
}

hipError_t launch_jac(const DNet &n, const double *la, int64_t n_cells, const double *y,
                      const double *T, double *jvals, hipStream_t st) {
  if (n_cells == 0) return hipSuccess;
  const size_t lds = sizeof(double) * size_t(n.ns + n.nr + (n.jac.n_slot > 0 ? n.jac.n_slot : 1));
  const int g = grid_for(k_jac, lds, n_cells);
  hipLaunchKernelGGL(k_jac, dim3(g), dim3(BLOCK), lds, st, n, la, n_cells, y, T, jvals);
  return hipGetLastError();
}

hipError_t launch_vjp(const DNet &n, const double *la, int64_t n_cells, const double *y,
                      const double *T, const double *v, double *gy, double *g_logalpha,
                      double *part, int part_rows, hipStream_t st) {
  if (n_cells == 0) {
    if (g_logalpha) {
      hipLaunchKernelGGL(k_fill, dim3((n.nr + BLOCK - 1) / BLOCK), dim3(BLOCK), 0, st, g_logalpha,
                         int64_t(n.nr), 0.0);
      return hipGetLastError();
    }
    return hipSuccess;
  }
  const size_t lds = sizeof(double) * size_t(2 * n.ns + n.nr + (n.gy.n_slot > 0 ? n.gy.n_slot : 1));
  // a fixed grid (independent of occupancy) keeps the cell-to-workgroup
  // assignment, and so the summation order, the same on every call
  const int g = int(n_cells < part_rows ? n_cells : part_rows);
  if (lds > 65536) hipFuncSetAttribute(reinterpret_cast<const void *>(k_vjp),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, int(lds));
  hipLaunchKernelGGL(k_vjp, dim3(g), dim3(BLOCK), lds, st, n, la, n_cells, y, T, v, gy,
                     g_logalpha ? part : nullptr);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || !g_logalpha) return e;
  hipLaunchKernelGGL(k_sum_rows, dim3((n.nr + BLOCK - 1) / BLOCK), dim3(BLOCK), 0, st, part, g,
                     n.nr, g_logalpha);
  return hipGetLastError();
}

}  // namespace ac
