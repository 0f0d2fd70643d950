// Temperature as a state variable (codes that solve temperature and
// abundances together within the stiff solver, Sec. 5): per cell the state
// is (n_1..n_ns, T), the rate coefficients follow the state's T, and
//
//     dT/dt = (sum_j heat_j R_j) / c_v - lambda (T - T_b),
//
// heat_j the energy released per reaction event, therm[c] = (c_v, T_b,
// lambda) per cell. The RHS recomputes every coefficient (one exp per
// reaction) on each call; the Jacobian adds to the pattern values a T
// column sum_j S_ij R_j dln k_j/dT, a T row sum_j heat_j dR_j/dn_a / c_v
// and the corner. One workgroup per cell, striding over cells; the
// per-reaction block and the partial sums live in LDS as in the
// fixed-temperature kernels.
#include "devchem.h"
#include "devla.h"

namespace ac {

template <int NT>
__global__ __launch_bounds__(NT) void k_rhs_th(DNet n, const double *__restrict__ la_over,
                                               int64_t n_cells, const double *__restrict__ y,
                                               const double *__restrict__ cond,
                                               const double *__restrict__ therm,
                                               double *__restrict__ dydt) {
  extern __shared__ double sm[];
  __shared__ double red[NT / 64];
  const int ns = n.ns, nv = ns + 1, nr = n.nr, nc = n.n_cond;
  double *ys = sm, *rs = ys + nv, *part = rs + nr;
  for (int64_t c = blockIdx.x; c < n_cells; c += gridDim.x) {
    load_cell<NT>(y + c * nv, ys, nv);
    __syncthreads();
    const double Tc = ys[ns];
    const double *th = therm + c * 3;
    const Env env = env_with_T(cond + c * nc, nc, Tc);
    double hsum = 0.0;
    for_rx<NT>(n, la_over, env, [&](int j, double kj, const Rx &r) {
      const double rj = reaction_rate(r.pair, kj, ys);
      rs[j] = rj;
      if (n.heat) hsum += n.heat[j] * rj;
    });
    __syncthreads();
    double *out = dydt + c * nv;
    segsum_chunks<NT, LAYOUT_SELL, false, false>(n.rhs, rs, ys, part, out);
    __syncthreads();
    segsum_finish<NT, false>(n.rhs, part, out);
    const double q = wg_sum<NT>(hsum, red);
    if (threadIdx.x == 0) out[ns] = q / th[0] - th[2] * (Tc - th[1]);
    __syncthreads();
  }
}

// jvals[c] = (pattern values [nnz_j], T column [ns], T row [ns], corner).
template <int NT>
__global__ __launch_bounds__(NT) void k_jac_th(DNet n, const double *__restrict__ la_over,
                                               int64_t n_cells, const double *__restrict__ y,
                                               const double *__restrict__ cond,
                                               const double *__restrict__ therm,
                                               double *__restrict__ jvals) {
  extern __shared__ double sm[];
  __shared__ double red[NT / 64];
  const int ns = n.ns, nv = ns + 1, nr = n.nr, nc = n.n_cond, nnz = n.nnz_j;
  double *ys = sm, *ks = ys + nv, *ws = ks + nr, *part = ws + nr;
  for (int64_t c = blockIdx.x; c < n_cells; c += gridDim.x) {
    load_cell<NT>(y + c * nv, ys, nv);
    __syncthreads();
    const double Tc = ys[ns];
    const double *th = therm + c * 3;
    const Env env = env_with_T(cond + c * nc, nc, Tc);
    double csum = 0.0;
    for_rx<NT>(n, la_over, env, [&](int j, double kj, const Rx &r) {
      ks[j] = kj;
      const double w = reaction_rate(r.pair, kj, ys) * rate_dlnk_dT(r, env.invT);
      ws[j] = w;
      if (n.heat) csum += n.heat[j] * w;
    });
    __syncthreads();
    double *out = jvals + c * (size_t(nnz) + 2 * ns + 1);
    // pattern values: tail partials, then every entry's heads and tails
    runsum_partials<NT>(n.jtail, ks, ys, part);
    __syncthreads();
    for (int e = threadIdx.x; e < nnz; e += NT) {
      double acc = term(n.jhead0[e], ks, ys);
      acc = __dadd_rn(acc, term(n.jhead1[e], ks, ys));
      const uint32_t td = n.jtaildesc[e];
      const int q0 = int(td >> 8), nq = int(td & 255u);
      for (int q = 0; q < nq; ++q) acc = __dadd_rn(acc, part[q0 + q]);
      out[e] = acc;
    }
    __syncthreads();
    // T column: rows of S applied to R_j dln k_j/dT
    segsum_chunks<NT, LAYOUT_SELL, false, false>(n.rhs, ws, ys, part, out + nnz);
    __syncthreads();
    segsum_finish<NT, false>(n.rhs, part, out + nnz);
    __syncthreads();
    // T row: reactant slots of each species applied to k_j heat_j / c_v
    for (int j = threadIdx.x; j < nr; j += NT) ws[j] = n.heat ? ks[j] * n.heat[j] / th[0] : 0.0;
    __syncthreads();
    segsum_chunks<NT, LAYOUT_SELL, false, true>(n.gy, ws, ys, part, out + nnz + ns);
    __syncthreads();
    segsum_finish<NT, false>(n.gy, part, out + nnz + ns);
    const double corner = wg_sum<NT>(csum, red) / th[0] - th[2];
    if (threadIdx.x == 0) out[nnz + 2 * ns] = corner;
    __syncthreads();
  }
}

size_t thermal_lds_bytes(const DNet &n, bool jac) {
  int slots = n.jtail.n_slot > n.rhs.n_slot ? n.jtail.n_slot : n.rhs.n_slot;
  slots = slots > n.gy.n_slot ? slots : n.gy.n_slot;
  slots = slots > 1 ? slots : 1;
  return sizeof(double) * (size_t(n.ns + 1) + size_t(jac ? 2 : 1) * n.nr + slots);
}

static int thermal_grid(int64_t n_cells) {
  int dev = 0, cus = 0;
  hipGetDevice(&dev);
  hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  const int64_t g = int64_t(cus > 0 ? cus : 256) * 2;
  return int(n_cells < g ? n_cells : g);
}

hipError_t launch_rhs_thermal(const DNet &n, const double *la, int64_t n_cells, const double *y,
                              const double *cond, const double *therm, double *dydt,
                              hipStream_t st) {
  if (n_cells == 0) return hipSuccess;
  constexpr int NT = 512;
  const size_t lds = thermal_lds_bytes(n, false);
  if (lds > 65536) hipFuncSetAttribute(reinterpret_cast<const void *>(k_rhs_th<NT>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, int(lds));
  hipLaunchKernelGGL(k_rhs_th<NT>, dim3(thermal_grid(n_cells)), dim3(NT), lds, st, n, la, n_cells,
                     y, cond, therm, dydt);
  return hipGetLastError();
}

hipError_t launch_jac_thermal(const DNet &n, const double *la, int64_t n_cells, const double *y,
                              const double *cond, const double *therm, double *jvals,
                              hipStream_t st) {
  if (n_cells == 0) return hipSuccess;
  constexpr int NT = 512;
  const size_t lds = thermal_lds_bytes(n, true);
  if (lds > 65536) hipFuncSetAttribute(reinterpret_cast<const void *>(k_jac_th<NT>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, int(lds));
  hipLaunchKernelGGL(k_jac_th<NT>, dim3(thermal_grid(n_cells)), dim3(NT), lds, st, n, la, n_cells,
                     y, cond, therm, jvals);
  return hipGetLastError();
}

}  // namespace ac
