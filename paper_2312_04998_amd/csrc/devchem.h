// Device helpers shared by the chemistry and integrator kernels: packed
// term evaluation, chunked gather sums over a schedule, reaction records.
#pragma once

#include <climits>

#include "devnet.h"

namespace ac {

constexpr int SELL_C = 64;     // slice width of every SELL schedule (one wavefront)
constexpr int UNROLL = 8;      // terms in flight per lane
constexpr uint32_t PAD_ITEM = 2047u << 16;   // coef 0, no density factor

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

// acc + one packed term. Schedules of S itself (no density factor, HASB =
// false) apply the coefficient inside a fused multiply-add: for the usual
// power-of-two coefficients coef * A[j] is exact, so this rounds exactly like
// the separate multiply and add, with two fewer instructions per term.
template <bool HASB>
__device__ __forceinline__ double term_add(double acc, uint32_t it, const double *__restrict__ A,
                                           const double *__restrict__ ys) {
  if (!HASB) return fma(double(int32_t(it) >> 27), A[it & 0xFFFFu], acc);
  return __dadd_rn(acc, term(it, A, ys));
}

template <bool STREAM>
__device__ __forceinline__ void put(double *p, double v) {
  if (STREAM) __builtin_nontemporal_store(v, p);
  else *p = v;
}

// Chunk sums of a schedule: single-chunk segments go straight to out,
// split segments leave partials in `part` for segsum_finish. Every chunk
// is summed left to right with the same operations in both layouts, so
// CSR and SELL give the same bits. SELL lanes of a slice loop to the slice
// width (wave-uniform) with UNROLL term loads issued before they are
// consumed; a slice position's length and destination are stored per
// position, so a wave reads them contiguously.
template <int NT, int LAYOUT, bool STREAM, bool HASB = true>
__device__ __forceinline__ void segsum_chunks(const DSched &s, const double *__restrict__ A,
                                              const double *__restrict__ ys, double *part,
                                              double *__restrict__ out) {
  if (LAYOUT == LAYOUT_SELL) {
    // SELL_P positions per lane at once, their descriptors, destinations
    // and items requested before any is used; a wave's 64 lanes share one
    // slice per position, so widths are wave-uniform. One position per
    // round measured fastest (more cost occupancy through registers).
    constexpr int SELL_P = 1;
    const int npos = s.n_slice * SELL_C;
    for (int pos0 = threadIdx.x; pos0 < npos; pos0 += SELL_P * NT) {
      int width[SELL_P], len[SELL_P], dst[SELL_P];
      const uint32_t *it[SELL_P];
#pragma unroll
      for (int p = 0; p < SELL_P; ++p) {
        const int pos = pos0 + p * NT;
        const bool ok = pos < npos;
        const int sl = ok ? pos / SELL_C : 0;
        const int base = ok ? s.slice_ptr[sl] : 0;
        width[p] = ok ? (s.slice_ptr[sl + 1] - base) / SELL_C : 0;
        len[p] = ok ? s.sell_len[pos] : 0;
        dst[p] = ok ? s.sell_dst[pos] : INT_MIN;
        it[p] = s.sell_items + base + (ok ? pos - sl * SELL_C : 0);
      }
      int wmax = 0;
#pragma unroll
      for (int p = 0; p < SELL_P; ++p) wmax = width[p] > wmax ? width[p] : wmax;
      double acc[SELL_P];
#pragma unroll
      for (int p = 0; p < SELL_P; ++p) acc[p] = 0.0;
      for (int k0 = 0; k0 < wmax; k0 += UNROLL) {
        uint32_t v[SELL_P][UNROLL];
#pragma unroll
        for (int p = 0; p < SELL_P; ++p)
#pragma unroll
          for (int u = 0; u < UNROLL; ++u)
            v[p][u] = (k0 + u < width[p]) ? it[p][(k0 + u) * SELL_C] : PAD_ITEM;
#pragma unroll
        for (int p = 0; p < SELL_P; ++p)
#pragma unroll
          for (int u = 0; u < UNROLL; ++u)
            if (k0 + u < len[p]) acc[p] = term_add<HASB>(acc[p], v[p][u], A, ys);
      }
#pragma unroll
      for (int p = 0; p < SELL_P; ++p) {
        const int d = dst[p];
        if (d == INT_MIN) continue;
        if (d >= 0) put<STREAM>(out + d, acc[p]);
        else part[-1 - d] = acc[p];
      }
    }
  } else {
    for (int ch = threadIdx.x; ch < s.n_chunk; ch += NT) {
      double acc = 0.0;
      const int p0 = s.chunk_ptr[ch], p1 = s.chunk_ptr[ch + 1];
      for (int k0 = p0; k0 < p1; k0 += UNROLL) {
        uint32_t v[UNROLL];
#pragma unroll
        for (int u = 0; u < UNROLL; ++u) v[u] = (k0 + u < p1) ? s.items[k0 + u] : PAD_ITEM;
#pragma unroll
        for (int u = 0; u < UNROLL; ++u)
          if (k0 + u < p1) acc = term_add<HASB>(acc, v[u], A, ys);
      }
      const int d = s.chunk_dst[ch];
      if (d >= 0) put<STREAM>(out + d, acc);
      else part[-1 - d] = acc;
    }
  }
}

// Equal-run partials: lane t sums the RUN_ITEMS items of run t left to
// right, closing a partial (into part, numbered from run_slot[t]) wherever
// the run's mask marks a new segment. All of a run's items are requested
// with eight 16-byte loads before any is used; runs are interleaved in
// blocks of 64, so each load of a wave reads 1 KB of contiguous memory.
template <int NT, bool HASB = true>
__device__ __forceinline__ void runsum_partials(const DSched &s, const double *__restrict__ A,
                                                const double *__restrict__ ys, double *part) {
  for (int t = threadIdx.x; t < s.n_run; t += NT) {
    const uint32_t mask = s.run_mask[t];
    int slot = s.run_slot[t];
    const int len = s.n_item - t * RUN_ITEMS < RUN_ITEMS ? s.n_item - t * RUN_ITEMS : RUN_ITEMS;
    const uint4 *it4 = s.run_items + size_t(t >> 6) * (RUN_ITEMS / 4) * 64 + (t & 63);
    uint4 w[RUN_ITEMS / 4];
#pragma unroll
    for (int q = 0; q < RUN_ITEMS / 4; ++q) w[q] = it4[q * 64];
    double acc = 0.0;
#pragma unroll
    for (int k = 0; k < RUN_ITEMS; ++k) {
      const uint4 &wq = w[k >> 2];
      const uint32_t it = (k & 3) == 0 ? wq.x : (k & 3) == 1 ? wq.y : (k & 3) == 2 ? wq.z : wq.w;
      if (k < len) {
        if (k > 0 && ((mask >> k) & 1u)) {
          part[slot++] = acc;
          acc = 0.0;
        }
        acc = term_add<HASB>(acc, it, A, ys);
      }
    }
    if (len > 0) part[slot] = acc;
  }
}

// One packed term for two cells whose values sit side by side in LDS:
// A2[j] = (A_j of cell 0, A_j of cell 1), y2[b] likewise, where y2[ynone]
// holds (1, 1) and stands for "no density factor" (b = NONE is clamped to
// ynone, every real species index is below it). acc += coef * (A_j y_b).
__device__ __forceinline__ void term_pair(uint32_t it, const double2 *__restrict__ A2,
                                          const double2 *__restrict__ y2, uint32_t ynone,
                                          double &acc0, double &acc1) {
  const uint32_t b = min((it >> 16) & 2047u, ynone);
  const double coef = double(int32_t(it) >> 27);
  const double2 kv = A2[it & 0xFFFFu], yv = y2[b];
  acc0 = fma(coef, kv.x * yv.x, acc0);
  acc1 = fma(coef, kv.y * yv.y, acc1);
}

// runsum_partials for two cells at once, over interleaved per-reaction
// values A2 and densities y2 (see term_pair); the partials of both cells
// go to part2[slot] as one pair. The run's mask, slot and items are loaded
// and decoded once for both cells, and every LDS access serves both.
template <int NT>
__device__ __forceinline__ void runsum_pairs(const DSched &s, const double2 *__restrict__ A2,
                                             const double2 *__restrict__ y2, uint32_t ynone,
                                             double2 *part2) {
  for (int t = threadIdx.x; t < s.n_run; t += NT) {
    const uint32_t mask = s.run_mask[t];
    int slot = s.run_slot[t];
    const int len = s.n_item - t * RUN_ITEMS < RUN_ITEMS ? s.n_item - t * RUN_ITEMS : RUN_ITEMS;
    const uint4 *it4 = s.run_items + size_t(t >> 6) * (RUN_ITEMS / 4) * 64 + (t & 63);
    uint4 w[RUN_ITEMS / 4];
#pragma unroll
    for (int q = 0; q < RUN_ITEMS / 4; ++q) w[q] = it4[q * 64];
    double acc0 = 0.0, acc1 = 0.0;
#pragma unroll
    for (int k = 0; k < RUN_ITEMS; ++k) {
      const uint4 &wq = w[k >> 2];
      const uint32_t it = (k & 3) == 0 ? wq.x : (k & 3) == 1 ? wq.y : (k & 3) == 2 ? wq.z : wq.w;
      if (k < len) {
        if (k > 0 && ((mask >> k) & 1u)) {
          part2[slot++] = make_double2(acc0, acc1);
          acc0 = 0.0;
          acc1 = 0.0;
        }
        term_pair(it, A2, y2, ynone, acc0, acc1);
      }
    }
    if (len > 0) part2[slot] = make_double2(acc0, acc1);
  }
}

// out[seg_out[k]] = sum of segment k's run partials, in order.
template <int NT, bool STREAM>
__device__ __forceinline__ void runsum_finish(const DSched &s, const double *part,
                                              double *__restrict__ out) {
  for (int k = threadIdx.x; k < s.n_seg; k += NT) {
    const int q0 = s.seg_run[2 * k], nq = s.seg_run[2 * k + 1];
    double acc = 0.0;
    for (int q = 0; q < nq; ++q) acc = __dadd_rn(acc, part[q0 + q]);
    put<STREAM>(out + s.seg_out[k], acc);
  }
}

// SELL sums for two cells at once, over interleaved per-reaction values
// A2[j] = (cell 0, cell 1): descriptors and items are loaded and decoded
// once and one LDS access serves both cells. Without a density factor
// (HASB = false: the rows of S) each chunk takes the same left-to-right
// fused multiply-adds as segsum_chunks, so the results are identical; with
// one, terms are term_pair's over the interleaved densities y2 (y2[ynone]
// = (1, 1)). Split segments leave pairs of partials in part2. out1 / the
// second cell may be absent (null).
template <int NT, bool HASB = false>
__device__ __forceinline__ void sell_pairs(const DSched &s, const double2 *__restrict__ A2,
                                           const double2 *__restrict__ y2, uint32_t ynone,
                                           double2 *part2, double *__restrict__ out0,
                                           double *__restrict__ out1) {
  const int npos = s.n_slice * SELL_C;
  for (int pos = threadIdx.x; pos < npos; pos += NT) {
    const int sl = pos / SELL_C;
    const int base = s.slice_ptr[sl];
    const int width = (s.slice_ptr[sl + 1] - base) / SELL_C;
    const int len = s.sell_len[pos];
    const int d = s.sell_dst[pos];
    const uint32_t *it = s.sell_items + base + (pos - sl * SELL_C);
    double acc0 = 0.0, acc1 = 0.0;
    for (int k0 = 0; k0 < width; k0 += UNROLL) {
      uint32_t v[UNROLL];
#pragma unroll
      for (int u = 0; u < UNROLL; ++u) v[u] = (k0 + u < width) ? it[(k0 + u) * SELL_C] : PAD_ITEM;
#pragma unroll
      for (int u = 0; u < UNROLL; ++u)
        if (k0 + u < len) {
          if (HASB) {
            term_pair(v[u], A2, y2, ynone, acc0, acc1);
          } else {
            const double coef = double(int32_t(v[u]) >> 27);
            const double2 a = A2[v[u] & 0xFFFFu];
            acc0 = fma(coef, a.x, acc0);
            acc1 = fma(coef, a.y, acc1);
          }
        }
    }
    if (d == INT_MIN) continue;
    if (d >= 0) {
      out0[d] = acc0;
      if (out1) out1[d] = acc1;
    } else {
      part2[-1 - d] = make_double2(acc0, acc1);
    }
  }
}

// segsum_finish for pairs of partials (out1 may be null).
template <int NT>
__device__ __forceinline__ void segsum_finish_pairs(const DSched &s, const double2 *part2,
                                                    double *__restrict__ out0,
                                                    double *__restrict__ out1) {
  for (int m = threadIdx.x; m < s.n_multi; m += NT) {
    const int q0 = s.multi_slot[m], q1 = s.multi_slot[m + 1];
    double2 acc = part2[q0];
    for (int q = q0 + 1; q < q1; ++q) {
      const double2 p = part2[q];
      acc.x = __dadd_rn(acc.x, p.x);
      acc.y = __dadd_rn(acc.y, p.y);
    }
    out0[s.multi_out[m]] = acc.x;
    if (out1) out1[s.multi_out[m]] = acc.y;
  }
}

template <int NT, bool STREAM>
__device__ __forceinline__ void segsum_finish(const DSched &s, const double *part,
                                              double *__restrict__ out) {
  for (int m = threadIdx.x; m < s.n_multi; m += NT) {
    const int q0 = s.multi_slot[m], q1 = s.multi_slot[m + 1];
    double acc = part[q0];
    for (int q = q0 + 1; q < q1; ++q) acc = __dadd_rn(acc, part[q]);
    put<STREAM>(out + s.multi_out[m], acc);
  }
}

// Full segmented sum (partials in LDS, so a barrier sits in between).
template <int NT, int LAYOUT, bool HASB = true>
__device__ __forceinline__ void segsum(const DSched &s, const double *A, const double *ys,
                                       double *part, double *out) {
  if (LAYOUT == LAYOUT_COO) {
    // scatter with LDS atomics into a per-cell accumulator (order varies)
    for (int i = threadIdx.x; i < s.n_seg; i += NT) part[i] = 0.0;
    __syncthreads();
    for (int p = threadIdx.x; p < s.n_item; p += NT)
      atomicAdd(&part[s.coo_out[p]], term_add<HASB>(0.0, s.items[p], A, ys));
    __syncthreads();
    for (int i = threadIdx.x; i < s.n_seg; i += NT) out[i] = part[i];
    return;
  }
  if (LAYOUT == LAYOUT_RUNS) {
    runsum_partials<NT, HASB>(s, A, ys, part);
    __syncthreads();
    runsum_finish<NT, false>(s, part, out);
    return;
  }
  segsum_chunks<NT, LAYOUT, false, HASB>(s, A, ys, part, out);
  __syncthreads();
  segsum_finish<NT, false>(s, part, out);
}

template <int NT>
__device__ __forceinline__ void load_cell(const double *__restrict__ src, double *dst, int n) {
  for (int i = threadIdx.x; i < n; i += NT) dst[i] = src[i];
}

// Reaction record: ln alpha, beta', gamma', reactant pair and rate law (two
// 16-byte loads); beta' and gamma' are the law's parameters in the form of
// rate_k.
struct Rx {
  double la, beta, gamma;
  uint32_t pair, law;
};

__device__ __forceinline__ Rx load_rx(const DNet &n, int j) {
  const uint4 a = n.rxpack[j], b = n.rxpack[n.nr + j];
  Rx r;
  r.la = __hiloint2double(int(a.y), int(a.x));
  r.beta = __hiloint2double(int(a.w), int(a.z));
  r.gamma = __hiloint2double(int(b.y), int(b.x));
  r.pair = b.z;
  r.law = b.w;
  return r;
}

// A cell's conditions in the form the rate laws use: L = ln(T/300),
// invT = 1/T and, when the network has rate laws, A_V, ln(zeta/zeta_0) and
// ln G_0.
struct Env {
  double L, invT, av, lnz, lng;
};

__device__ __forceinline__ Env env_of(const double *p, int nc) {
  Env e;
  const double Tc = p[0];
  e.L = log(Tc / 300.0);
  e.invT = 1.0 / Tc;
  if (nc > 1) {
    e.av = p[1];
    e.lnz = log(p[2]);
    e.lng = log(p[3]);
  } else {
    e.av = e.lnz = e.lng = 0.0;
  }
  return e;
}

__device__ __forceinline__ Env cell_env(const double *__restrict__ cond, int64_t c, int nc) {
  return env_of(cond + c * nc, nc);
}

// Conditions a cell's integration accepts: T > 0 and the others >= 0, all
// finite.
__device__ __forceinline__ bool cell_env_ok(const double *__restrict__ cond, int64_t c, int nc) {
  const double *p = cond + c * nc;
  bool ok = isfinite(p[0]) && p[0] > 0.0;
  for (int i = 1; i < nc; ++i) ok = ok && isfinite(p[i]) && p[i] >= 0.0;
  return ok;
}

// k_j = exp(ln alpha + beta' ln(T/300) - gamma' X + Y), with (X, Y) =
// (1/T, 0) for the modified Arrhenius law, (-, ln zeta) for direct
// cosmic-ray ionisation (beta' = gamma' = 0), (1, ln zeta) for cosmic-ray
// induced photons (gamma' = -ln(gamma / (1 - albedo))) and (A_V, ln G_0)
// for FUV photoreactions (beta' = 0).
__device__ __forceinline__ double rate_k(double la, double beta, double gamma, uint32_t law,
                                         const Env &e) {
  const double X = law == AC_LAW_PHOTO ? e.av : law == AC_LAW_CRPHOT ? 1.0 : e.invT;
  const double Y = law == AC_LAW_KOOIJ ? 0.0 : law == AC_LAW_PHOTO ? e.lng : e.lnz;
  return exp(la + beta * e.L - gamma * X + Y);
}

__device__ __forceinline__ double rate_k(const Rx &r, const Env &e) {
  return rate_k(r.la, r.beta, r.gamma, r.law, e);
}

// d ln k / dT of a record at 1/T: (beta + gamma/T)/T for the modified
// Arrhenius law, beta/T for cosmic-ray induced photons, 0 for the
// temperature-independent laws.
__device__ __forceinline__ double rate_dlnk_dT(const Rx &r, double invT) {
  return r.law == AC_LAW_KOOIJ ? (r.beta + r.gamma * invT) * invT
         : r.law == AC_LAW_CRPHOT ? r.beta * invT
                                  : 0.0;
}

// A cell's conditions with the temperature taken from the state (the
// temperature-coupled mode: cond[0] is not used).
__device__ __forceinline__ Env env_with_T(const double *p, int nc, double T) {
  Env e;
  e.L = log(T / 300.0);
  e.invT = 1.0 / T;
  if (nc > 1) {
    e.av = p[1];
    e.lnz = log(p[2]);
    e.lng = log(p[3]);
  } else {
    e.av = e.lnz = e.lng = 0.0;
  }
  return e;
}

__device__ __forceinline__ double reaction_rate(uint32_t pair, double k, const double *ys) {
  double r = k * ys[pair & 0xFFFFu];
  const uint32_t b = pair >> 16;
  if (b != 0xFFFFu) r *= ys[b];
  return r;
}

constexpr int RXU = 4;   // reaction records in flight per lane

// for_reactions with the reaction's record: fn(j, k_j, record).
template <int NT, typename F>
__device__ __forceinline__ void for_rx(const DNet &n, const double *__restrict__ la_over,
                                       const Env &env, F fn) {
  for (int j0 = threadIdx.x; j0 < n.nr; j0 += RXU * NT) {
    Rx r[RXU];
#pragma unroll
    for (int u = 0; u < RXU; ++u) {
      const int j = j0 + u * NT;
      if (j < n.nr) {
        r[u] = load_rx(n, j);
        if (la_over) r[u].la = la_over[j];
      }
    }
#pragma unroll
    for (int u = 0; u < RXU; ++u) {
      const int j = j0 + u * NT;
      if (j < n.nr) fn(j, rate_k(r[u], env), r[u]);
    }
  }
}

// For every reaction j of this thread (j = tid + m*NT), with RXU records
// loaded before any is used: fn(j, k_j, pair).
template <int NT, typename F>
__device__ __forceinline__ void for_reactions(const DNet &n, const double *__restrict__ la_over,
                                              const Env &env, F fn) {
  for (int j0 = threadIdx.x; j0 < n.nr; j0 += RXU * NT) {
    Rx r[RXU];
#pragma unroll
    for (int u = 0; u < RXU; ++u) {
      const int j = j0 + u * NT;
      if (j < n.nr) {
        r[u] = load_rx(n, j);
        if (la_over) r[u].la = la_over[j];
      }
    }
#pragma unroll
    for (int u = 0; u < RXU; ++u) {
      const int j = j0 + u * NT;
      if (j < n.nr) fn(j, rate_k(r[u], env), r[u].pair);
    }
  }
}

}  // namespace ac
