// Workgroup-level dense FP64 linear algebra for the Newton step of the
// implicit integrator: LU with partial pivoting (right-looking, 16-column
// panels, trailing update on the FP64 matrix cores) and the triangular
// solves A x = b and A^T x = b. One workgroup owns one matrix; matrices are
// row-major with leading dimension lda in global memory (L2-resident per
// slot), right-hand sides live in LDS.
#pragma once

#include <hip/hip_runtime.h>

#include <climits>
#include <cstdint>

namespace ac {

typedef double d4_t __attribute__((ext_vector_type(4)));

// Sum over the workgroup; every thread gets the same value (fixed tree).
template <int NT>
__device__ __forceinline__ double wg_sum(double v, double *red) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double s = red[0];
#pragma unroll
  for (int w = 1; w < NT / 64; ++w) s += red[w];
  __syncthreads();
  return s;
}

// Largest |value|, smallest index among ties; every thread gets the pair.
template <int NT>
__device__ __forceinline__ void wg_argmax(double &v, int &idx, double *red, int *redi) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const double ov = __shfl_xor(v, o);
    const int oi = __shfl_xor(idx, o);
    if (ov > v || (ov == v && oi < idx)) {
      v = ov;
      idx = oi;
    }
  }
  if ((threadIdx.x & 63) == 0) {
    red[threadIdx.x >> 6] = v;
    redi[threadIdx.x >> 6] = idx;
  }
  __syncthreads();
  v = red[0];
  idx = redi[0];
#pragma unroll
  for (int w = 1; w < NT / 64; ++w)
    if (red[w] > v || (red[w] == v && redi[w] < idx)) {
      v = red[w];
      idx = redi[w];
    }
  __syncthreads();
}

// A22 -= L21 U12 for the panel [k0, kend): 16x16 output tiles per wave,
// each the sum of ceil((kend-k0)/4) v_mfma_f64_16x16x4 products. Operand
// lanes: A[l%16][l/16], B[l/16][l%16]; result element v of lane l is row
// l/16 + 4v, column l%16.
template <int NT>
__device__ __forceinline__ void trailing_update(double *__restrict__ A, int lda, int n, int k0,
                                                int kend) {
  const int m = n - kend;
  if (m <= 0) return;
  const int nt = (m + 15) >> 4;
  const int lane = threadIdx.x & 63, li = lane & 15, lk = lane >> 4;
  for (int t = threadIdx.x >> 6; t < nt * nt; t += NT / 64) {
    const int ti = t / nt, tj = t - ti * nt;
    const int r0 = kend + 16 * ti, c0 = kend + 16 * tj;
    const int col = c0 + li;
    d4_t acc;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int row = r0 + lk + 4 * v;
      acc[v] = (row < n && col < n) ? A[size_t(row) * lda + col] : 0.0;
    }
    const int ar = r0 + li;
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) {
      const int kc = k0 + 4 * kk + lk;
      const double a = (ar < n && kc < kend) ? A[size_t(ar) * lda + kc] : 0.0;
      const double b = (kc < kend && col < n) ? A[size_t(kc) * lda + col] : 0.0;
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(-a, b, acc, 0, 0, 0);
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int row = r0 + lk + 4 * v;
      if (row < n && col < n) A[size_t(row) * lda + col] = acc[v];
    }
  }
}

// In-place P A = L U (unit lower L), piv[k] = row swapped with row k at
// step k (whole rows swapped). Returns 0 or 1 + the first zero pivot.
// red: >= NT/64 doubles, redi: >= NT/64 ints of LDS.
template <int NT>
__device__ int wg_lu(double *__restrict__ A, int lda, int n, int *__restrict__ piv, double *red,
                     int *redi) {
  int info = 0;
  for (int k0 = 0; k0 < n; k0 += 16) {
    const int kend = k0 + 16 < n ? k0 + 16 : n;
    for (int c = k0; c < kend; ++c) {
      double best = -1.0;
      int bi = INT_MAX;
      for (int i = c + threadIdx.x; i < n; i += NT) {
        const double v = fabs(A[size_t(i) * lda + c]);
        if (v > best) {
          best = v;
          bi = i;
        }
      }
      wg_argmax<NT>(best, bi, red, redi);
      const int p = best < 0.0 ? c : bi;
      if (threadIdx.x == 0) piv[c] = p;
      if (p != c)
        for (int j = threadIdx.x; j < n; j += NT) {
          const double t = A[size_t(c) * lda + j];
          A[size_t(c) * lda + j] = A[size_t(p) * lda + j];
          A[size_t(p) * lda + j] = t;
        }
      __syncthreads();
      const double pivot = A[size_t(c) * lda + c];
      if (pivot != 0.0) {
        const double *Ac = A + size_t(c) * lda;
        for (int i = c + 1 + threadIdx.x; i < n; i += NT) {
          double *Ai = A + size_t(i) * lda;
          const double l = Ai[c] / pivot;
          Ai[c] = l;
          for (int j = c + 1; j < kend; ++j) Ai[j] -= l * Ac[j];
        }
      } else if (!info) {
        info = c + 1;
      }
      __syncthreads();
    }
    // U12 = L11^{-1} A12, one column per thread
    for (int j = kend + threadIdx.x; j < n; j += NT)
      for (int r = k0 + 1; r < kend; ++r) {
        double s = A[size_t(r) * lda + j];
        for (int q = k0; q < r; ++q) s -= A[size_t(r) * lda + q] * A[size_t(q) * lda + j];
        A[size_t(r) * lda + j] = s;
      }
    __syncthreads();
    trailing_update<NT>(A, lda, n, k0, kend);
    __syncthreads();
  }
  return info;
}

// Solves with the factors of wg_lu: A x = b (trans = false) or A^T x = b.
// x (LDS) holds b on entry and x on return. The triangular solves run in
// blocks of SB rows: the diagonal block is staged in LDS (blk, SB*SB
// doubles) and solved by the first wavefront, then every thread updates
// the remaining rows with the block's solution.
constexpr int SB = 32;

template <int NT>
__device__ void wg_solve(const double *__restrict__ LU, int lda, int n,
                         const int *__restrict__ piv, double *x, bool trans, double *blk) {
  const int lane = threadIdx.x & 63;
  const bool w0 = threadIdx.x < 64;
  if (!trans) {
    if (threadIdx.x == 0)
      for (int k = 0; k < n; ++k) {
        const int p = piv[k];
        if (p != k) {
          const double t = x[k];
          x[k] = x[p];
          x[p] = t;
        }
      }
    __syncthreads();
    // L y = P b, L unit lower
    for (int b0 = 0; b0 < n; b0 += SB) {
      const int bs = b0 + SB < n ? SB : n - b0;
      for (int e = threadIdx.x; e < bs * bs; e += NT)
        blk[e] = LU[size_t(b0 + e / bs) * lda + b0 + e % bs];
      __syncthreads();
      if (w0) {
        double xr = lane < bs ? x[b0 + lane] : 0.0;
        for (int q = 0; q < bs - 1; ++q) {
          const double xq = __shfl(xr, q);
          if (lane > q && lane < bs) xr -= blk[lane * bs + q] * xq;
        }
        if (lane < bs) x[b0 + lane] = xr;
      }
      __syncthreads();
      for (int i = b0 + bs + threadIdx.x; i < n; i += NT) {
        const double *Li = LU + size_t(i) * lda + b0;
        double s = 0.0;
        for (int q = 0; q < bs; ++q) s += Li[q] * x[b0 + q];
        x[i] -= s;
      }
      __syncthreads();
    }
    // U x = y
    for (int bend = n; bend > 0; bend -= SB) {
      const int b0 = bend - SB > 0 ? bend - SB : 0, bs = bend - b0;
      for (int e = threadIdx.x; e < bs * bs; e += NT)
        blk[e] = LU[size_t(b0 + e / bs) * lda + b0 + e % bs];
      __syncthreads();
      if (w0) {
        double xr = lane < bs ? x[b0 + lane] : 0.0;
        for (int q = bs - 1; q >= 0; --q) {
          if (lane == q) xr = xr / blk[q * bs + q];
          const double xq = __shfl(xr, q);
          if (lane < q) xr -= blk[lane * bs + q] * xq;
        }
        if (lane < bs) x[b0 + lane] = xr;
      }
      __syncthreads();
      for (int i = threadIdx.x; i < b0; i += NT) {
        const double *Ui = LU + size_t(i) * lda + b0;
        double s = 0.0;
        for (int q = 0; q < bs; ++q) s += Ui[q] * x[b0 + q];
        x[i] -= s;
      }
      __syncthreads();
    }
  } else {
    // U^T z = b (lower, diagonal of U)
    for (int b0 = 0; b0 < n; b0 += SB) {
      const int bs = b0 + SB < n ? SB : n - b0;
      for (int e = threadIdx.x; e < bs * bs; e += NT)
        blk[e] = LU[size_t(b0 + e / bs) * lda + b0 + e % bs];
      __syncthreads();
      if (w0) {
        double xr = lane < bs ? x[b0 + lane] : 0.0;
        for (int q = 0; q < bs; ++q) {
          if (lane == q) xr = xr / blk[q * bs + q];
          const double xq = __shfl(xr, q);
          if (lane > q && lane < bs) xr -= blk[q * bs + lane] * xq;
        }
        if (lane < bs) x[b0 + lane] = xr;
      }
      __syncthreads();
      for (int i = b0 + bs + threadIdx.x; i < n; i += NT) {
        double s = 0.0;
        for (int q = 0; q < bs; ++q) s += LU[size_t(b0 + q) * lda + i] * x[b0 + q];
        x[i] -= s;
      }
      __syncthreads();
    }
    // L^T w = z (upper, unit diagonal)
    for (int bend = n; bend > 0; bend -= SB) {
      const int b0 = bend - SB > 0 ? bend - SB : 0, bs = bend - b0;
      for (int e = threadIdx.x; e < bs * bs; e += NT)
        blk[e] = LU[size_t(b0 + e / bs) * lda + b0 + e % bs];
      __syncthreads();
      if (w0) {
        double xr = lane < bs ? x[b0 + lane] : 0.0;
        for (int q = bs - 1; q > 0; --q) {
          const double xq = __shfl(xr, q);
          if (lane < q) xr -= blk[q * bs + lane] * xq;
        }
        if (lane < bs) x[b0 + lane] = xr;
      }
      __syncthreads();
      for (int i = threadIdx.x; i < b0; i += NT) {
        double s = 0.0;
        for (int q = 0; q < bs; ++q) s += LU[size_t(b0 + q) * lda + i] * x[b0 + q];
        x[i] -= s;
      }
      __syncthreads();
    }
    // x = P^T w: swaps in reverse order
    if (threadIdx.x == 0)
      for (int k = n - 1; k >= 0; --k) {
        const int p = piv[k];
        if (p != k) {
          const double t = x[k];
          x[k] = x[p];
          x[p] = t;
        }
      }
    __syncthreads();
  }
}

}  // namespace ac
