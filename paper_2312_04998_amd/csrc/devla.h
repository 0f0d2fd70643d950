// Workgroup-level dense FP64 linear algebra for the Newton step of the
// implicit integrator: LU with partial pivoting (right-looking, 16-column
// panels factored in LDS, row swaps outside the panel applied afterwards,
// trailing update on the FP64 matrix cores) and the triangular solves
// A x = b and A^T x = b. One workgroup owns one matrix; matrices are
// row-major with leading dimension lda in global memory, right-hand sides
// live in LDS. Every loop over matrix data keeps many independent loads in
// flight: a single workgroup per cell is latency-bound otherwise.
#pragma once

#include <hip/hip_runtime.h>

#include <climits>
#include <cstdint>

namespace ac {

typedef double d4_t __attribute__((ext_vector_type(4)));

constexpr int PW = 16;   // LU panel width
constexpr int LU_GROUP = 4;   // panels per trailing-matrix pass
constexpr int SB = 64;        // triangular-solve block
constexpr int SBP = SB + 1;   // its LDS row stride (odd: row-wise lane reads avoid bank conflicts)

// LDS the factorisation / solves need besides the right-hand side (doubles).
__host__ __device__ inline int la_scratch_doubles(int n) {
  const int pan = n * PW + PW * PW;
  const int blk = 3 * SB * SBP;   // the solves' two staged diagonal blocks and one off-diagonal
  return pan > blk ? pan : blk;
}

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

// Rank-16 updates of the region rows [R0, R1) x cols [C0, C1) of A by the
// nsrc full-width panels at columns K0, K0 + PW, ..., applied in that
// order: A -= L_s U_s, with U_s the panel's PW rows of A and L_s its
// columns below them, read from A, or for the last panel from the LDS panel
// `pan` when lds_last is set (row r - pk0 of pan is matrix row r). Each
// wave owns 32x32 blocks (2x2 tiles of 16x16), two at a time; every panel
// adds four v_mfma_f64_16x16x4 products (K = 16) per tile, so an element
// takes exactly the products, in the same order, as one update per panel
// would. Operand lanes: A[l%16][l/16], B[l/16][l%16]; result element v of
// lane l is row l/16 + 4v, column l%16.
struct RegionBlock {
  int r0, c0;
  d4_t acc[2][2];
  double bop[2][4];
};

__device__ __forceinline__ void rb_load(RegionBlock &B, const double *__restrict__ A, int lda,
                                        int R1, int C1) {
  const int lane = threadIdx.x & 63, li = lane & 15, lk = lane >> 4;
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      const int col = B.c0 + 16 * b + li;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = B.r0 + 16 * a + lk + 4 * v;
        B.acc[a][b][v] = (row < R1 && col < C1) ? A[size_t(row) * lda + col] : 0.0;
      }
    }
}

__device__ __forceinline__ void rb_load_u(RegionBlock &B, const double *__restrict__ A, int lda,
                                          int C1, int ks) {
  const int lane = threadIdx.x & 63, li = lane & 15, lk = lane >> 4;
#pragma unroll
  for (int b = 0; b < 2; ++b) {
    const int col = B.c0 + 16 * b + li;
#pragma unroll
    for (int kk = 0; kk < 4; ++kk)
      B.bop[b][kk] = col < C1 ? A[size_t(ks + 4 * kk + lk) * lda + col] : 0.0;
  }
}

__device__ __forceinline__ void rb_mfma(RegionBlock &B, const double *__restrict__ A, int lda,
                                        int R1, int ks, const double *pan, int pk0, bool lds) {
  const int lane = threadIdx.x & 63, li = lane & 15, lk = lane >> 4;
#pragma unroll
  for (int a = 0; a < 2; ++a) {
    const int row = B.r0 + 16 * a + li;   // row of the L operand
    const bool ok = row < R1;
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) {
      const int kc = 4 * kk + lk;
      double l = 0.0;
      if (ok) l = lds ? pan[(row - pk0) * PW + kc] : A[size_t(row) * lda + ks + kc];
#pragma unroll
      for (int b = 0; b < 2; ++b)
        B.acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(-l, B.bop[b][kk], B.acc[a][b], 0, 0, 0);
    }
  }
}

__device__ __forceinline__ void rb_store(const RegionBlock &B, double *__restrict__ A, int lda,
                                         int R1, int C1) {
  const int lane = threadIdx.x & 63, li = lane & 15, lk = lane >> 4;
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      const int col = B.c0 + 16 * b + li;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = B.r0 + 16 * a + lk + 4 * v;
        if (row < R1 && col < C1) A[size_t(row) * lda + col] = B.acc[a][b][v];
      }
    }
}

template <int NT>
__device__ __forceinline__ void region_update(double *__restrict__ A, int lda, int R0, int R1,
                                              int C0, int C1, int K0, int nsrc, const double *pan,
                                              int pk0, bool lds_last) {
  if (R1 <= R0 || C1 <= C0 || nsrc <= 0) return;
  const int nbc = (C1 - C0 + 31) >> 5, nblk = ((R1 - R0 + 31) >> 5) * nbc;
  constexpr int NW = NT / 64;
  for (int t = threadIdx.x >> 6; t < nblk; t += 2 * NW) {
    const bool two = t + NW < nblk;
    RegionBlock B0, B1;
    B0.r0 = R0 + 32 * (t / nbc);
    B0.c0 = C0 + 32 * (t % nbc);
    B1.r0 = R0 + 32 * ((t + NW) / nbc);
    B1.c0 = C0 + 32 * ((t + NW) % nbc);
    rb_load(B0, A, lda, R1, C1);
    if (two) rb_load(B1, A, lda, R1, C1);
    for (int s = 0; s < nsrc; ++s) {
      const int ks = K0 + PW * s;
      const bool lds = lds_last && s + 1 == nsrc;
      rb_load_u(B0, A, lda, C1, ks);
      if (two) rb_load_u(B1, A, lda, C1, ks);
      rb_mfma(B0, A, lda, R1, ks, pan, pk0, lds);
      if (two) rb_mfma(B1, A, lda, R1, ks, pan, pk0, lds);
    }
    rb_store(B0, A, lda, R1, C1);
    if (two) rb_store(B1, A, lda, R1, C1);
  }
}

// Value of lane `src` (wave-uniform) of a double, through scalar registers.
__device__ __forceinline__ double bcast(double v, int src) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), src);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), src);
  return __hiloint2double(hi, lo);
}

// Lane exchange through the DPP crossbar (no LDS round trip); CTRL is a
// full-wave data-parallel-primitive control code.
template <int CTRL>
__device__ __forceinline__ double dpp_d(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}

template <int CTRL>
__device__ __forceinline__ void argmax_step(double &v, int &idx) {
  const double ov = dpp_d<CTRL>(v);
  const int oi = __builtin_amdgcn_update_dpp(0, idx, CTRL, 0xF, 0xF, false);
  if (ov > v || (ov == v && oi < idx)) {
    v = ov;
    idx = oi;
  }
}

__device__ __forceinline__ void argmax_pick(double &v, int &idx, double ov, int oi) {
  if (ov > v || (ov == v && oi < idx)) {
    v = ov;
    idx = oi;
  }
}

// Pivot search over the workgroup: largest value, smallest index among
// ties; every thread gets the pair. Within a wave: quad swaps, then the
// half-row and row mirrors leave every 16-lane row with its row's best,
// and the four rows are combined through scalar registers. Leaves red/redi
// to be reused only after the caller's next barrier.
template <int NT>
__device__ __forceinline__ void wg_argmax_open(double &v, int &idx, double *red, int *redi) {
  argmax_step<0xB1>(v, idx);    // quad_perm [1,0,3,2]
  argmax_step<0x4E>(v, idx);    // quad_perm [2,3,0,1]
  argmax_step<0x141>(v, idx);   // row_half_mirror
  argmax_step<0x140>(v, idx);   // row_mirror
  double w = bcast(v, 0);
  int wi = __builtin_amdgcn_readlane(idx, 0);
  argmax_pick(w, wi, bcast(v, 16), __builtin_amdgcn_readlane(idx, 16));
  argmax_pick(w, wi, bcast(v, 32), __builtin_amdgcn_readlane(idx, 32));
  argmax_pick(w, wi, bcast(v, 48), __builtin_amdgcn_readlane(idx, 48));
  if ((threadIdx.x & 63) == 0) {
    red[threadIdx.x >> 6] = w;
    redi[threadIdx.x >> 6] = wi;
  }
  __syncthreads();
  v = red[0];
  idx = redi[0];
#pragma unroll
  for (int w2 = 1; w2 < NT / 64; ++w2) argmax_pick(v, idx, red[w2], redi[w2]);
}

// One column c of the panel factorisation (see panel_factor), unrolled
// at compile time so that the register-resident rows are indexed by
// constants only.
template <int NT, int R, int C>
struct PanelColumns {
  static __device__ __forceinline__ void run(double (&a)[R][PW], int (&lp)[R], int k0, int kw, int m,
                                             double *urow, double *red, int *redi, int *ipiv,
                                             int &info) {
    if (C < kw) {
      double best = -1.0;
      int bl = INT_MAX;
#pragma unroll
      for (int i = 0; i < R; ++i)
        if (lp[i] < m && lp[i] >= C) {
          const double v = fabs(a[i][C]);
          if (v > best || (v == best && lp[i] < bl)) {
            best = v;
            bl = lp[i];
          }
        }
      wg_argmax_open<NT>(best, bl, red, redi);
      const int L = best < 0.0 ? C : bl;
#pragma unroll
      for (int i = 0; i < R; ++i)
        if (lp[i] == L)
#pragma unroll
          for (int j = 0; j < PW; ++j) urow[j] = a[i][j];
      if (threadIdx.x == 0) ipiv[C] = L;
      __syncthreads();
      const double pivot = urow[C];
#pragma unroll
      for (int i = 0; i < R; ++i) {
        if (lp[i] == C)
          lp[i] = L;
        else if (lp[i] == L)
          lp[i] = C;
      }
      if (pivot != 0.0) {
#pragma unroll
        for (int i = 0; i < R; ++i)
          if (lp[i] > C && lp[i] < m) {
            const double l = a[i][C] / pivot;
            a[i][C] = l;
#pragma unroll
            for (int j = C + 1; j < PW; ++j) a[i][j] -= l * urow[j];
          }
      } else if (!info) {
        info = k0 + C + 1;
      }
      PanelColumns<NT, R, C + 1>::run(a, lp, k0, kw, m, urow, red, redi, ipiv, info);
    }
  }
};

template <int NT, int R>
struct PanelColumns<NT, R, PW> {
  static __device__ __forceinline__ void run(double (&)[R][PW], int (&)[R], int, int, int, double *,
                                             double *, int *, int *, int &) {}
};

// Factors the m x kw panel at (k0, k0) with partial pivoting. Thread t
// keeps panel rows t, t + NT, ... (R of them) in registers; row exchanges
// are not carried out but tracked: lp[i] is the current (logical) position
// of the thread's i-th row, so the pivot choice, the multipliers and the
// final order are those of the explicit-swap algorithm. Two barriers per
// column: one for the pivot search, one to publish the pivot row (urow, PW
// doubles of LDS). On return the factored panel is in LDS (`pan`, logical
// order) and in A, ipiv[c] is the logical row exchanged with row c, and
// mv holds the (destination, source) row moves the other columns need.
template <int NT, int R>
__device__ __forceinline__ void panel_factor(double *__restrict__ A, int lda, int k0, int kw, int m,
                                             double *pan, double *urow, double *red, int *redi,
                                             int *ipiv, int *mv, int &info) {
  double a[R][PW];
  int lp[R];
#pragma unroll
  for (int i = 0; i < R; ++i) {
    const int r = threadIdx.x + i * NT;
    lp[i] = r;
#pragma unroll
    for (int j = 0; j < PW; ++j)
      a[i][j] = (r < m && j < kw) ? A[size_t(k0 + r) * lda + k0 + j] : 0.0;
  }
  PanelColumns<NT, R, 0>::run(a, lp, k0, kw, m, urow, red, redi, ipiv, info);
#pragma unroll
  for (int i = 0; i < R; ++i) {
    const int r = threadIdx.x + i * NT;
    if (r < m) {
#pragma unroll
      for (int j = 0; j < PW; ++j) pan[lp[i] * PW + j] = a[i][j];
#pragma unroll
      for (int j = 0; j < PW; ++j)
        if (j < kw) A[size_t(k0 + lp[i]) * lda + k0 + j] = a[i][j];
      if (lp[i] != r) {
        const int s = atomicAdd(mv, 1);
        mv[2 + 2 * s] = lp[i];
        mv[3 + 2 * s] = r;
      }
    }
  }
}

// In-place P A = L U (unit lower L). piv[k] = row exchanged with row k at
// step k (LAPACK convention, whole rows); perm[i] = original row that ends
// up in row i (so P b = b[perm]). Returns 0 or 1 + the first zero pivot.
// n <= 2 * NT. pan: la_scratch_doubles(n) doubles of LDS; red/redi: NT/64
// entries; ipiv: 9*PW + 2 ints of LDS.
template <int NT>
__device__ __forceinline__ int wg_lu(double *__restrict__ A, int lda, int n, int *__restrict__ piv,
                                     int *__restrict__ perm, double *pan, double *red, int *redi,
                                     int *ipiv) {
  int info = 0;
  int *mv = ipiv + PW;                       // [2 + 4 * PW] ints: count, pad, (dst, src) pairs
  double *inv = pan + size_t(n) * PW;        // PW x PW: L11^{-1} (first PW doubles: pivot row)
  // Panels go in groups of LU_GROUP, so that the trailing matrix is read and
  // written once per group (rank-16 LU_GROUP updates): before a panel is
  // factored, the group's earlier panels update its columns; after its row
  // exchanges they update its U rows; once the group is complete, the rest
  // of the trailing matrix takes all of the group's updates in one pass.
  // Every element gets the same products in the same order as with one
  // update per panel. Panels of a group are full width except possibly the
  // matrix's last. K0: the group's first column; gi: its panels so far.
  int K0 = 0, gi = 0;
  for (int k0 = 0; k0 < n; k0 += PW) {
    const int kw = k0 + PW < n ? PW : n - k0;
    const int m = n - k0;
    // the group's earlier panels on this panel's columns
    region_update<NT>(A, lda, k0, n, k0, k0 + kw, K0, gi, pan, 0, false);
    if (threadIdx.x == 0) mv[0] = 0;
    __syncthreads();
    if (m <= NT)
      panel_factor<NT, 1>(A, lda, k0, kw, m, pan, inv, red, redi, ipiv, mv, info);
    else
      panel_factor<NT, 2>(A, lda, k0, kw, m, pan, inv, red, redi, ipiv, mv, info);
    if (threadIdx.x < kw) piv[k0 + threadIdx.x] = k0 + ipiv[threadIdx.x];
    __syncthreads();
    // the moved rows of every other column: each wave owns a tile of
    // nm rows x cw columns per round and issues all of the tile's loads
    // before its stores (a wave executes in order, so no barrier is needed)
    {
      const int nm = mv[0];
      if (nm > 0) {
        constexpr int MV_U = 8, NW = NT / 64;
        const int lgcw = 9 - (nm > 1 ? 32 - __clz(nm - 1) : 0);   // nm * cw <= 64 * MV_U
        const int cw = 1 << lgcw, ncol = n - kw;
        const int lane = threadIdx.x & 63;
        for (int c0 = (threadIdx.x >> 6) * cw; c0 < ncol; c0 += NW * cw) {
          double v[MV_U];
#pragma unroll
          for (int u = 0; u < MV_U; ++u) {
            const int e = lane + 64 * u, q = e >> lgcw, ci = c0 + (e & (cw - 1));
            const int col = ci < k0 ? ci : ci + kw;
            v[u] = (q < nm && ci < ncol) ? A[size_t(k0 + mv[3 + 2 * q]) * lda + col] : 0.0;
          }
#pragma unroll
          for (int u = 0; u < MV_U; ++u) {
            const int e = lane + 64 * u, q = e >> lgcw, ci = c0 + (e & (cw - 1));
            const int col = ci < k0 ? ci : ci + kw;
            if (q < nm && ci < ncol) A[size_t(k0 + mv[2 + 2 * q]) * lda + col] = v[u];
          }
        }
      }
    }
    const int kend = k0 + kw;
    if (gi > 0) {
      // the group's earlier panels on this panel's (exchanged) U rows
      __syncthreads();
      region_update<NT>(A, lda, k0, kend, kend, n, K0, gi, pan, 0, false);
    }
    // U12 = L11^{-1} A12 on the matrix cores: lane jc < PW forms column jc
    // of the inverse of the unit lower 16x16 L11 (identity beyond kw) in
    // registers, then every 16-column tile of A12 is one 16x16x16 product.
    if (threadIdx.x < PW) {
      const int jc = threadIdx.x;
      double col[PW];
#pragma unroll
      for (int r = 0; r < PW; ++r) {
        double v = r == jc ? 1.0 : 0.0;
        if (r < kw)
#pragma unroll
          for (int q = 0; q < r; ++q)
            if (q >= jc) v -= pan[r * PW + q] * col[q];
        col[r] = v;
      }
#pragma unroll
      for (int r = 0; r < PW; ++r) inv[r * PW + jc] = col[r];
    }
    __syncthreads();
    {
      const int mt = (n - kend + 15) >> 4;
      const int lane = threadIdx.x & 63, li = lane & 15, lk = lane >> 4;
      for (int t = threadIdx.x >> 6; t < mt; t += NT / 64) {
        const int col = kend + 16 * t + li;
        double bop[4];
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) {
          const int kc = 4 * kk + lk;
          bop[kk] = (kc < kw && col < n) ? A[size_t(k0 + kc) * lda + col] : 0.0;
        }
        d4_t acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int kk = 0; kk < 4; ++kk)
          acc = __builtin_amdgcn_mfma_f64_16x16x4f64(inv[li * PW + 4 * kk + lk], bop[kk], acc, 0, 0, 0);
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int r = lk + 4 * v;
          if (r < kw && col < n) A[size_t(k0 + r) * lda + col] = acc[v];
        }
      }
    }
    __syncthreads();
    if (++gi == LU_GROUP || kend >= n) {
      // the whole group on the rest of the trailing matrix (this panel's L
      // from LDS)
      region_update<NT>(A, lda, kend, n, kend, n, K0, gi, pan, k0, true);
      K0 = kend;
      gi = 0;
    }
    __syncthreads();
  }
  // permutation from the swap sequence (once per factorisation)
  if (threadIdx.x == 0) {
    int *pm = reinterpret_cast<int *>(pan);
    for (int i = 0; i < n; ++i) pm[i] = i;
    for (int k = 0; k < n; ++k) {
      const int p = piv[k];
      const int t = pm[k];
      pm[k] = pm[p];
      pm[p] = t;
    }
  }
  __syncthreads();
  if (perm)
    for (int i = threadIdx.x; i < n; i += NT) perm[i] = reinterpret_cast<int *>(pan)[i];
  __syncthreads();
  return info;
}

// Block of the triangular solves: rows [b0, b0+bs), the diagonal block
// staged in LDS (row stride SBP, zero beyond bs) and solved by the first
// wavefront (lane = row). In the chains below each step's operand comes
// from registers loaded 16 at a time, and the lane holding the newest
// unknown hands it to the others through a scalar register. stage_block
// runs on NTH threads, t = 0 .. NTH-1 being the caller's index among them.
template <int NTH>
__device__ __forceinline__ void stage_block(const double *LU, int lda, int b0, int bs, double *blk,
                                            int t) {
  constexpr int U = (SB * SB + NTH - 1) / NTH;   // every load of the block in flight at once
  double v[U];
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int e = t + u * NTH, r = e / SB, q = e - r * SB;
    v[u] = (e < SB * SB && r < bs && q < bs) ? LU[size_t(b0 + r) * lda + b0 + q] : 0.0;
  }
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int e = t + u * NTH, r = e / SB, q = e - r * SB;
    if (e < SB * SB) blk[r * SBP + q] = v[u];
  }
}

// out[i] -= sum_{q < bs} M(i, q) x[b0 + q] with M(i, q) = rowmajor ?
// LU[i][b0+q] : LU[b0+q][i], for i in [i0, i1), on NTH threads (t as in
// stage_block; NTH a multiple of 4, t = threadIdx.x - a multiple of 64).
// Row-major: four lanes share a row (interleaved columns, so a quad reads
// 32 contiguous bytes), reduced with shuffles. Column-major: one lane per
// row, so a wave reads contiguous rows. All 16 loads of a lane are in
// flight together. A row's sum depends only on its data, not on which
// threads form it.
template <int NTH, bool ROWMAJOR>
__device__ __forceinline__ void block_gemv(const double *LU, int lda, int b0, int bs, int i0, int i1,
                                           double *x, int t) {
  if constexpr (ROWMAJOR) {
    const int sub = t & 3;
    for (int base = i0; base < i1; base += NTH / 4) {
      const int i = base + (t >> 2);
      const bool ok = i < i1;
      double v[16];
#pragma unroll
      for (int u = 0; u < 16; ++u) {
        const int q = 4 * u + sub;
        v[u] = (ok && q < bs) ? LU[size_t(i) * lda + b0 + q] : 0.0;
      }
      double s = 0.0;
#pragma unroll
      for (int u = 0; u < 16; ++u) {
        const int q = 4 * u + sub;
        s += v[u] * (q < bs ? x[b0 + q] : 0.0);
      }
      s += __shfl_xor(s, 1);
      s += __shfl_xor(s, 2);
      if (ok && sub == 0) x[i] -= s;
    }
  } else {
    for (int i = i0 + t; i < i1; i += NTH) {
      double s = 0.0;
      for (int q0 = 0; q0 < bs; q0 += 16) {
        double v[16];
#pragma unroll
        for (int u = 0; u < 16; ++u)
          v[u] = q0 + u < bs ? LU[size_t(b0 + q0 + u) * lda + i] : 0.0;
#pragma unroll
        for (int u = 0; u < 16; ++u) s += v[u] * (q0 + u < bs ? x[b0 + q0 + u] : 0.0);
      }
      x[i] -= s;
    }
  }
}

// The off-diagonal block of the next step (rows [n0, n0 + ns) x columns
// [b0, b0 + bs) of M, M as in block_gemv) into LDS (row stride SBP), on NTH
// threads (t as in stage_block).
template <int NTH, bool ROWMAJOR>
__device__ __forceinline__ void stage_off(const double *LU, int lda, int b0, int bs, int n0, int ns,
                                          double *off, int t) {
  constexpr int U = (SB * SB + NTH - 1) / NTH;
  double v[U];
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int e = t + u * NTH;
    // row-major M: e walks rows of M; column-major: e walks rows of LU
    const int a = e / SB, q = e - a * SB;
    bool ok;
    if (ROWMAJOR) ok = e < SB * SB && a < ns && q < bs;
    else ok = e < SB * SB && a < bs && q < ns;
    v[u] = ok ? (ROWMAJOR ? LU[size_t(n0 + a) * lda + b0 + q] : LU[size_t(b0 + a) * lda + n0 + q])
              : 0.0;
  }
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int e = t + u * NTH;
    const int a = e / SB, q = e - a * SB;
    if (e < SB * SB) {
      if (ROWMAJOR) off[a * SBP + q] = v[u];
      else off[q * SBP + a] = v[u];
    }
  }
}

// block_gemv for the rows of the next step, from the staged off-diagonal
// block (row i - n0 of `off`), with the same per-row sums.
template <int NTH, bool ROWMAJOR>
__device__ __forceinline__ void off_gemv(const double *off, int b0, int bs, int n0, int ns, double *x,
                                         int t) {
  if constexpr (ROWMAJOR) {
    const int sub = t & 3;
    for (int base = 0; base < ns; base += NTH / 4) {
      const int a = base + (t >> 2);
      const bool ok = a < ns;
      double s = 0.0;
#pragma unroll
      for (int u = 0; u < 16; ++u) {
        const int q = 4 * u + sub;
        s += (ok && q < bs ? off[a * SBP + q] : 0.0) * (q < bs ? x[b0 + q] : 0.0);
      }
      s += __shfl_xor(s, 1);
      s += __shfl_xor(s, 2);
      if (ok && sub == 0) x[n0 + a] -= s;
    }
  } else {
    for (int a = t; a < ns; a += NTH) {
      double s = 0.0;
      for (int q0 = 0; q0 < bs; q0 += 16) {
#pragma unroll
        for (int u = 0; u < 16; ++u)
          s += (q0 + u < bs ? off[a * SBP + q0 + u] : 0.0) * (q0 + u < bs ? x[b0 + q0 + u] : 0.0);
      }
      x[n0 + a] -= s;
    }
  }
}

// The chains of the four triangular solves on a staged diagonal block
// (first wavefront only; x in LDS).
// L y = b on the block, L unit lower.
__device__ __forceinline__ void chain_l(const double *blk, int b0, int bs, double *x) {
  const int lane = threadIdx.x & 63;
  double xr = lane < bs ? x[b0 + lane] : 0.0;
  for (int q0 = 0; q0 < bs - 1; q0 += 16) {
    double o[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) o[u] = blk[lane * SBP + q0 + u];
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      if (q0 + u < bs - 1) {
        const double xq = bcast(xr, q0 + u);
        if (lane > q0 + u) xr -= o[u] * xq;
      }
    }
  }
  if (lane < bs) x[b0 + lane] = xr;
}

// U x = y on the block; the unknown of row q is scaled by 1/U(q,q), formed
// up front.
__device__ __forceinline__ void chain_u(const double *blk, int b0, int bs, double *x) {
  const int lane = threadIdx.x & 63;
  double xr = lane < bs ? x[b0 + lane] : 0.0;
  const double rd = lane < bs ? 1.0 / blk[lane * SBP + lane] : 0.0;
  for (int q1 = bs; q1 > 0; q1 -= 16) {   // steps q = q1-1 .. q1-16
    double o[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) o[u] = q1 - 1 - u >= 0 ? blk[lane * SBP + q1 - 1 - u] : 0.0;
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int q = q1 - 1 - u;
      if (q >= 0) {
        if (lane == q) xr *= rd;
        const double xq = bcast(xr, q);
        if (lane < q) xr -= o[u] * xq;
      }
    }
  }
  if (lane < bs) x[b0 + lane] = xr;
}

// U^T z = b on the block (lower, diagonal of U).
__device__ __forceinline__ void chain_ut(const double *blk, int b0, int bs, double *x) {
  const int lane = threadIdx.x & 63;
  double xr = lane < bs ? x[b0 + lane] : 0.0;
  const double rd = lane < bs ? 1.0 / blk[lane * SBP + lane] : 0.0;
  for (int q0 = 0; q0 < bs; q0 += 16) {
    double o[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) o[u] = blk[(q0 + u) * SBP + lane];
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int q = q0 + u;
      if (q < bs) {
        if (lane == q) xr *= rd;
        const double xq = bcast(xr, q);
        if (lane > q && lane < bs) xr -= o[u] * xq;
      }
    }
  }
  if (lane < bs) x[b0 + lane] = xr;
}

// L^T w = z on the block (upper, unit diagonal).
__device__ __forceinline__ void chain_lt(const double *blk, int b0, int bs, double *x) {
  const int lane = threadIdx.x & 63;
  double xr = lane < bs ? x[b0 + lane] : 0.0;
  for (int q1 = bs; q1 > 1; q1 -= 16) {   // steps q = q1-1 .. max(1, q1-16)
    double o[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) o[u] = q1 - 1 - u >= 1 ? blk[(q1 - 1 - u) * SBP + lane] : 0.0;
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int q = q1 - 1 - u;
      if (q >= 1) {
        const double xq = bcast(xr, q);
        if (lane < q) xr -= o[u] * xq;
      }
    }
  }
  if (lane < bs) x[b0 + lane] = xr;
}

// One blocked triangular solve, forward (FWD: blocks from the top) or
// backward, with a one-block look-ahead: while the first wavefront runs the
// chain of block k, the other wavefronts stage block k+1 and the block of
// block k's columns on block k+1's rows, and apply block k-1's columns to
// the rows beyond block k; then the whole workgroup applies block k's
// columns to the rows of block k+1 (the only rows the next chain needs)
// from LDS. Every row receives the blocks' contributions in the same
// order, each summed the same way, as without the look-ahead.
// blk: 3 * SB * SBP doubles of LDS.
template <int NT, bool ROWMAJOR, bool FWD, int CHAIN>
__device__ __forceinline__ void tri_solve(const double *__restrict__ LU, int lda, int n, double *x,
                                          double *blk) {
  static_assert(NT >= 128 && NT % 64 == 0, "the look-ahead needs at least two wavefronts");
  const int nb = (n + SB - 1) / SB;
  auto b0_of = [&](int k) { return FWD ? k * SB : (n - (k + 1) * SB > 0 ? n - (k + 1) * SB : 0); };
  auto bs_of = [&](int k) {
    return FWD ? (k * SB + SB < n ? SB : n - k * SB) : n - k * SB - b0_of(k);
  };
  stage_block<NT>(LU, lda, b0_of(0), bs_of(0), blk, threadIdx.x);
  __syncthreads();
  for (int k = 0; k < nb; ++k) {
    const int b0 = b0_of(k), bs = bs_of(k);
    double *cur = blk + (k & 1) * (SB * SBP);
    if (threadIdx.x < 64) {
      if (CHAIN == 0) chain_l(cur, b0, bs, x);
      else if (CHAIN == 1) chain_u(cur, b0, bs, x);
      else if (CHAIN == 2) chain_ut(cur, b0, bs, x);
      else chain_lt(cur, b0, bs, x);
    } else {
      const int t = threadIdx.x - 64;
      if (k + 1 < nb) {
        stage_block<NT - 64>(LU, lda, b0_of(k + 1), bs_of(k + 1),
                             blk + ((k + 1) & 1) * (SB * SBP), t);
        stage_off<NT - 64, ROWMAJOR>(LU, lda, b0, bs, b0_of(k + 1), bs_of(k + 1),
                                     blk + 2 * (SB * SBP), t);
      }
      if (k >= 1) {
        // block k-1's columns, rows beyond block k
        const int p0 = b0_of(k - 1), ps = bs_of(k - 1);
        if (FWD) block_gemv<NT - 64, ROWMAJOR>(LU, lda, p0, ps, b0 + bs, n, x, t);
        else block_gemv<NT - 64, ROWMAJOR>(LU, lda, p0, ps, 0, b0, x, t);
      }
    }
    __syncthreads();
    if (k + 1 < nb) {
      // block k's columns, rows of block k+1, from the staged block
      const int n0 = b0_of(k + 1), ns_ = bs_of(k + 1);
      off_gemv<NT, ROWMAJOR>(blk + 2 * (SB * SBP), b0, bs, n0, ns_, x, threadIdx.x);
      __syncthreads();
    }
  }
}

// Solves with the factors of wg_lu: A x = b (trans = false) or A^T x = b.
// x (LDS, n doubles) holds b on entry and x on return; tmp (LDS, n
// doubles) is scratch; blk: 3 * SB * SBP doubles of LDS.
template <int NT>
__device__ __forceinline__ void wg_solve(const double *__restrict__ LU, int lda, int n,
                         const int *__restrict__ perm, double *x, double *tmp, bool trans,
                         double *blk) {
  if (!trans) {
    for (int i = threadIdx.x; i < n; i += NT) tmp[i] = x[perm[i]];
    __syncthreads();
    for (int i = threadIdx.x; i < n; i += NT) x[i] = tmp[i];
    tri_solve<NT, true, true, 0>(LU, lda, n, x, blk);    // L y = P b (its first barrier
                                                          // also orders the copy above)
    tri_solve<NT, true, false, 1>(LU, lda, n, x, blk);   // U x = y
  } else {
    tri_solve<NT, false, true, 2>(LU, lda, n, x, blk);   // U^T z = b
    tri_solve<NT, false, false, 3>(LU, lda, n, x, blk);  // L^T w = z
    // x = P^T w: x[perm[i]] = w[i]
    for (int i = threadIdx.x; i < n; i += NT) tmp[perm[i]] = x[i];
    __syncthreads();
    for (int i = threadIdx.x; i < n; i += NT) x[i] = tmp[i];
  }
  __syncthreads();
}

}  // namespace ac
