// Host-side plan of the integrator's Newton solve with a sparse front and
// a dense Schur tail.
//
// The Newton matrix M = I - c J has the pattern of the Jacobian plus the
// diagonal. DLSODES, the integrator of the paper (Sec. 3), solves with it
// through a sparse direct method under a minimum-degree order. Here the
// species that the minimum-degree order eliminates first (the front, n1 of
// them) couple to few others; eliminating them fills little. The rest (the
// tail, n2 species) fill in almost completely and are better served by a
// dense factorisation on the matrix cores.
//
// With the species permuted to positions (front first), M = [A B; C D].
// A Gauss-Jordan sweep over the front pivots turns it in place into
//   [A^-1, A^-1 B; -C A^-1, S],  S = D - C A^-1 B,
// and S is then factored densely with partial pivoting. Solves need one
// sparse product before and one after the dense solve with S:
//   M x = b:    z2 = S^-1 (b2 - C A^-1 b1),     z1 = A^-1 b1 - A^-1 B z2
//   M^T x = b:  z2 = S^-T (b2 - (A^-1 B)^T b1), z1 = A^-T b1 - (C A^-1)^T z2
// Pivots of the sweep are not exchanged (as in the Yale sparse package
// behind DLSODES); the front is chosen by structure only. Front pivots that
// share no entry at the time of their sweep are swept together, in levels.
#pragma once

#include <cstddef>
#include <cstdint>
#include <vector>

namespace ac {

struct FrontPlan {
  int n = 0;       // state size (species)
  int n1 = 0;      // front size
  int n2 = 0;      // tail size (dense Schur complement)
  int lda2 = 0;    // leading dimension of S (n2 rounded up to 16)
  int vofs = 0;    // offset (doubles) of the sparse values after S in the slot
  int nv = 0;      // sparse values (front rows and front columns of the swept matrix)
  int n_lev = 0;   // sweep levels
  std::vector<int32_t> perm;      // [n] position -> species
  std::vector<int32_t> lev_ptr;   // [n_lev + 1] front positions swept in each level
  // the sparse values in CSR over positions: front rows (A^-1 then A^-1 B
  // entries), tail rows (-C A^-1 entries), columns ascending
  std::vector<int32_t> row_ptr;   // [n + 1]
  std::vector<int32_t> col;       // [nv]
  std::vector<int32_t> rsplit;    // [n1] first entry of front row k with column >= n1
  std::vector<int32_t> vdiag;     // [n1] entry of (k, k)
  // the same entries by column: rows ascending, with their CSR index
  std::vector<int32_t> cptr;      // [n + 1]
  std::vector<int32_t> crow;      // [nv]
  std::vector<int32_t> cidx;      // [nv]
  std::vector<int32_t> csplit;    // [n1] first entry of front column k with row >= n1
  // destination of every Jacobian pattern entry (CSR order): a sparse value
  // index (>= 0) or -(1 + i2 * lda2 + j2) for S
  std::vector<int32_t> asm_dst;
  // sweep updates: per level the targets (same code as asm_dst), each with
  // its products (index of a_ik, index of a_kj), pivots in sweep order
  std::vector<int32_t> tg_ptr;    // [n_lev + 1]
  std::vector<int32_t> tgt;       // [n_tgt]
  std::vector<int32_t> op_ptr;    // [n_tgt + 1]
  std::vector<int32_t> ops;       // [2 n_op] pairs
  // The solves' four sparse products (forward before / after the dense
  // solve: rows over [row_ptr, rsplit) or the whole tail row, then front
  // rows over [rsplit, row_ptr+1); transposed: the same by column) cut into
  // pieces of at most FRONT_PIECE entries, so that long rows are summed by
  // several threads. Gather g: output position r owns pieces
  // gseg[g*(n+1) + r] .. gseg[g*(n+1) + r + 1] - 1; piece p covers entries
  // [gpc[2p], gpc[2p+1]) (CSR entries for the row gathers 0, 1, CSC
  // entries for the column gathers 2, 3); gbase[g] is its first piece.
  std::vector<int32_t> gseg;      // [4 (n + 1)]
  std::vector<int32_t> gpc;       // [2 n_piece]
  int gbase[5] = {0, 0, 0, 0, 0};
  double cost_front = 0.0, cost_dense = 0.0;   // modelled seconds per factorisation
  // Temperature-coupled state only (n = species + 1): destinations of the
  // temperature column (one per species), the temperature row and the
  // corner, coded as asm_dst (whose entries are the species pattern's).
  std::vector<int32_t> tcol_dst, trow_dst;
  int32_t corner_dst = 0;
};

constexpr int FRONT_PIECE = 16;
constexpr int FRONT_MAX_PIECES = 8192;   // partial sums per gather (doubles of LDS)

// Builds the plan for an n x n Jacobian pattern (CSR, natural order) whose
// Newton matrix region holds max_doubles doubles per slot.
FrontPlan build_front_plan(int n, const std::vector<int32_t> &j_row_ptr,
                           const std::vector<int32_t> &j_col, size_t max_doubles);

// The plan for the temperature-coupled state (ns species + T): the
// species pattern with a full temperature row and column.
FrontPlan build_front_plan_thermal(int ns, const std::vector<int32_t> &j_row_ptr,
                                   const std::vector<int32_t> &j_col, size_t max_doubles);

}  // namespace ac
