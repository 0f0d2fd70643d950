// Host-side network build: stoichiometry storage, traversal orders, the
// Jacobian pattern and the segmented-sum schedules the kernels walk.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "frontlu.h"

namespace ac {

// A packed term of a segmented sum: value = coef * A[j] * (b == NONE ? 1 : y[b]).
//   bits  0..15  j    (reaction, < 65536)
//   bits 16..26  b    (species, NONE = 2047)
//   bits 27..31  coef (two's complement, -16..15)
constexpr uint32_t ITEM_NONE = 2047u;
inline uint32_t pack_item(int j, int b, int coef) {
  return uint32_t(j) | (uint32_t(b < 0 ? ITEM_NONE : b) << 16) | (uint32_t(coef & 31) << 27);
}

// out[seg_out[s]] = sum of the items of segment s, for segments in
// traversal order. Segments are cut into chunks of at most `chunk` items
// (an empty segment gets one empty chunk); every layout visits the same
// items in the same order inside a chunk. A segment with one chunk is
// written straight from that chunk; the chunks of a longer segment leave
// partial sums in slots that a second pass adds in chunk order.
struct Schedule {
  int n_seg = 0, n_chunk = 0, n_item = 0, chunk = 0;
  std::vector<int32_t> seg_out;    // [n_seg] natural index of the s-th traversed segment
  std::vector<int32_t> seg_chunk;  // [n_seg+1] chunk range of segment s
  std::vector<int32_t> chunk_ptr;  // [n_chunk+1] item range of chunk (CSR order)
  std::vector<uint32_t> items;     // [n_item] CSR order
  std::vector<int32_t> chunk_dst;  // [n_chunk] >= 0: output index; < 0: partial slot -1-dst
  int n_slot = 0, n_multi = 0;
  std::vector<int32_t> multi_out;  // [n_multi] output index of a split segment
  std::vector<int32_t> multi_slot; // [n_multi+1] slot range (slots follow chunk order)
  // SELL-C-sigma over chunks
  int sell_c = 0, sell_sigma = 0, n_slice = 0;
  std::vector<int32_t> slice_ptr;  // [n_slice+1] offsets into sell_items
  std::vector<int32_t> sell_chunk; // [n_slice*sell_c] chunk id at a position, -1 = pad
  std::vector<int32_t> sell_len;   // [n_slice*sell_c] items of that chunk (0 for pads)
  std::vector<int32_t> sell_dst;   // [n_slice*sell_c] chunk_dst of that chunk (INT32_MIN for pads)
  std::vector<uint32_t> sell_items;
  // COO: output index of every item (CSR order)
  std::vector<int32_t> coo_out;
  // Runs: the CSR item list cut into equal runs of RUN_LEN items (items is
  // padded to a whole number of runs). run_mask bit k marks item k of the
  // run as the start of a partial sum (a new segment, or the run's first
  // item); partials are numbered run by run from run_slot[t]; segment s
  // (traversal order) owns the consecutive partials seg_run[2s] ..
  // seg_run[2s] + seg_run[2s+1] - 1.
  int n_run = 0, n_rslot = 0;
  // items of the runs, interleaved so that lane l of a 64-run block reads its
  // 16-byte word q at ((block * RUN_LEN / 4 + q) * 64 + l): a wave's loads
  // are contiguous
  std::vector<uint32_t> run_items;
  std::vector<uint32_t> run_mask;
  std::vector<int32_t> run_slot;   // [n_run]
  std::vector<int32_t> seg_run;    // [2 n_seg]
};

constexpr int RUN_LEN = 32;   // items per run (one 32-bit mask word)

struct HostNet {
  int ns = 0, nr = 0;
  // reaction data
  std::vector<double> log_alpha, beta, gamma;
  // rate law per reaction (AC_LAW_*), empty when every reaction follows the
  // modified Arrhenius law; the device records carry the law code and the
  // parameters in the form ln k = ln alpha + beta' ln(T/300) - gamma' X + Y
  // (see devchem.h rate_k)
  std::vector<int8_t> law;
  // energy released per reaction event (temperature-coupled mode), or empty
  std::vector<double> heat;
  std::vector<uint32_t> rpair;        // reactant a | b << 16, 0xFFFF = none
  // per reaction, in three planes of nr 16-byte words: (ln alpha, beta'),
  // (gamma', rpair, law), and the net column of S as up to 8 16-bit
  // (species | coef << 11) halves (0xFFFF = none)
  std::vector<uint32_t> rxpack;
  // S in CSR (natural rows, reactions ascending) and CCS (per reaction)
  std::vector<int32_t> s_row_ptr, s_col, s_val;
  std::vector<int32_t> s_col_ptr, s_row, s_cval;
  // Jacobian pattern, CSR natural rows / ascending columns
  std::vector<int32_t> j_row_ptr, j_col;
  std::vector<int32_t> perm;          // species traversal order
  Schedule rhs;                       // rows of S: items (j, NONE, S_ij)
  Schedule jac;                       // pattern entries: items (j, other reactant, S_ij*mult)
  // Two-tier Jacobian: per entry e (natural order) its first two terms
  // (PAD if absent) and a tail descriptor (first slot << 8 | number of
  // slots, 0 = no tail); the remaining terms of every entry form the
  // `jtail` schedule whose chunk partials land in those slots.
  std::vector<uint32_t> jhead0, jhead1, jtaildesc;
  std::vector<int32_t> jent_row;      // row of every pattern entry (columns: j_col)
  Schedule jtail;
  Schedule gy;                        // species a: items (j, other reactant, mult) over slots of a
  FrontPlan front;                    // the integrator's Newton solve (sparse front, dense tail)
  FrontPlan front_th;                 // the same for the temperature-coupled state
  int layout = 0, ordering = 0;
};

// Doubles of an integrator slot's Newton-matrix region: (ns + 1) rows
// (room for the temperature-coupled state) of lda = ns + 1 rounded up to 16.
inline int newton_lda(int ns) { return (ns + 1 + 15) / 16 * 16; }
inline size_t newton_region_doubles(int ns) { return size_t(ns + 1) * size_t(newton_lda(ns)); }

// Returns an empty string on success, else the reason (code in *code).
std::string build_network(int ns, int nr, const int32_t *reactants, const int32_t *products,
                          const double *alpha, const double *beta, const double *gamma,
                          const int8_t *law, const int8_t *composition, int n_elem,
                          bool check_balance, int layout, int ordering, int chunk, int sell_c,
                          int sell_sigma, HostNet &out, int *code);

// Species order by the chosen rule over the pattern of S (CSR rows).
std::vector<int32_t> species_order(int ns, const std::vector<int32_t> &row_ptr,
                                   const std::vector<int32_t> &col, int nr, int ordering);

// Schedule from per-segment item lists (natural index) and a traversal order.
void build_schedule(const std::vector<std::vector<uint32_t>> &seg_items,
                    const std::vector<int32_t> &order, int chunk, int sell_c, int sell_sigma,
                    Schedule &s);

}  // namespace ac
