// C ABI of libastrochem.so: argument checks, network upload, launches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/astrochem.h"
#include "devbdf.h"
#include "devla.h"
#include "devnet.h"
#include "netbuild.h"

struct ac_net {
  ac::HostNet host;
  ac::DNet d{};
  void *dbuf = nullptr;
  double *vjp_part = nullptr;   // [vjp_rows][n_reactions] per-workgroup partial sums
  int vjp_rows = 0;
  int device = 0;
};

namespace {

thread_local std::string g_err;

ac_status fail(ac_status s, const std::string &msg) {
  g_err = msg;
  return s;
}

ac_status hip_fail(hipError_t e, const char *what) {
  g_err = std::string(what) + ": " + hipGetErrorString(e);
  return AC_EHIP;
}

// Packs host vectors into one device allocation (256-byte aligned pieces).
struct Packer {
  struct Piece { const void *src; size_t bytes; size_t off; };
  std::vector<Piece> pieces;
  size_t total = 0;
  template <typename T>
  size_t add(const std::vector<T> &v) {
    size_t off = total;
    pieces.push_back({v.data(), v.size() * sizeof(T), off});
    total += (v.size() * sizeof(T) + 255) / 256 * 256;
    if (v.empty()) total += 256;
    return off;
  }
};

template <typename T>
const T *at(void *base, size_t off) {
  return reinterpret_cast<const T *>(static_cast<char *>(base) + off);
}

struct SchedOff {
  size_t seg_out, seg_chunk, chunk_ptr, chunk_dst, multi_out, multi_slot, items, slice_ptr,
      sell_chunk, sell_len, sell_dst, sell_items, coo_out, run_items, run_mask, run_slot, seg_run;
};

static_assert(ac::RUN_LEN == ac::RUN_ITEMS, "host and device run lengths differ");
static_assert(ac::FRONT_MAX_PIECES <= 3 * ac::SB * ac::SBP,
              "the front gathers' partial sums must fit the solves' LDS block");

SchedOff add_sched(Packer &p, const ac::Schedule &s) {
  SchedOff o;
  o.seg_out = p.add(s.seg_out);
  o.seg_chunk = p.add(s.seg_chunk);
  o.chunk_ptr = p.add(s.chunk_ptr);
  o.chunk_dst = p.add(s.chunk_dst);
  o.multi_out = p.add(s.multi_out);
  o.multi_slot = p.add(s.multi_slot);
  o.items = p.add(s.items);
  o.slice_ptr = p.add(s.slice_ptr);
  o.sell_chunk = p.add(s.sell_chunk);
  o.sell_len = p.add(s.sell_len);
  o.sell_dst = p.add(s.sell_dst);
  o.sell_items = p.add(s.sell_items);
  o.coo_out = p.add(s.coo_out);
  o.run_items = p.add(s.run_items);
  o.run_mask = p.add(s.run_mask);
  o.run_slot = p.add(s.run_slot);
  o.seg_run = p.add(s.seg_run);
  return o;
}

ac::DSched dev_sched(void *b, const ac::Schedule &s, const SchedOff &o) {
  ac::DSched d{};
  d.n_seg = s.n_seg;
  d.n_chunk = s.n_chunk;
  d.n_item = s.n_item;
  d.n_slot = s.n_slot;
  d.n_multi = s.n_multi;
  d.seg_out = at<int32_t>(b, o.seg_out);
  d.seg_chunk = at<int32_t>(b, o.seg_chunk);
  d.chunk_ptr = at<int32_t>(b, o.chunk_ptr);
  d.chunk_dst = at<int32_t>(b, o.chunk_dst);
  d.multi_out = at<int32_t>(b, o.multi_out);
  d.multi_slot = at<int32_t>(b, o.multi_slot);
  d.items = at<uint32_t>(b, o.items);
  d.sell_c = s.sell_c;
  d.n_slice = s.n_slice;
  d.slice_ptr = at<int32_t>(b, o.slice_ptr);
  d.sell_chunk = at<int32_t>(b, o.sell_chunk);
  d.sell_len = at<int32_t>(b, o.sell_len);
  d.sell_dst = at<int32_t>(b, o.sell_dst);
  d.sell_items = at<uint32_t>(b, o.sell_items);
  d.coo_out = at<int32_t>(b, o.coo_out);
  d.n_run = s.n_run;
  d.n_rslot = s.n_rslot;
  d.run_items = at<uint4>(b, o.run_items);
  d.run_mask = at<uint32_t>(b, o.run_mask);
  d.run_slot = at<int32_t>(b, o.run_slot);
  d.seg_run = at<int32_t>(b, o.seg_run);
  return d;
}

constexpr int VJP_ROWS = 512;   // fixed VJP grid: the cell-to-workgroup map never changes

}  // namespace

extern "C" {

const char *ac_status_string(ac_status s) {
  switch (s) {
    case AC_OK: return "ok";
    case AC_EINVAL: return "invalid argument";
    case AC_ENOMEM: return "out of memory";
    case AC_EHIP: return "HIP runtime error";
    case AC_EUNBALANCED: return "reaction does not conserve elements/charge";
    case AC_ECAPACITY: return "workspace capacity exceeded";
    case AC_ELIMIT: return "network exceeds a compiled limit";
  }
  return "unknown status";
}

int ac_last_error(char *buf, size_t n) {
  if (buf && n) {
    size_t m = std::min(n - 1, g_err.size());
    std::memcpy(buf, g_err.data(), m);
    buf[m] = 0;
  }
  return int(g_err.size());
}

ac_status ac_net_create(const ac_net_desc *desc, ac_net **out) {
  if (!desc || !out) return fail(AC_EINVAL, "null argument");
  *out = nullptr;
  if (desc->block != 0 && desc->block != 256 && desc->block != 512 && desc->block != 1024)
    return fail(AC_EINVAL, "block must be 0, 256, 512 or 1024");
  ac_net *net = new (std::nothrow) ac_net();
  if (!net) return fail(AC_ENOMEM, "host allocation failed");
  int code = 0;
  std::string err;
  try {
    err = ac::build_network(desc->n_species, desc->n_reactions, desc->reactants, desc->products,
                            desc->alpha, desc->beta, desc->gamma, desc->rate_law,
                            desc->composition, desc->n_elem,
                            desc->check_balance != 0, desc->layout, desc->ordering, desc->chunk,
                            desc->sell_c, desc->sell_sigma, net->host, &code);
  } catch (const std::bad_alloc &) {
    delete net;
    return fail(AC_ENOMEM, "host allocation failed during network build");
  }
  if (!err.empty()) {
    delete net;
    return fail(ac_status(code), err);
  }
  if (desc->heat) {
    for (int j = 0; j < desc->n_reactions; ++j)
      if (!std::isfinite(desc->heat[j])) {
        delete net;
        return fail(AC_EINVAL, "reaction " + std::to_string(j) + ": heat must be finite");
      }
    net->host.heat.assign(desc->heat, desc->heat + desc->n_reactions);
  }
  const ac::HostNet &H = net->host;
  Packer p;
  const size_t o_la = p.add(H.log_alpha), o_be = p.add(H.beta), o_ga = p.add(H.gamma);
  const size_t o_rp = p.add(H.rpair), o_rx = p.add(H.rxpack);
  const size_t o_cp = p.add(H.s_col_ptr), o_cr = p.add(H.s_row), o_cv = p.add(H.s_cval);
  const SchedOff o_rhs = add_sched(p, H.rhs), o_jac = add_sched(p, H.jac), o_gy = add_sched(p, H.gy);
  const SchedOff o_jt = add_sched(p, H.jtail);
  const size_t o_h0 = p.add(H.jhead0), o_h1 = p.add(H.jhead1), o_td = p.add(H.jtaildesc);
  const size_t o_er = p.add(H.jent_row), o_ec = p.add(H.j_col);
  const size_t o_ht = p.add(H.heat);
  struct FrontOff {
    size_t perm, lev, rp, col, rs, dg, cp, cr, ci, cs, asmd, tgp, tg, opp, ops, gs, gp, tc, tr;
  };
  auto add_front = [&](const ac::FrontPlan &FP) {
    FrontOff o;
    o.perm = p.add(FP.perm);
    o.lev = p.add(FP.lev_ptr);
    o.rp = p.add(FP.row_ptr);
    o.col = p.add(FP.col);
    o.rs = p.add(FP.rsplit);
    o.dg = p.add(FP.vdiag);
    o.cp = p.add(FP.cptr);
    o.cr = p.add(FP.crow);
    o.ci = p.add(FP.cidx);
    o.cs = p.add(FP.csplit);
    o.asmd = p.add(FP.asm_dst);
    o.tgp = p.add(FP.tg_ptr);
    o.tg = p.add(FP.tgt);
    o.opp = p.add(FP.op_ptr);
    o.ops = p.add(FP.ops);
    o.gs = p.add(FP.gseg);
    o.gp = p.add(FP.gpc);
    o.tc = p.add(FP.tcol_dst);
    o.tr = p.add(FP.trow_dst);
    return o;
  };
  const FrontOff o_fr = add_front(H.front), o_frth = add_front(H.front_th);
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) {
    (void)hipGetLastError();
    *out = net;   // host-only handle: queries work, kernels report AC_EHIP
    return AC_OK;
  }
  hipGetDevice(&net->device);
  hipError_t e = hipMalloc(&net->dbuf, p.total);
  if (e != hipSuccess) {
    delete net;
    return hip_fail(e, "hipMalloc(network)");
  }
  std::vector<char> staging(p.total, 0);
  for (auto &pc : p.pieces)
    if (pc.bytes) std::memcpy(staging.data() + pc.off, pc.src, pc.bytes);
  e = hipMemcpy(net->dbuf, staging.data(), p.total, hipMemcpyHostToDevice);
  if (e == hipSuccess) {
    net->vjp_rows = VJP_ROWS;
    e = hipMalloc(&net->vjp_part, sizeof(double) * size_t(VJP_ROWS) * H.nr);
  }
  if (e != hipSuccess) {
    hipFree(net->dbuf);
    delete net;
    return hip_fail(e, "network upload");
  }
  void *b = net->dbuf;
  ac::DNet &d = net->d;
  d.ns = H.ns;
  d.nr = H.nr;
  d.nnz_j = int(H.j_col.size());
  d.layout = H.layout;
  d.block = desc->block;   // 0: chosen per kernel from its LDS size
  d.n_cond = H.law.empty() ? 1 : AC_NCOND;
  d.log_alpha = at<double>(b, o_la);
  d.beta = at<double>(b, o_be);
  d.gamma = at<double>(b, o_ga);
  d.rpair = at<uint32_t>(b, o_rp);
  d.rxpack = at<uint4>(b, o_rx);
  d.s_col_ptr = at<int32_t>(b, o_cp);
  d.s_row = at<int32_t>(b, o_cr);
  d.s_cval = at<int32_t>(b, o_cv);
  d.rhs = dev_sched(b, H.rhs, o_rhs);
  d.jac = dev_sched(b, H.jac, o_jac);
  d.gy = dev_sched(b, H.gy, o_gy);
  d.jtail = dev_sched(b, H.jtail, o_jt);
  d.jhead0 = at<uint32_t>(b, o_h0);
  d.jhead1 = at<uint32_t>(b, o_h1);
  d.jtaildesc = at<uint32_t>(b, o_td);
  d.jent_row = at<int32_t>(b, o_er);
  d.jent_col = at<int32_t>(b, o_ec);
  d.heat = H.heat.empty() ? nullptr : at<double>(b, o_ht);
  auto dev_front = [&](const ac::FrontPlan &FP, const FrontOff &o) {
    ac::DFront f{};
    f.n = FP.n;
    f.n1 = FP.n1;
    f.n2 = FP.n2;
    f.lda2 = FP.lda2;
    f.vofs = FP.vofs;
    f.nv = FP.nv;
    f.n_lev = FP.n_lev;
    f.perm = at<int32_t>(b, o.perm);
    f.lev_ptr = at<int32_t>(b, o.lev);
    f.row_ptr = at<int32_t>(b, o.rp);
    f.col = at<int32_t>(b, o.col);
    f.rsplit = at<int32_t>(b, o.rs);
    f.vdiag = at<int32_t>(b, o.dg);
    f.cptr = at<int32_t>(b, o.cp);
    f.crow = at<int32_t>(b, o.cr);
    f.cidx = at<int32_t>(b, o.ci);
    f.csplit = at<int32_t>(b, o.cs);
    f.asm_dst = at<int32_t>(b, o.asmd);
    f.tg_ptr = at<int32_t>(b, o.tgp);
    f.tgt = at<int32_t>(b, o.tg);
    f.op_ptr = at<int32_t>(b, o.opp);
    f.ops = at<int2>(b, o.ops);
    f.gseg = at<int32_t>(b, o.gs);
    f.gpc = at<int2>(b, o.gp);
    for (int g = 0; g < 5; ++g) f.gbase[g] = FP.gbase[g];
    f.tcol_dst = FP.tcol_dst.empty() ? nullptr : at<int32_t>(b, o.tc);
    f.trow_dst = FP.trow_dst.empty() ? nullptr : at<int32_t>(b, o.tr);
    f.corner_dst = FP.corner_dst;
    return f;
  };
  d.fr = dev_front(H.front, o_fr);
  d.fr_th = dev_front(H.front_th, o_frth);
  *out = net;
  return AC_OK;
}

ac_status ac_net_destroy(ac_net *net) {
  if (!net) return AC_OK;
  hipFree(net->dbuf);
  hipFree(net->vjp_part);
  delete net;
  return AC_OK;
}

ac_status ac_net_info(const ac_net *net, int64_t *nnz_s, int64_t *nnz_j, int64_t *n_contrib,
                      int64_t *n_chunks) {
  if (!net) return fail(AC_EINVAL, "null network");
  if (nnz_s) *nnz_s = int64_t(net->host.s_col.size());
  if (nnz_j) *nnz_j = int64_t(net->host.j_col.size());
  if (n_contrib) *n_contrib = int64_t(net->host.jac.n_item);
  if (n_chunks) *n_chunks = int64_t(net->host.rhs.n_chunk);
  return AC_OK;
}

ac_status ac_net_stoich(const ac_net *net, int32_t *row_ptr, int32_t *reaction, int32_t *value) {
  if (!net || !row_ptr || !reaction || !value) return fail(AC_EINVAL, "null argument");
  const auto &H = net->host;
  std::copy(H.s_row_ptr.begin(), H.s_row_ptr.end(), row_ptr);
  std::copy(H.s_col.begin(), H.s_col.end(), reaction);
  std::copy(H.s_val.begin(), H.s_val.end(), value);
  return AC_OK;
}

ac_status ac_net_jac_pattern(const ac_net *net, int32_t *row_ptr, int32_t *col) {
  if (!net || !row_ptr || !col) return fail(AC_EINVAL, "null argument");
  std::copy(net->host.j_row_ptr.begin(), net->host.j_row_ptr.end(), row_ptr);
  std::copy(net->host.j_col.begin(), net->host.j_col.end(), col);
  return AC_OK;
}

ac_status ac_net_row_order(const ac_net *net, int32_t *perm) {
  if (!net || !perm) return fail(AC_EINVAL, "null argument");
  std::copy(net->host.perm.begin(), net->host.perm.end(), perm);
  return AC_OK;
}

ac_status ac_net_front_info(const ac_net *net, int32_t *n_front, int32_t *n_levels,
                            int64_t *n_values, int64_t *n_updates, double *cost_ratio,
                            int32_t *order) {
  if (!net) return fail(AC_EINVAL, "null network");
  const ac::FrontPlan &F = net->host.front;
  if (n_front) *n_front = F.n1;
  if (n_levels) *n_levels = F.n_lev;
  if (n_values) *n_values = F.nv;
  if (n_updates) *n_updates = int64_t(F.ops.size() / 2);
  if (cost_ratio) *cost_ratio = F.cost_dense > 0.0 ? F.cost_front / F.cost_dense : 1.0;
  if (order) std::copy(F.perm.begin(), F.perm.end(), order);
  return AC_OK;
}

ac_status ac_sparse_format(int32_t n_rows, int32_t n_cols, const int32_t *dense, int32_t fmt,
                           int32_t width, int64_t *n_val, int32_t *val, int32_t *idx,
                           int32_t *idx2, int32_t *ptr) {
  if (n_rows <= 0 || n_cols <= 0 || !dense || !n_val || !val || !idx || !ptr)
    return fail(AC_EINVAL, "null or empty argument");
  std::vector<int32_t> v, ix, ix2, pt;
  auto A = [&](int i, int j) { return dense[size_t(i) * n_cols + j]; };
  if (fmt == AC_FMT_COO || fmt == AC_FMT_CRS) {
    if (fmt == AC_FMT_CRS) pt.push_back(0);
    for (int i = 0; i < n_rows; ++i) {
      for (int j = 0; j < n_cols; ++j)
        if (A(i, j)) {
          v.push_back(A(i, j));
          ix.push_back(j);
          ix2.push_back(i);
        }
      if (fmt == AC_FMT_CRS) pt.push_back(int32_t(v.size()));
    }
    if (fmt == AC_FMT_COO && !idx2) return fail(AC_EINVAL, "COO needs idx2");
  } else if (fmt == AC_FMT_CCS) {
    pt.push_back(0);
    for (int j = 0; j < n_cols; ++j) {
      for (int i = 0; i < n_rows; ++i)
        if (A(i, j)) {
          v.push_back(A(i, j));
          ix.push_back(i);
        }
      pt.push_back(int32_t(v.size()));
    }
  } else if (fmt == AC_FMT_SELL) {
    if (width <= 0) return fail(AC_EINVAL, "SELL needs a positive width");
    // one chunk per row (no splitting), no sorting: the schedule builder
    // with chunk = n_cols and sigma = 1
    std::vector<std::vector<uint32_t>> seg(n_rows);
    std::vector<std::vector<int>> vals(n_rows);
    for (int i = 0; i < n_rows; ++i)
      for (int j = 0; j < n_cols; ++j)
        if (A(i, j)) {
          seg[i].push_back(uint32_t(j));
          vals[i].push_back(A(i, j));
        }
    std::vector<int32_t> order(n_rows);
    for (int i = 0; i < n_rows; ++i) order[i] = i;
    ac::Schedule s;
    ac::build_schedule(seg, order, std::max(1, n_cols), width, 1, s);
    for (int sl = 0; sl < s.n_slice; ++sl) {
      const int w = (s.slice_ptr[sl + 1] - s.slice_ptr[sl]) / width;
      pt.push_back(w);
      for (int k = 0; k < w; ++k)
        for (int l = 0; l < width; ++l) {
          const int p = sl * width + l;
          const int row = p < n_rows ? s.sell_chunk[p] : -1;
          if (row >= 0 && k < int(vals[row].size())) {
            v.push_back(vals[row][k]);
            ix.push_back(int32_t(seg[row][k]));
          } else {
            // padding: value 0 with a valid column (the row's last one)
            v.push_back(0);
            ix.push_back(row >= 0 && !seg[row].empty() ? int32_t(seg[row].back()) : 0);
          }
        }
    }
  } else {
    return fail(AC_EINVAL, "unknown format");
  }
  if (int64_t(v.size()) > *n_val) {
    *n_val = int64_t(v.size());
    return fail(AC_EINVAL, "output capacity too small");
  }
  *n_val = int64_t(v.size());
  std::copy(v.begin(), v.end(), val);
  std::copy(ix.begin(), ix.end(), idx);
  if (fmt == AC_FMT_COO) std::copy(ix2.begin(), ix2.end(), idx2);
  std::copy(pt.begin(), pt.end(), ptr);
  return AC_OK;
}

// ----------------------------------------------------------------- kernels

static ac_status check_cells(const ac_net *net, int64_t n_cells) {
  if (!net) return fail(AC_EINVAL, "null network");
  if (n_cells < 0) return fail(AC_EINVAL, "n_cells < 0");
  if (!net->dbuf) return fail(AC_EHIP, "network has no device copy (no GPU at creation)");
  return AC_OK;
}

ac_status ac_rates(const ac_net *net, const double *log_alpha, int64_t n_cells, const double *T,
                   double *k, ac_stream stream) {
  if (ac_status s = check_cells(net, n_cells)) return s;
  if (n_cells && (!T || !k)) return fail(AC_EINVAL, "null T or k");
  hipError_t e = ac::launch_rates(net->d, log_alpha, n_cells, T, k, hipStream_t(stream));
  return e == hipSuccess ? AC_OK : hip_fail(e, "ac_rates launch");
}

ac_status ac_rhs(const ac_net *net, const double *log_alpha, int64_t n_cells, const double *y,
                 const double *T, double *dydt, ac_stream stream) {
  if (ac_status s = check_cells(net, n_cells)) return s;
  if (n_cells && (!y || !T || !dydt)) return fail(AC_EINVAL, "null y, T or dydt");
  hipError_t e = ac::launch_rhs(net->d, log_alpha, n_cells, y, T, nullptr, dydt, hipStream_t(stream));
  return e == hipSuccess ? AC_OK : hip_fail(e, "ac_rhs launch");
}

ac_status ac_rhs_k(const ac_net *net, int64_t n_cells, const double *k, const double *y,
                   double *dydt, ac_stream stream) {
  if (ac_status s = check_cells(net, n_cells)) return s;
  if (n_cells && (!k || !y || !dydt)) return fail(AC_EINVAL, "null k, y or dydt");
  hipError_t e = ac::launch_rhs(net->d, nullptr, n_cells, y, nullptr, k, dydt, hipStream_t(stream));
  return e == hipSuccess ? AC_OK : hip_fail(e, "ac_rhs_k launch");
}

ac_status ac_jac(const ac_net *net, const double *log_alpha, int64_t n_cells, const double *y,
                 const double *T, double *jvals, ac_stream stream) {
  if (ac_status s = check_cells(net, n_cells)) return s;
  if (n_cells && (!y || !T || !jvals)) return fail(AC_EINVAL, "null y, T or jvals");
  hipError_t e = ac::launch_jac(net->d, log_alpha, n_cells, y, T, jvals, hipStream_t(stream));
  return e == hipSuccess ? AC_OK : hip_fail(e, "ac_jac launch");
}

ac_status ac_rhs_jac(const ac_net *net, const double *log_alpha, int64_t n_cells,
                     const double *y, const double *T, double *dydt, double *jvals,
                     ac_stream stream) {
  if (ac_status s = check_cells(net, n_cells)) return s;
  if (n_cells && (!y || !T || !dydt || !jvals)) return fail(AC_EINVAL, "null y, T, dydt or jvals");
  hipError_t e = ac::launch_rhs_jac(net->d, log_alpha, n_cells, y, T, dydt, jvals,
                                    hipStream_t(stream));
  return e == hipSuccess ? AC_OK : hip_fail(e, "ac_rhs_jac launch");
}

ac_status ac_vjp(const ac_net *net, const double *log_alpha, int64_t n_cells, const double *y,
                 const double *T, const double *v, double *gy, double *g_logalpha,
                 ac_stream stream) {
  if (ac_status s = check_cells(net, n_cells)) return s;
  if (n_cells && (!y || !T || !v)) return fail(AC_EINVAL, "null y, T or v");
  hipError_t e = ac::launch_vjp(net->d, log_alpha, n_cells, y, T, v, gy, g_logalpha,
                                net->vjp_part, net->vjp_rows, hipStream_t(stream));
  return e == hipSuccess ? AC_OK : hip_fail(e, "ac_vjp launch");
}

ac_status ac_vjp_static(const ac_net *net, const double *log_alpha, int64_t n_cells,
                        const double *y, const double *T, const double *v, double *gy,
                        double *g_logalpha, ac_stream stream) {
  if (ac_status s = check_cells(net, n_cells)) return s;
  if (n_cells && (!y || !T || !v)) return fail(AC_EINVAL, "null y, T or v");
  double *part = nullptr;
  if (g_logalpha) {
    if (net->d.nr > ac::VJP_STATIC_NR)
      return fail(AC_ELIMIT, "ac_vjp_static: the library's scratch holds partial sums of at most " +
                                 std::to_string(ac::VJP_STATIC_NR) + " reactions");
    hipError_t e = ac::vjp_static_scratch(&part);
    if (e != hipSuccess) return hip_fail(e, "ac_vjp_static scratch lookup");
  }
  static_assert(ac::VJP_STATIC_ROWS == VJP_ROWS, "same fixed grid as ac_vjp");
  hipError_t e = ac::launch_vjp(net->d, log_alpha, n_cells, y, T, v, gy, g_logalpha, part,
                                ac::VJP_STATIC_ROWS, hipStream_t(stream));
  return e == hipSuccess ? AC_OK : hip_fail(e, "ac_vjp_static launch");
}

static ac_status thermal_args(const ac_net *net, int64_t n_cells, const double *y,
                              const double *T, const double *therm) {
  if (ac_status s = check_cells(net, n_cells)) return s;
  if (n_cells && (!y || !T || !therm)) return fail(AC_EINVAL, "null y, T or therm");
  return AC_OK;
}

ac_status ac_rhs_thermal(const ac_net *net, const double *log_alpha, int64_t n_cells,
                         const double *y, const double *T, const double *therm, double *dydt,
                         ac_stream stream) {
  if (ac_status s = thermal_args(net, n_cells, y, T, therm)) return s;
  if (n_cells && !dydt) return fail(AC_EINVAL, "null dydt");
  hipError_t e = ac::launch_rhs_thermal(net->d, log_alpha, n_cells, y, T, therm, dydt,
                                        hipStream_t(stream));
  return e == hipSuccess ? AC_OK : hip_fail(e, "ac_rhs_thermal launch");
}

ac_status ac_jac_thermal(const ac_net *net, const double *log_alpha, int64_t n_cells,
                         const double *y, const double *T, const double *therm, double *jvals,
                         ac_stream stream) {
  if (ac_status s = thermal_args(net, n_cells, y, T, therm)) return s;
  if (n_cells && !jvals) return fail(AC_EINVAL, "null jvals");
  hipError_t e = ac::launch_jac_thermal(net->d, log_alpha, n_cells, y, T, therm, jvals,
                                        hipStream_t(stream));
  return e == hipSuccess ? AC_OK : hip_fail(e, "ac_jac_thermal launch");
}

// ---------------------------------------------------------- dense LU

ac_status ac_lu_factor(int32_t n, int32_t lda, int64_t n_mat, double *A, int32_t *piv,
                       int32_t *info, ac_stream stream) {
  if (n <= 0 || lda < n || n_mat < 0) return fail(AC_EINVAL, "need n > 0, lda >= n, n_mat >= 0");
  if (n_mat && (!A || !piv)) return fail(AC_EINVAL, "null A or piv");
  if (n > 2 * ac::BDF_NT || sizeof(double) * (size_t(n) * 16 + 256) > 160 * 1024)
    return fail(AC_ELIMIT, "n too large for a workgroup-resident LU panel (n <= 1024)");
  hipError_t e = ac::launch_lu_factor(n, lda, n_mat, A, piv, info, hipStream_t(stream));
  return e == hipSuccess ? AC_OK : hip_fail(e, "ac_lu_factor launch");
}

ac_status ac_lu_solve(int32_t n, int32_t lda, int64_t n_mat, const double *LU,
                      const int32_t *piv, double *b, int32_t trans, ac_stream stream) {
  if (n <= 0 || lda < n || n_mat < 0) return fail(AC_EINVAL, "need n > 0, lda >= n, n_mat >= 0");
  if (n_mat && (!LU || !piv || !b)) return fail(AC_EINVAL, "null LU, piv or b");
  if (sizeof(double) * (size_t(2) * n + 2 * ac::SB * ac::SBP) + sizeof(int) * size_t(n) > 160 * 1024)
    return fail(AC_ELIMIT, "n too large for an LDS-resident right-hand side");
  hipError_t e = ac::launch_lu_solve(n, lda, n_mat, LU, piv, b, trans, hipStream_t(stream));
  return e == hipSuccess ? AC_OK : hip_fail(e, "ac_lu_solve launch");
}

}  // extern "C"

// ---------------------------------------------------------- integrator

struct ac_ws {
  const ac_net *net = nullptr;
  int n_slots = 0;
  size_t bytes = 0;
  void *buf = nullptr;
  unsigned *queue = nullptr;
  ac::WsView W{};
  void *adj_buf = nullptr;   // adjoint slots (ac_ws_reserve_adjoint)
  size_t adj_bytes = 0;
  ac::AdjView A{};
  int adj_tape = 0;          // longest tape the reserved slots hold (0: no adjoint capacity)
  double *rows = nullptr;    // [max_cells][n_reactions] per-cell dL/dlog alpha rows
  int max_cells = 0;
  unsigned *host_count = nullptr;   // pinned word the integrator writes its progress to
};

extern "C" {

ac_status ac_ws_create(const ac_net *net, int32_t n_slots, ac_ws **out) {
  if (!net || !out) return fail(AC_EINVAL, "null argument");
  *out = nullptr;
  if (!net->dbuf) return fail(AC_EHIP, "network has no device copy (no GPU at creation)");
  if (n_slots < 0) return fail(AC_EINVAL, "n_slots < 0");
  if (net->d.ns + 1 > 2 * ac::BDF_NT || ac::bdf_lds_bytes(net->d) > 160 * 1024)
    return fail(AC_ELIMIT, "network too large for the integrator's LDS working set");
  const int resident = ac::bdf_resident_blocks(net->d);
  ac_ws *ws = new (std::nothrow) ac_ws();
  if (!ws) return fail(AC_ENOMEM, "host allocation failed");
  ws->net = net;
  ws->n_slots = n_slots ? n_slots : resident;
  // every slot has room for the temperature-coupled state (ns + 1 values):
  // Newton matrix, Jacobian pattern values plus its T column, T row and
  // corner, difference array, pivots and permutation
  const int ns = net->d.ns, nv = ns + 1, nr = net->d.nr, nnz = net->d.nnz_j;
  const int lda = ac::newton_lda(ns);
  auto r256 = [](size_t b) { return (b + 255) / 256 * 256; };
  // also holds the Schur tail and the swept front values (the plan is
  // sized to this region)
  const size_t m_b = r256(sizeof(double) * ac::newton_region_doubles(ns));
  const size_t j_b = r256(sizeof(double) * (size_t(nnz) + 2 * size_t(ns) + 1));
  const size_t t_b = r256(sizeof(double) * size_t(std::max(1, net->host.jtail.n_slot)));
  const size_t d_b = r256(sizeof(double) * size_t(8) * nv);
  const size_t k_b = r256(sizeof(double) * size_t(nr));
  const size_t p_b = r256(sizeof(int) * size_t(2 * nv));
  const size_t per = m_b + j_b + t_b + d_b + k_b + p_b;
  ws->bytes = per * size_t(ws->n_slots) + 256;
  hipError_t e = hipMalloc(&ws->buf, ws->bytes);
  if (e != hipSuccess) {
    delete ws;
    return hip_fail(e, "hipMalloc(workspace)");
  }
  char *b = static_cast<char *>(ws->buf);
  const size_t S = size_t(ws->n_slots);
  ac::WsView &W = ws->W;
  W.M = reinterpret_cast<double *>(b);
  b += m_b * S;
  W.J = reinterpret_cast<double *>(b);
  b += j_b * S;
  W.tail = reinterpret_cast<double *>(b);
  b += t_b * S;
  W.D = reinterpret_cast<double *>(b);
  b += d_b * S;
  W.k = reinterpret_cast<double *>(b);
  b += k_b * S;
  W.piv = reinterpret_cast<int *>(b);
  b += p_b * S;
  ws->queue = reinterpret_cast<unsigned *>(b);
  W.m_stride = m_b / sizeof(double);
  W.j_stride = j_b / sizeof(double);
  W.tail_stride = t_b / sizeof(double);
  W.d_stride = d_b / sizeof(double);
  W.k_stride = k_b / sizeof(double);
  W.piv_stride = p_b / sizeof(int);
  W.lda = lda;
  // Debug aid: ASTROCHEM_POISON_WS=1 fills the floating-point slot regions
  // with NaN so any read of state a cell did not write itself shows up.
  const char *poison = std::getenv("ASTROCHEM_POISON_WS");
  if (poison && poison[0] == '1') {
    const size_t fp_bytes = (m_b + j_b + t_b + d_b + k_b) * S;
    e = hipMemset(ws->buf, 0xFF, fp_bytes);
    if (e == hipSuccess) e = hipMemset(W.piv, 0, p_b * S);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) {
      hipFree(ws->buf);
      delete ws;
      return hip_fail(e, "workspace poison fill");
    }
  }
  // the pinned host word the integrator reports its progress to
  e = hipHostMalloc(reinterpret_cast<void **>(&ws->host_count), sizeof(unsigned));
  void *dp = nullptr;
  if (e == hipSuccess) {
    *ws->host_count = 0u;
    e = hipHostGetDevicePointer(&dp, ws->host_count, 0);
  }
  if (e != hipSuccess) {
    if (ws->host_count) hipHostFree(ws->host_count);
    hipFree(ws->buf);
    delete ws;
    return hip_fail(e, "workspace progress word");
  }
  ws->W.progress = static_cast<unsigned *>(dp);
  *out = ws;
  return AC_OK;
}

ac_status ac_ws_destroy(ac_ws *ws) {
  if (!ws) return AC_OK;
  if (ws->adj_buf) hipFree(ws->adj_buf);
  if (ws->rows) hipFree(ws->rows);
  if (ws->host_count) hipHostFree(ws->host_count);
  hipFree(ws->buf);
  delete ws;
  return AC_OK;
}

ac_status ac_ws_progress(ac_ws *ws, int64_t *cells_taken) {
  if (!ws || !cells_taken) return fail(AC_EINVAL, "null argument");
  // written by the running kernel (system-scope stores); no GPU call here
  *cells_taken = int64_t(*static_cast<volatile unsigned *>(ws->host_count));
  return AC_OK;
}

ac_status ac_ws_info(const ac_ws *ws, int32_t *n_slots, int64_t *bytes) {
  if (!ws) return fail(AC_EINVAL, "null workspace");
  if (n_slots) *n_slots = ws->n_slots;
  if (bytes) *bytes = int64_t(ws->bytes + ws->adj_bytes);
  return AC_OK;
}

static ac_status integ_args(ac_ws *ws, int64_t n_cells, const double *y, const double *T,
                            double t_end, const ac_integ_opts *o) {
  if (!ws || !o) return fail(AC_EINVAL, "null workspace or options");
  if (n_cells < 0) return fail(AC_EINVAL, "n_cells < 0");
  if (n_cells && (!y || !T)) return fail(AC_EINVAL, "null y or T");
  if (!(o->rtol > 0.0) || !(o->atol >= 0.0)) return fail(AC_EINVAL, "need rtol > 0, atol >= 0");
  if (o->q_max < 1 || o->q_max > 5) return fail(AC_EINVAL, "q_max must be 1..5");
  if (o->max_steps < 1) return fail(AC_EINVAL, "max_steps must be >= 1");
  if (!(t_end >= 0.0) || !std::isfinite(t_end)) return fail(AC_EINVAL, "t_end must be finite and >= 0");
  if (o->linear_solver != AC_LINSOLVE_AUTO && o->linear_solver != AC_LINSOLVE_DENSE)
    return fail(AC_EINVAL, "linear_solver must be AC_LINSOLVE_AUTO or AC_LINSOLVE_DENSE");
  return AC_OK;
}

static ac::BdfParams bdf_params(const ac_integ_opts *o, double t_end) {
  ac::BdfParams P{o->rtol, o->atol, o->h0, t_end, o->q_max, o->max_steps, o->newton_tol};
  P.linear_solver = o->linear_solver;
  return P;
}

ac_status ac_integrate(ac_ws *ws, const double *log_alpha, int64_t n_cells, double *y,
                       const double *T, double t_end, const ac_integ_opts *opts,
                       int32_t *cell_status, int32_t *cell_stats, ac_event *tape,
                       int32_t tape_cap, int32_t *tape_len, ac_stream stream) {
  if (ac_status s = integ_args(ws, n_cells, y, T, t_end, opts)) return s;
  if (tape && (tape_cap <= 0 || !tape_len)) return fail(AC_EINVAL, "tape needs tape_cap > 0 and tape_len");
  ac::BdfParams P = bdf_params(opts, t_end);
  P.order = opts->cell_order;
  ac::CellOut out{cell_status, cell_stats};
  ac::TapeView tv{reinterpret_cast<ac::AcEvent *>(tape), tape ? tape_len : nullptr, tape ? tape_cap : 0};
  hipError_t e = ac::launch_bdf(ws->net->d, log_alpha, n_cells, y, T, nullptr, P, out, tv, ws->W,
                                ws->queue,
                                ws->n_slots, hipStream_t(stream));
  return e == hipSuccess ? AC_OK : hip_fail(e, "ac_integrate launch");
}

ac_status ac_integrate_thermal(ac_ws *ws, const double *log_alpha, int64_t n_cells, double *y,
                               const double *T, const double *therm, double t_end,
                               const ac_integ_opts *opts, int32_t *cell_status,
                               int32_t *cell_stats, ac_stream stream) {
  if (ac_status s = integ_args(ws, n_cells, y, T, t_end, opts)) return s;
  if (n_cells && !therm) return fail(AC_EINVAL, "null therm");
  ac::BdfParams P = bdf_params(opts, t_end);
  P.order = opts->cell_order;
  ac::CellOut out{cell_status, cell_stats};
  ac::TapeView tv{nullptr, nullptr, 0};
  hipError_t e = ac::launch_bdf(ws->net->d, log_alpha, n_cells, y, T, therm, P, out, tv, ws->W,
                                ws->queue, ws->n_slots, hipStream_t(stream));
  return e == hipSuccess ? AC_OK : hip_fail(e, "ac_integrate_thermal launch");
}

ac_status ac_integrate_plain(ac_ws *ws, const double *log_alpha, int64_t n_cells, double *y,
                             const double *T, double t_end, const ac_integ_opts *opts,
                             int32_t *cell_status, int32_t *cell_stats, ac_stream stream) {
  if (ac_status s = integ_args(ws, n_cells, y, T, t_end, opts)) return s;
  ac::BdfParams P = bdf_params(opts, t_end);
  const int ns = ws->net->d.ns;
  for (int64_t c = 0; c < n_cells; ++c) {
    ac::CellOut out{cell_status ? cell_status + c : nullptr,
                    cell_stats ? cell_stats + c * AC_NSTAT : nullptr};
    ac::TapeView tv{nullptr, nullptr, 0};
    hipError_t e = ac::launch_bdf(ws->net->d, log_alpha, 1, y + c * ns, T + c * ws->net->d.n_cond,
                                  nullptr, P, out, tv, ws->W,
                                  nullptr, 1, hipStream_t(stream));
    if (e != hipSuccess) return hip_fail(e, "ac_integrate_plain launch");
  }
  return AC_OK;
}

ac_status ac_newton_solve(ac_ws *ws, int64_t n_mat, const double *jvals, const double *c,
                          double *b, int32_t trans, int32_t linear_solver, int32_t *info,
                          ac_stream stream) {
  if (!ws) return fail(AC_EINVAL, "null workspace");
  if (n_mat < 0) return fail(AC_EINVAL, "n_mat < 0");
  if (n_mat && (!jvals || !c || !b)) return fail(AC_EINVAL, "null jvals, c or b");
  if (trans != 0 && trans != 1) return fail(AC_EINVAL, "trans must be 0 or 1");
  if (linear_solver != AC_LINSOLVE_AUTO && linear_solver != AC_LINSOLVE_DENSE)
    return fail(AC_EINVAL, "linear_solver must be AC_LINSOLVE_AUTO or AC_LINSOLVE_DENSE");
  ac::BdfParams P{};
  P.linear_solver = linear_solver;
  hipError_t e = ac::launch_newton(ws->net->d, n_mat, jvals, c, b, trans,
                                   ac::use_front(ws->net->d, P), ws->W, ws->n_slots, info,
                                   hipStream_t(stream));
  return e == hipSuccess ? AC_OK : hip_fail(e, "ac_newton_solve launch");
}

// Adjoint slots for tapes of up to max_tape events: a checkpoint store
// (max_tape / every + 1 difference arrays), the converged states of one
// segment or, with keep_states and when they fit the budget over all
// slots, of every step, the adjoint difference array; plus per-cell rows of
// dL/dlog alpha for max_cells cells.
constexpr size_t ADJ_ALL_STATES_BUDGET = size_t(32) << 30;   // bytes over all slots

static ac_status adj_reserve(ac_ws *ws, int max_tape, int every, bool keep_states,
                             int max_cells) {
  const int ns = ws->net->d.ns, nr = ws->net->d.nr;
  const size_t S = size_t(ws->n_slots);
  const int ckcap = max_tape / every + 1;
  bool all_states = keep_states &&
                    sizeof(double) * size_t(max_tape) * ns * S <= ADJ_ALL_STATES_BUDGET;
  const int segcap = all_states ? max_tape : every;
  auto r256 = [](size_t b) { return (b + 255) / 256 * 256; };
  const size_t dsz = size_t(8) * ns;
  const size_t db_b = r256(sizeof(double) * dsz);
  const size_t ck_b = r256(sizeof(double) * dsz * size_t(ckcap));
  const size_t sy_b = r256(sizeof(double) * size_t(segcap) * ns);
  const size_t ce_b = r256(sizeof(int) * size_t(ckcap));
  const size_t bytes = (db_b + ck_b + sy_b + ce_b) * S;
  hipError_t e = hipDeviceSynchronize();   // nothing may still use the old buffers
  if (e != hipSuccess) return hip_fail(e, "adjoint reservation (sync)");
  if (ws->adj_buf) hipFree(ws->adj_buf);
  if (ws->rows) hipFree(ws->rows);
  ws->adj_buf = nullptr;
  ws->rows = nullptr;
  ws->adj_bytes = 0;
  ws->adj_tape = 0;
  ws->max_cells = 0;
  void *p = nullptr;
  e = hipMalloc(&p, bytes);
  if (e != hipSuccess) return hip_fail(e, "hipMalloc(adjoint workspace)");
  ws->adj_buf = p;
  if (max_cells > 0) {
    e = hipMalloc(reinterpret_cast<void **>(&ws->rows), sizeof(double) * size_t(max_cells) * nr);
    if (e != hipSuccess) {
      hipFree(ws->adj_buf);
      ws->adj_buf = nullptr;
      return hip_fail(e, "hipMalloc(adjoint gradient rows)");
    }
  }
  ws->adj_bytes = bytes + sizeof(double) * size_t(max_cells) * nr;
  char *b = static_cast<char *>(p);
  ac::AdjView &A = ws->A;
  A.Db = reinterpret_cast<double *>(b);
  b += db_b * S;
  A.ck = reinterpret_cast<double *>(b);
  b += ck_b * S;
  A.segY = reinterpret_cast<double *>(b);
  b += sy_b * S;
  A.ckev = reinterpret_cast<int *>(b);
  A.db_stride = db_b / sizeof(double);
  A.ck_stride = ck_b / sizeof(double);
  A.segy_stride = sy_b / sizeof(double);
  A.ckev_stride = ce_b / sizeof(int);
  A.ckcap = ckcap;
  A.every = every;
  A.segcap = segcap;
  A.all_states = all_states ? 1 : 0;
  ws->adj_tape = max_tape;
  ws->max_cells = max_cells;
  return AC_OK;
}

ac_status ac_ws_reserve_adjoint(ac_ws *ws, const ac_adj_reserve *r) {
  if (!ws || !r) return fail(AC_EINVAL, "null workspace or reservation");
  const int every = r->checkpoint_every ? r->checkpoint_every : ac::CK_EVERY;
  if (r->max_tape <= 0 || every <= 0 || r->max_cells < 0)
    return fail(AC_EINVAL, "need max_tape > 0, checkpoint_every >= 0, max_cells >= 0");
  return adj_reserve(ws, r->max_tape, every, r->keep_states != 0, r->max_cells);
}

ac_status ac_ws_adjoint_info(const ac_ws *ws, int32_t *max_tape, int32_t *checkpoint_every,
                             int32_t *keeps_states, int32_t *max_cells) {
  if (!ws) return fail(AC_EINVAL, "null workspace");
  if (max_tape) *max_tape = ws->adj_tape;
  if (checkpoint_every) *checkpoint_every = ws->adj_tape ? ws->A.every : 0;
  if (keeps_states) *keeps_states = ws->adj_tape ? ws->A.all_states : 0;
  if (max_cells) *max_cells = ws->max_cells;
  return AC_OK;
}

// The reserved slots serve a call with this tape capacity and interval.
static ac_status adj_capacity(const ac_ws *ws, int tape_cap, const ac_integ_opts *o) {
  const int every = o->checkpoint_every ? o->checkpoint_every : ac::CK_EVERY;
  if (every <= 0) return fail(AC_EINVAL, "checkpoint_every must be >= 0");
  if (ws->adj_tape <= 0)
    return fail(AC_ECAPACITY, "workspace has no adjoint capacity (ac_ws_reserve_adjoint)");
  if (tape_cap > ws->adj_tape || every != ws->A.every)
    return fail(AC_ECAPACITY, "tape longer than the workspace's adjoint reservation (" +
                                  std::to_string(ws->adj_tape) + " events) or a checkpoint "
                                  "interval other than the reserved " +
                                  std::to_string(ws->A.every));
  return AC_OK;
}

ac_status ac_replay(ac_ws *ws, const double *log_alpha, int64_t n_cells, const double *y0,
                    const double *T, const ac_integ_opts *opts, const ac_event *tape,
                    int32_t tape_cap, const int32_t *tape_len, double *y_final,
                    int32_t *cell_status, int32_t *cell_stats, ac_stream stream) {
  if (ac_status s = integ_args(ws, n_cells, y0, T, 0.0, opts)) return s;
  if (tape_cap <= 0) return fail(AC_EINVAL, "tape_cap must be > 0");
  if (n_cells && (!tape || !tape_len || !y_final))
    return fail(AC_EINVAL, "null tape, tape_len or y_final");
  if (!n_cells) return AC_OK;
  if (ac_status s = adj_capacity(ws, tape_cap, opts)) return s;
  ac::BdfParams P = bdf_params(opts, 0.0);
  ac::AdjIO io{reinterpret_cast<const ac::AcEvent *>(tape), tape_len, tape_cap, y0, T, nullptr,
               y_final, nullptr, nullptr, cell_status, cell_stats};
  hipError_t e = ac::launch_adjoint(ws->net->d, log_alpha, n_cells, io, P, ws->W, ws->A,
                                    ws->queue, ws->n_slots, hipStream_t(stream));
  return e == hipSuccess ? AC_OK : hip_fail(e, "ac_replay launch");
}

ac_status ac_integrate_adjoint(ac_ws *ws, const double *log_alpha, int64_t n_cells,
                               const double *y0, const double *T, const ac_integ_opts *opts,
                               const ac_event *tape, int32_t tape_cap, const int32_t *tape_len,
                               const double *lambda, double *y_final, double *dL_dy0,
                               double *g_cells, double *dL_dlogalpha, int32_t *cell_status,
                               int32_t *cell_stats, ac_stream stream) {
  if (ac_status s = integ_args(ws, n_cells, y0, T, 0.0, opts)) return s;
  if (tape_cap <= 0) return fail(AC_EINVAL, "tape_cap must be > 0");
  if (n_cells && (!tape || !tape_len || !lambda || !dL_dy0))
    return fail(AC_EINVAL, "null tape, tape_len, lambda or dL_dy0");
  hipStream_t st = hipStream_t(stream);
  const ac::DNet &d = ws->net->d;
  if (!n_cells) {
    if (dL_dlogalpha) {
      hipError_t e = ac::launch_sum_rows(nullptr, 0, d.nr, dL_dlogalpha, false, st);
      if (e != hipSuccess) return hip_fail(e, "ac_integrate_adjoint reduction");
    }
    return AC_OK;
  }
  if (ac_status s = adj_capacity(ws, tape_cap, opts)) return s;
  if (dL_dlogalpha && !g_cells && ws->max_cells <= 0)
    return fail(AC_ECAPACITY, "dL_dlogalpha without g_cells needs the workspace's gradient rows "
                              "(ac_adj_reserve.max_cells > 0)");
  ac::AdjView A = ws->A;
  if (opts->adj_recompute) A.all_states = 0;   // segments recomputed from checkpoints
  ac::BdfParams P = bdf_params(opts, 0.0);
  // cells in chunks: all at once into the caller's rows, or max_cells at a
  // time into the workspace's rows, each chunk's rows added to the sum in
  // cell order (the same order as one pass over every row)
  const int64_t chunk = g_cells || !dL_dlogalpha ? n_cells : int64_t(ws->max_cells);
  const int nc = d.n_cond, ns = d.ns;
  for (int64_t c0 = 0; c0 < n_cells; c0 += chunk) {
    const int64_t m = n_cells - c0 < chunk ? n_cells - c0 : chunk;
    double *rows = g_cells ? g_cells + c0 * d.nr : (dL_dlogalpha ? ws->rows : nullptr);
    ac::AdjIO io{reinterpret_cast<const ac::AcEvent *>(tape) + c0 * tape_cap, tape_len + c0,
                 tape_cap, y0 + c0 * ns, T + c0 * nc, lambda + c0 * ns,
                 y_final ? y_final + c0 * ns : nullptr, dL_dy0 + c0 * ns, rows,
                 cell_status ? cell_status + c0 : nullptr,
                 cell_stats ? cell_stats + c0 * AC_NSTAT : nullptr};
    hipError_t e = ac::launch_adjoint(d, log_alpha, m, io, P, ws->W, A, ws->queue, ws->n_slots, st);
    if (e != hipSuccess) return hip_fail(e, "ac_integrate_adjoint launch");
    if (dL_dlogalpha && !g_cells) {
      e = ac::launch_sum_rows(ws->rows, m, d.nr, dL_dlogalpha, c0 > 0, st);
      if (e != hipSuccess) return hip_fail(e, "ac_integrate_adjoint reduction");
    }
  }
  if (dL_dlogalpha && g_cells) {
    hipError_t e = ac::launch_sum_rows(g_cells, n_cells, d.nr, dL_dlogalpha, false, st);
    if (e != hipSuccess) return hip_fail(e, "ac_integrate_adjoint reduction");
  }
  return AC_OK;
}

}  // extern "C"
