// libuclp host runtime: the C ABI of include/uc_lp.h.
//
// Layers (bottom up):
//   presolve   validation, removal of fixed columns and empty rows, 'L' rows
//              negated, equality rows first, row-block partitions
//   Instance   one LP: host copy of the internal problem and one device arena
//              (CSR of A and A^T, FP64 and FP32 scaled values, scaled data,
//              iterates of both precisions, partial sums)
//   setup      device transpose, Ruiz + Pock-Chambolle scaling, power
//              iteration for ||A_hat||_2, initial iterates
//   Engine     one device, an HBM budget, a FIFO of queued solves and a slot
//              table; a worker thread runs epochs of kkt_every PDHG iterations
//              over every resident instance with batched kernels, then one
//              FP64 KKT check per instance, restart / primal-weight /
//              termination decisions on the host, and admission of queued
//              instances at the epoch boundary.
//
// The method (restarted reflected-Halpern PDHG with adaptive restarts and a
// smoothed primal weight, after Applegate et al. 2021 and Lu & Yang 2024) is
// the first-order LP solve that the paper runs on its GPU leg (Sec. II-C,
// III-C) with the limits of Sec. II-D.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <deque>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "../../include/uc_lp.h"
#include "check.h"
#include "uclp_dev.h"

using namespace uclp;

// ---------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------

static thread_local std::string g_err;

static int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

#define HIPOK(call)                                                                          \
  do {                                                                                       \
    hipError_t e_ = (call);                                                                  \
    if (e_ != hipSuccess)                                                                    \
      return fail(UC_LP_EHIP, "%s failed: %s (%s:%d)", #call, hipGetErrorString(e_), __FILE__, \
                  __LINE__);                                                                 \
  } while (0)

static double now_s() {
  using namespace std::chrono;
  return duration<double>(steady_clock::now().time_since_epoch()).count();
}

// ---------------------------------------------------------------------------
// options
// ---------------------------------------------------------------------------

extern "C" void uc_lp_opts_default(uc_lp_opts* o) {
  if (!o) return;
  std::memset(o, 0, sizeof *o);
  o->precision = UC_LP_FP32_MIXED_POLISH;
  o->kkt_every = 64;
  o->ruiz_iters = 10;
  o->power_iters = 64;
  o->iter_limit = 100000;
  o->eps_rel = 1e-4;
  o->eps_abs_feas = 0.0;
  o->eps_polish = 1e-8;
  o->time_limit_s = 3600.0;
  o->step_scale = 0.99;
  o->spmv_algo = UC_LP_SPMV_ROWSPLIT;
  o->verbose = 0;
  o->timing = 0;
  o->restart_to_current = 0;
  o->restart_sufficient = 0.2;
  o->restart_necessary = 0.9;
  o->restart_artificial = 0.36;
  o->pw_smoothing = 0.8;
  o->halpern_gamma = 1.0;
  o->pw_max_change = 4.0;
  o->pw_integral = 0.0;
  o->pw_balance = 0.5;
  o->pw_balance_polish = 0.0;
  o->fp32_stall_checks = 24;
  o->reserved = 0;
  o->eps_gap_rel = 0.0;
  o->eps_refine = 1e-2;
  o->refine_growth = 1e4;
  o->refine_max_rounds = 200;
  o->reserved2 = 0;
  o->pw_balance_refine = 0.5;
  o->refine_diverge = 0.0;
}

static int check_opts(const uc_lp_opts& o) {
  if (o.precision < 0 || o.precision > 3) return fail(UC_LP_ENOTSUP, "precision %d", o.precision);
  if (!(o.eps_refine > 0 && o.eps_refine < 1) || !(o.refine_growth > 1) || o.refine_max_rounds < 0 ||
      o.refine_max_rounds > 1000 || o.reserved2 != 0 ||
      !(o.pw_balance_refine >= 0 && o.pw_balance_refine <= 1) ||
      !(o.refine_diverge == 0 || (o.refine_diverge > 1 && std::isfinite(o.refine_diverge))))
    return fail(UC_LP_EINVAL, "refinement parameters out of range");
  if (o.kkt_every < 1 || o.kkt_every > 1 << 20) return fail(UC_LP_EINVAL, "kkt_every %d", o.kkt_every);
  if (o.ruiz_iters < 0 || o.ruiz_iters > 1000) return fail(UC_LP_EINVAL, "ruiz_iters");
  if (o.power_iters < 1 || o.power_iters > 100000) return fail(UC_LP_EINVAL, "power_iters");
  if (o.iter_limit < 1) return fail(UC_LP_EINVAL, "iter_limit");
  if (!(o.eps_rel > 0) || !(o.eps_polish > 0) || !(o.eps_abs_feas >= 0))
    return fail(UC_LP_EINVAL, "tolerances must be positive");
  if (!(o.time_limit_s > 0)) return fail(UC_LP_EINVAL, "time_limit_s");
  if (!(o.step_scale > 0 && o.step_scale < 1)) return fail(UC_LP_EINVAL, "step_scale in (0,1)");
  if (o.spmv_algo != UC_LP_SPMV_ROWSPLIT) return fail(UC_LP_ENOTSUP, "spmv_algo %d for PDHG", o.spmv_algo);
  if (!(o.restart_sufficient > 0 && o.restart_sufficient <= o.restart_necessary && o.restart_necessary < 1) ||
      !(o.restart_artificial > 0 && o.restart_artificial <= 1) || !(o.pw_smoothing >= 0 && o.pw_smoothing <= 1) ||
      (o.restart_to_current != 0 && o.restart_to_current != 1) || !(o.halpern_gamma >= 0 && o.halpern_gamma <= 1) ||
      !(o.pw_max_change == 0 || o.pw_max_change >= 1) || o.fp32_stall_checks < 0 || o.reserved != 0 ||
      !(o.pw_integral >= 0 && o.pw_integral <= 1) || !(o.pw_balance >= 0 && o.pw_balance <= 1) ||
      !(o.pw_balance_polish >= 0 && o.pw_balance_polish <= 1) || !(o.eps_gap_rel >= 0 && o.eps_gap_rel < 1))
    return fail(UC_LP_EINVAL, "restart / primal-weight parameters out of range");
  return UC_LP_OK;
}

// ---------------------------------------------------------------------------
// validation and minimal presolve
// ---------------------------------------------------------------------------

static int validate_csr(int32_t m, int32_t n, int64_t nnz, const int32_t* rp, const int32_t* ci,
                        const double* v) {
  if (m < 1 || n < 1) return fail(UC_LP_EINVAL, "m=%d n=%d must be >= 1", m, n);
  if (nnz < 0 || nnz > INT32_MAX) return fail(UC_LP_EINVAL, "nnz=%lld out of range", (long long)nnz);
  if (!rp || (nnz > 0 && (!ci || !v))) return fail(UC_LP_EINVAL, "NULL CSR array");
  if (rp[0] != 0) return fail(UC_LP_EINVAL, "row_ptr[0] != 0");
  if (rp[m] != nnz) return fail(UC_LP_EINVAL, "row_ptr[m]=%d != nnz", rp[m]);
  std::vector<int32_t> seen(n, -1);
  for (int32_t r = 0; r < m; ++r) {
    if (rp[r + 1] < rp[r]) return fail(UC_LP_EINVAL, "row_ptr not monotone at row %d", r);
    for (int32_t k = rp[r]; k < rp[r + 1]; ++k) {
      const int32_t c = ci[k];
      if (c < 0 || c >= n) return fail(UC_LP_EINVAL, "column index %d out of range at entry %d", c, k);
      if (seen[c] == r) return fail(UC_LP_EINVAL, "duplicate entry (%d,%d)", r, c);
      seen[c] = r;
      if (!std::isfinite(v[k])) return fail(UC_LP_EINVAL, "non-finite matrix value at entry %d", k);
    }
  }
  return UC_LP_OK;
}

// Runs f(t) for t in [0, count) on up to count host threads (the calling
// thread takes t = 0) and joins them.  For independent per-scenario or
// per-range host work; f must not throw.
template <typename F>
static void fork_join(int count, F f) {
  std::vector<std::thread> th;
  th.reserve(count > 1 ? count - 1 : 0);
  for (int t = 1; t < count; ++t) th.emplace_back(f, t);
  if (count > 0) f(0);
  for (auto& x : th) x.join();
}

static int validate_data(int32_t m, int32_t n, const double* c, const double* b, const char* sense,
                         const double* lb, const double* ub) {
  if (!c || !b || !sense || !lb || !ub) return fail(UC_LP_EINVAL, "NULL data array");
  for (int32_t j = 0; j < n; ++j) {
    if (!std::isfinite(c[j])) return fail(UC_LP_EINVAL, "non-finite cost c[%d]", j);
    if (std::isnan(lb[j]) || std::isnan(ub[j])) return fail(UC_LP_EINVAL, "NaN bound at column %d", j);
    if (lb[j] > ub[j]) return fail(UC_LP_EINVAL, "lb > ub at column %d", j);
    if (lb[j] == INFINITY || ub[j] == -INFINITY) return fail(UC_LP_EINVAL, "infinite bound on the wrong side at column %d", j);
  }
  for (int32_t i = 0; i < m; ++i) {
    if (!std::isfinite(b[i])) return fail(UC_LP_EINVAL, "non-finite right-hand side b[%d]", i);
    if (sense[i] != 'E' && sense[i] != 'G' && sense[i] != 'L')
      return fail(UC_LP_EINVAL, "unknown sense code %d at row %d", (int)sense[i], i);
  }
  return UC_LP_OK;
}

static void partition_rows(const std::vector<int>& ptr, int rows, std::vector<int>& blk) {
  blk.clear();
  blk.push_back(0);
  int r = 0;
  while (r < rows) {
    const int start = r;
    const int z0 = ptr[r];
    if (ptr[r + 1] - z0 > kNnzTile) {
      ++r;
      blk.push_back(r);
      continue;
    }
    while (r < rows && r - start < kRowsPerBlock && ptr[r + 1] - z0 <= kNnzTile) ++r;
    blk.push_back(r);
  }
}

struct HostProblem {
  int32_t m = 0, n = 0;
  int64_t nnz = 0;
  // original data (kept for update_data and postsolve)
  std::vector<int32_t> o_ptr, o_col;
  std::vector<double> o_val, o_c, o_b, o_lb, o_ub;
  std::vector<char> o_sense;
  // internal problem
  int mi = 0, ni = 0, m_eq = 0;
  int64_t nnzi = 0;
  std::vector<int> a_ptr, a_col, t_ptr, a_blk, t_blk;
  std::vector<int> a_seg, t_seg;  // entry offset of each row block (nblk + 1)
  std::vector<int> a_flag, t_flag;  // TileFlag bits of each row block
  std::vector<int> fx_row, fx_col;  // entries of A in fixed columns
  std::vector<double> fx_val;
  std::vector<int> a_base, t_base;  // Tile::base of each row block
  std::vector<uint16_t> a_end, t_end;  // row ends relative to the row block's first entry
  std::vector<double> a_val, c, b, l, u;
  std::vector<int> row_map;  // internal row -> original row (negative: -(row+1), negated 'L')
  std::vector<int> col_map;  // internal column -> original column
  std::vector<int> int_col;  // original column -> internal column or -1 (fixed)
  double obj_offset = 0.0;
  double norm_b = 0.0, norm_c = 0.0;
  bool infeasible = false;
};

// Tiles of one matrix of one slot: rows [r0, r1) and entries [k0, k1) of each
// row block, taken from the host copies of the partition and row pointers.
static void push_tiles(std::vector<Tile>& v, int slot, const std::vector<int>& blk, const std::vector<int>& ptr,
                       const std::vector<int>* flags = nullptr, const std::vector<int>* base = nullptr) {
  for (size_t b = 0; b + 1 < blk.size(); ++b) {
    Tile t;
    t.slot = slot;
    t.blk = (int)b;
    t.r0 = blk[b];
    t.r1 = blk[b + 1];
    t.k0 = ptr[t.r0];
    t.k1 = ptr[t.r1];
    t.flags = flags ? (*flags)[b] : 0;
    t.base = base ? (*base)[b] : -1;
    v.push_back(t);
  }
}

// Tile::base of every row block of A and of A^T: the smallest gathered index
// when the block fits the LDS tile and its gathered indices span less than
// 2^kPackShift, else -1.
static void block_bases(HostProblem& P) {
  const int na = (int)P.a_blk.size() - 1, nt = (int)P.t_blk.size() - 1;
  std::vector<int> lo(std::max(nt, 0), INT32_MAX), hi(std::max(nt, 0), -1);
  std::vector<int> tblk_of(P.ni);
  for (int bk = 0; bk < nt; ++bk)
    for (int j = P.t_blk[bk]; j < P.t_blk[bk + 1]; ++j) tblk_of[j] = bk;
  P.a_base.assign(std::max(na, 0), -1);
  for (int bk = 0; bk < na; ++bk) {
    const int k0 = P.a_ptr[P.a_blk[bk]], k1 = P.a_ptr[P.a_blk[bk + 1]];
    if (k1 == k0 || k1 - k0 > kNnzTile) continue;
    int mn = INT32_MAX, mx = -1;
    for (int k = k0; k < k1; ++k) {
      mn = std::min(mn, P.a_col[k]);
      mx = std::max(mx, P.a_col[k]);
    }
    if (mx - mn < (1 << kPackShift)) P.a_base[bk] = mn;
  }
  for (int i = 0; i < P.mi; ++i)
    for (int k = P.a_ptr[i]; k < P.a_ptr[i + 1]; ++k) {
      const int tb = tblk_of[P.a_col[k]];
      lo[tb] = std::min(lo[tb], i);
      hi[tb] = std::max(hi[tb], i);
    }
  P.t_base.assign(std::max(nt, 0), -1);
  for (int bk = 0; bk < nt; ++bk) {
    const int z = P.t_ptr[P.t_blk[bk + 1]] - P.t_ptr[P.t_blk[bk]];
    if (z == 0 || z > kNnzTile) continue;
    if (hi[bk] - lo[bk] < (1 << kPackShift)) P.t_base[bk] = lo[bk];
  }
}

// End of every row's entries relative to its block's first entry (a block
// holds at most kNnzTile entries, so the offsets fit 16 bits); long-row blocks
// never read them and get 0.
static void block_row_ends(const std::vector<int>& ptr, const std::vector<int>& blk, std::vector<uint16_t>& end) {
  end.assign(ptr.size() - 1, 0);
  for (size_t bk = 0; bk + 1 < blk.size(); ++bk) {
    const int z0 = ptr[blk[bk]];
    if (ptr[blk[bk + 1]] - z0 > kNnzTile) continue;
    for (int r = blk[bk]; r < blk[bk + 1]; ++r) end[r] = (uint16_t)(ptr[r + 1] - z0);
  }
}

static bool is_pos_zero(double v) { return v == 0.0 && !std::signbit(v); }

// Per-block TileFlag bits of P's internal data over S's row blocks (exact
// comparisons).
static void block_flags(HostProblem& P, const HostProblem& S) {
  const int nt = (int)S.t_blk.size() - 1, na = (int)S.a_blk.size() - 1;
  P.t_flag.assign(std::max(nt, 0), 0);
  P.a_flag.assign(std::max(na, 0), 0);
  for (int bk = 0; bk < nt; ++bk) {
    int f = kColC0 | kColL0 | kColLInf | kColLNegU | kColUInf;
    for (int j = S.t_blk[bk]; j < S.t_blk[bk + 1]; ++j) {
      if (!is_pos_zero(P.c[j])) f &= ~kColC0;
      if (!is_pos_zero(P.l[j])) f &= ~kColL0;
      if (!(std::isinf(P.l[j]) && P.l[j] < 0)) f &= ~kColLInf;
      if (!(P.l[j] == -P.u[j] && std::signbit(P.l[j]) != std::signbit(P.u[j]))) f &= ~kColLNegU;
      if (!(std::isinf(P.u[j]) && P.u[j] > 0)) f &= ~kColUInf;
    }
    P.t_flag[bk] = f;
  }
  for (int bk = 0; bk < na; ++bk) {
    int f = kRowB0;
    for (int i = S.a_blk[bk]; i < S.a_blk[bk + 1]; ++i)
      if (!is_pos_zero(P.b[i])) f = 0;
    P.a_flag[bk] = f;
  }
}

// Data-dependent part of the presolve (right-hand side shift, objective
// offset, norms, feasibility of removed rows).  The structure (which columns
// are fixed and which rows are empty) is fixed at create time.
// P holds the data (o_c, o_b, o_lb, o_ub in, c, b, l, u and the block flags
// out); S holds the structure (maps, fixed entries, blocks).  S is P itself
// except for the scenarios of a batch, which share their base's structure.
static void presolve_data(HostProblem& P, const HostProblem& S) {
  const int32_t m = P.m;
  std::vector<double> shift(m, 0.0);
  P.obj_offset = 0.0;
  for (size_t e = 0; e < S.fx_row.size(); ++e) shift[S.fx_row[e]] += S.fx_val[e] * P.o_lb[S.fx_col[e]];
  for (int32_t j = 0; j < P.n; ++j)
    if (S.int_col[j] < 0) P.obj_offset += P.o_c[j] * P.o_lb[j];
  P.infeasible = false;
  std::vector<char> kept(m, 0);
  for (int i = 0; i < P.mi; ++i) {
    const int enc = S.row_map[i];
    const int r = enc >= 0 ? enc : -enc - 1;
    kept[r] = 1;
    const double sgn = enc >= 0 ? 1.0 : -1.0;
    P.b[i] = sgn * (P.o_b[r] - shift[r]);
  }
  for (int32_t r = 0; r < m; ++r) {
    if (kept[r]) continue;
    const double rhs = P.o_b[r] - shift[r];  // removed row reads 0 (=,>=,<=) rhs
    const double tol = 1e-9 * (1.0 + std::fabs(P.o_b[r]));
    if ((S.o_sense[r] == 'E' && std::fabs(rhs) > tol) || (S.o_sense[r] == 'G' && rhs > tol) ||
        (S.o_sense[r] == 'L' && rhs < -tol))
      P.infeasible = true;
  }
  for (int j = 0; j < P.ni; ++j) {
    const int o = S.col_map[j];
    P.c[j] = P.o_c[o];
    P.l[j] = P.o_lb[o];
    P.u[j] = P.o_ub[o];
  }
  double nb = 0, nc = 0;
  for (int32_t r = 0; r < m; ++r) nb += P.o_b[r] * P.o_b[r];
  for (int32_t j = 0; j < P.n; ++j) nc += P.o_c[j] * P.o_c[j];
  P.norm_b = std::sqrt(nb);
  P.norm_c = std::sqrt(nc);
  block_flags(P, S);
}

static void presolve_structure(HostProblem& P) {
  const int32_t m = P.m, n = P.n;
  P.int_col.assign(n, -1);
  P.col_map.clear();
  for (int32_t j = 0; j < n; ++j)
    if (!(P.o_lb[j] == P.o_ub[j])) {
      P.int_col[j] = (int)P.col_map.size();
      P.col_map.push_back(j);
    }
  P.ni = (int)P.col_map.size();
  // entries in fixed columns, for the right-hand-side shift of presolve_data
  P.fx_row.clear();
  P.fx_col.clear();
  P.fx_val.clear();
  for (int32_t r = 0; r < m; ++r)
    for (int32_t k = P.o_ptr[r]; k < P.o_ptr[r + 1]; ++k)
      if (P.int_col[P.o_col[k]] < 0) {
        P.fx_row.push_back(r);
        P.fx_col.push_back(P.o_col[k]);
        P.fx_val.push_back(P.o_val[k]);
      }
  // rows with at least one entry in a kept column; E rows first
  std::vector<int> cnt(m, 0);
  for (int32_t r = 0; r < m; ++r)
    for (int32_t k = P.o_ptr[r]; k < P.o_ptr[r + 1]; ++k)
      if (P.int_col[P.o_col[k]] >= 0) ++cnt[r];
  P.row_map.clear();
  for (int pass = 0; pass < 2; ++pass)
    for (int32_t r = 0; r < m; ++r) {
      if (cnt[r] == 0) continue;
      const bool eq = P.o_sense[r] == 'E';
      if ((pass == 0) != eq) continue;
      P.row_map.push_back(P.o_sense[r] == 'L' ? -(r + 1) : r);
    }
  P.m_eq = 0;
  for (int enc : P.row_map)
    if (enc >= 0 && P.o_sense[enc] == 'E') ++P.m_eq;
  P.mi = (int)P.row_map.size();
  P.a_ptr.assign(P.mi + 1, 0);
  P.a_col.clear();
  P.a_val.clear();
  for (int i = 0; i < P.mi; ++i) {
    const int enc = P.row_map[i];
    const int r = enc >= 0 ? enc : -enc - 1;
    const double sgn = enc >= 0 ? 1.0 : -1.0;
    // keep the columns of a row in increasing internal order
    std::vector<std::pair<int, double>> ent;
    for (int32_t k = P.o_ptr[r]; k < P.o_ptr[r + 1]; ++k) {
      const int jc = P.int_col[P.o_col[k]];
      if (jc >= 0) ent.emplace_back(jc, sgn * P.o_val[k]);
    }
    std::sort(ent.begin(), ent.end());
    for (auto& e : ent) {
      P.a_col.push_back(e.first);
      P.a_val.push_back(e.second);
    }
    P.a_ptr[i + 1] = (int)P.a_col.size();
  }
  P.nnzi = (int64_t)P.a_col.size();
  // transposed row pointer (column counts) and both partitions
  P.t_ptr.assign(P.ni + 1, 0);
  for (int c : P.a_col) ++P.t_ptr[c + 1];
  for (int j = 0; j < P.ni; ++j) P.t_ptr[j + 1] += P.t_ptr[j];
  partition_rows(P.a_ptr, P.mi, P.a_blk);
  partition_rows(P.t_ptr, P.ni, P.t_blk);
  P.a_seg.resize(P.a_blk.size());
  P.t_seg.resize(P.t_blk.size());
  for (size_t b = 0; b < P.a_blk.size(); ++b) P.a_seg[b] = P.a_ptr[P.a_blk[b]];
  for (size_t b = 0; b < P.t_blk.size(); ++b) P.t_seg[b] = P.t_ptr[P.t_blk[b]];
  block_bases(P);
  block_row_ends(P.a_ptr, P.a_blk, P.a_end);
  block_row_ends(P.t_ptr, P.t_blk, P.t_end);
  P.b.assign(P.mi, 0.0);
  P.c.assign(P.ni, 0.0);
  P.l.assign(P.ni, 0.0);
  P.u.assign(P.ni, 0.0);
}

// ---------------------------------------------------------------------------
// device arena of one instance
// ---------------------------------------------------------------------------

struct Arena {
  char* base = nullptr;
  size_t bytes = 0, used = 0;
  template <typename T>
  T* take(size_t count) {
    const size_t off = (used + 255) & ~(size_t)255;
    used = off + std::max<size_t>(count, 1) * sizeof(T);
    return base ? reinterpret_cast<T*>(base + off) : nullptr;
  }
};

template <typename T>
static void carve_vecs(Arena& A, Vecs<T>& V, int n, int m, int ns) {
  V.x = A.take<T>((size_t)n * ns);
  V.x0 = A.take<T>((size_t)n * ns);
  V.xbar = A.take<T>((size_t)n * ns);
  V.xhat = A.take<T>((size_t)n * ns);
  V.y = A.take<T>((size_t)m * ns);
  V.y0 = A.take<T>((size_t)m * ns);
  V.yhat = A.take<T>((size_t)m * ns);
  V.c = A.take<T>((size_t)n * ns);
  V.l = A.take<T>((size_t)n * ns);
  V.u = A.take<T>((size_t)n * ns);
  V.b = A.take<T>((size_t)m * ns);
}

struct DevMem {
  Arena ar;
  int *a_ptr, *a_col, *t_ptr, *t_col, *a_blk, *t_blk;
  double *a_raw, *t_raw;
  double *a_v64, *t_v64;
  float *a_v32, *t_v32;
  int *a_seg, *t_seg, *a_cs, *t_cs;
  unsigned short *a_dst, *t_dst;
  unsigned *a_pk, *t_pk;
  int *a_base, *t_base;
  unsigned short *a_end, *t_end;
  double *a_vs64, *t_vs64;
  float *a_vs32, *t_vs32;
  double *c_in, *b_in, *l_in, *u_in;  // unscaled internal data (scenario-major)
  double *dr, *dc, *fr, *fc;
  double *part_a, *part_t, *scal;
  double *x_out, *y_out, *x_warm, *y_warm;
  double *pv, *pw, *pu, *red_part, *red_out;  // power iteration / norms
  float* ylo32;  // lower bound of the inequality duals (refinement rounds)
  int *row_of, *keys_in, *keys_out, *perm_in, *perm_out;
  void* sort_temp;
  size_t sort_bytes;
  Vecs<float> f;
  Vecs<double> d;
  SlotDev* slot_dev;  // device copy of this instance's descriptor
  unsigned long long* tick;  // device clock stamp
};

static void carve(DevMem& D, const HostProblem& P, int ns) {
  Arena& A = D.ar;
  const int m = P.mi, n = P.ni;
  const int64_t z = P.nnzi;
  D.a_ptr = A.take<int>(m + 1);
  D.a_col = A.take<int>(z);
  D.t_ptr = A.take<int>(n + 1);
  D.t_col = A.take<int>(z);
  D.a_blk = A.take<int>(P.a_blk.size());
  D.t_blk = A.take<int>(P.t_blk.size());
  D.a_raw = A.take<double>(z);
  D.t_raw = A.take<double>(z);
  D.a_v64 = A.take<double>(z);
  D.t_v64 = A.take<double>(z);
  D.a_v32 = A.take<float>(z);
  D.t_v32 = A.take<float>(z);
  D.a_seg = A.take<int>(P.a_seg.size());
  D.t_seg = A.take<int>(P.t_seg.size());
  D.a_cs = A.take<int>(z);
  D.t_cs = A.take<int>(z);
  D.a_dst = A.take<unsigned short>(z);
  D.t_dst = A.take<unsigned short>(z);
  D.a_pk = A.take<unsigned>(z);
  D.t_pk = A.take<unsigned>(z);
  D.a_base = A.take<int>(P.a_base.size());
  D.t_base = A.take<int>(P.t_base.size());
  D.a_end = A.take<unsigned short>(P.a_end.size());
  D.t_end = A.take<unsigned short>(P.t_end.size());
  D.a_vs64 = A.take<double>(z);
  D.t_vs64 = A.take<double>(z);
  D.a_vs32 = A.take<float>(z);
  D.t_vs32 = A.take<float>(z);
  D.c_in = A.take<double>((size_t)n * ns);
  D.l_in = A.take<double>((size_t)n * ns);
  D.u_in = A.take<double>((size_t)n * ns);
  D.b_in = A.take<double>((size_t)m * ns);
  D.dr = A.take<double>(m);
  D.dc = A.take<double>(n);
  D.fr = A.take<double>(m);
  D.fc = A.take<double>(n);
  const size_t na = P.a_blk.size(), nt = P.t_blk.size();
  D.part_a = A.take<double>(na * RQ_N * ns);
  D.part_t = A.take<double>(nt * CQ_N * ns);
  D.scal = A.take<double>((size_t)kScal * ns);
  D.x_out = A.take<double>((size_t)n * ns);
  D.y_out = A.take<double>((size_t)m * ns);
  D.x_warm = A.take<double>((size_t)n * ns);
  D.y_warm = A.take<double>((size_t)m * ns);
  D.pv = A.take<double>(n);
  D.pw = A.take<double>(n);
  D.pu = A.take<double>(m);
  D.red_part = A.take<double>(1024);
  D.red_out = A.take<double>(8);
  D.ylo32 = A.take<float>(m);
  D.row_of = A.take<int>(z);
  D.keys_in = D.a_col;  // the sort reads the column indices in place
  D.keys_out = A.take<int>(z);
  D.perm_in = A.take<int>(z);
  D.perm_out = A.take<int>(z);
  D.sort_bytes = std::max(radix_sort_temp_bytes(z, n),
                          std::max(seg_sort_temp_bytes(z, (int)P.a_blk.size() - 1, n),
                                   seg_sort_temp_bytes(z, (int)P.t_blk.size() - 1, m)));
  D.sort_temp = A.take<char>(D.sort_bytes);
  carve_vecs(A, D.f, n, m, ns);
  carve_vecs(A, D.d, n, m, ns);
  D.slot_dev = A.take<SlotDev>(1);
  D.tick = A.take<unsigned long long>(1);
}

static size_t arena_bytes(const HostProblem& P, int ns) {
  DevMem D;
  std::memset((void*)&D, 0, sizeof D);
  carve(D, P, ns);
  return D.ar.used + 256;
}

// ---------------------------------------------------------------------------
// engine and instance
// ---------------------------------------------------------------------------

// Epochs in flight: the worker enqueues epoch e + 1 before it reads the
// status of epoch e, so the device never waits for the host between epochs.
constexpr int kRing = 2;

struct uc_engine {
  int device = 0;
  size_t budget = 0, used = 0;
  int max_slots = 1;
  bool private_engine = false;
  hipStream_t stream = nullptr;
  std::thread worker;
  std::mutex mu;
  std::condition_variable cv;
  std::deque<uc_lp*> queue;
  std::vector<uc_lp*> active;
  bool shutdown = false;
  // device tables of the current layout
  bool layout_valid = false;  // false: rebuilt before the next epoch
  SlotDev* d_slots = nullptr;
  Tile* d_tiles = nullptr;
  size_t tile_cap = 0;
  int* d_ids = nullptr;
  double* d_scal = nullptr;   // device, max_slots * kScal (one copy per check)
  double* d_red2 = nullptr;   // device, max_slots * kRedChunks * (RQ_N + CQ_N)
  ChkState* d_chk = nullptr;  // device, max_slots: run state, advanced by the check kernel
  ChkParams* d_prm = nullptr; // device, max_slots
  ChkState* h_ring = nullptr; // pinned, kRing * max_slots: run state after each epoch
  size_t off_t0 = 0, off_a1 = 0, off_a0 = 0;
  int nT1 = 0, nT0 = 0, nA1 = 0, nA0 = 0, K = 64;
  bool timing = false;
  hipEvent_t ring_ev[kRing] = {};
  hipEvent_t tev[kRing][4] = {};  // start / stop of the timed primal and dual launch of each epoch
  SlotDev* h_slots = nullptr;  // pinned, max_slots
  double tick_rate = 0;        // device clock ticks per second
  std::string err;
};

// Iterative refinement state of one solve (UC_LP_FP32_REFINE).  The refined
// point (x*, y*) lives in the instance's FP64 x_hat, y_hat; while a
// correction problem runs, the scaled data arrays (FP64 and FP32) hold its
// data and the FP32 iterates its solution.
struct RefineRun {
  int round = 0;          // correction problems started so far
  double dp = 1, dd = 1;  // D_P, D_D of the running correction problem
  bool have_outer = false;
  // the refined point at the last round boundary (original problem)
  double pobj = 0, dobj = 0, rel_primal = 0, rel_dual = 0, rel_gap = 0, rel_kkt = 0, abs_inf = 0;
  double rel_kkt_inner = 0;
  std::vector<int> t_flag, a_flag;  // tile flags while correction data are loaded
  // the best refined point so far (its copy is in x_warm, y_warm, which the
  // rounds leave unused): a run that ends short of its target returns it
  // (a round can end worse than it began)
  bool have_best = false;
  double best[7] = {0, 0, 0, 0, 0, 0, 0};  // pobj, dobj, rel_primal, rel_dual, rel_gap, rel_kkt, abs_inf
};

struct uc_lp {
  uc_engine* eng = nullptr;
  bool owns_engine = false;
  uc_lp_opts opts;
  HostProblem P;
  DevMem D;
  bool uploaded = false;
  bool setup_done = false;
  size_t need_bytes = 0;
  std::atomic<int> status{UC_LP_IDLE};
  std::atomic<bool> cancel{false};
  mutable std::mutex mu;
  std::condition_variable done_cv;
  uc_lp_info info;
  std::vector<double> warm_x, warm_y;  // internal space
  bool has_warm = false;
  std::vector<double> sol_x, sol_y;    // original space
  ChkState chk;             // run state (the device's copy is ahead while epochs run)
  ChkParams prm;
  double t_start = 0;       // host clock at admission
  double t_stamp = 0;       // host clock at the device clock stamp
  uint64_t tick_start = 0;  // device clock when iterations start
  int host_stop = 0;        // terminal status the host imposes (time limit, cancel)
  int slot = -1;
  double t_request = 0;
  double hs_bytes[2][2] = {{0, 0}, {0, 0}};  // [precision][primal, dual] per half-step launch
  // timed launches by precision (0 FP64, 1 FP32)
  double timed_primal_ms[2] = {0, 0}, timed_dual_ms[2] = {0, 0};
  long long timed_n[2] = {0, 0};
  int data_gen = 0;  // bumped by uc_lp_update_data (tile flags depend on the data)
  RefineRun ref;
};

static void set_info(uc_lp* lp, const uc_lp_info& in) {
  std::lock_guard<std::mutex> g(lp->mu);
  lp->info = in;
}

static uc_lp_info get_info(const uc_lp* lp) {
  std::lock_guard<std::mutex> g(lp->mu);
  return lp->info;
}

static void finish_status(uc_lp* lp, int status) {
  {
    std::lock_guard<std::mutex> g(lp->mu);
    lp->info.status = status;
    lp->status.store(status);
  }
  lp->done_cv.notify_all();
}

static bool terminal(int s) {
  return s == UC_LP_OPTIMAL || s == UC_LP_ITER_LIMIT || s == UC_LP_TIME_LIMIT || s == UC_LP_CANCELLED ||
         s == UC_LP_NUMERICAL || s == UC_LP_INFEASIBLE || s == UC_LP_FAILED;
}

// ---- device memory of an instance ------------------------------------------

static int upload(uc_lp* lp) {
  HostProblem& P = lp->P;
  DevMem& D = lp->D;
  hipStream_t s = lp->eng->stream;
  std::memset((void*)&D, 0, sizeof D);
  const size_t bytes = arena_bytes(P, 1);
  void* base = nullptr;
  hipError_t e = hipMalloc(&base, bytes);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return fail(UC_LP_ENOMEM, "hipMalloc(%zu) failed: %s", bytes, hipGetErrorString(e));
  }
  D.ar.base = (char*)base;
  D.ar.bytes = bytes;
  carve(D, P, 1);
  HIPOK(hipMemcpyAsync(D.a_ptr, P.a_ptr.data(), sizeof(int) * (P.mi + 1), hipMemcpyHostToDevice, s));
  if (P.nnzi) {
    HIPOK(hipMemcpyAsync(D.a_col, P.a_col.data(), sizeof(int) * P.nnzi, hipMemcpyHostToDevice, s));
    HIPOK(hipMemcpyAsync(D.a_raw, P.a_val.data(), sizeof(double) * P.nnzi, hipMemcpyHostToDevice, s));
  }
  HIPOK(hipMemcpyAsync(D.t_ptr, P.t_ptr.data(), sizeof(int) * (P.ni + 1), hipMemcpyHostToDevice, s));
  HIPOK(hipMemcpyAsync(D.a_blk, P.a_blk.data(), sizeof(int) * P.a_blk.size(), hipMemcpyHostToDevice, s));
  HIPOK(hipMemcpyAsync(D.t_blk, P.t_blk.data(), sizeof(int) * P.t_blk.size(), hipMemcpyHostToDevice, s));
  HIPOK(hipMemcpyAsync(D.a_seg, P.a_seg.data(), sizeof(int) * P.a_seg.size(), hipMemcpyHostToDevice, s));
  HIPOK(hipMemcpyAsync(D.t_seg, P.t_seg.data(), sizeof(int) * P.t_seg.size(), hipMemcpyHostToDevice, s));
  if (!P.a_base.empty())
    HIPOK(hipMemcpyAsync(D.a_base, P.a_base.data(), sizeof(int) * P.a_base.size(), hipMemcpyHostToDevice, s));
  if (!P.t_base.empty())
    HIPOK(hipMemcpyAsync(D.t_base, P.t_base.data(), sizeof(int) * P.t_base.size(), hipMemcpyHostToDevice, s));
  if (!P.a_end.empty())
    HIPOK(hipMemcpyAsync(D.a_end, P.a_end.data(), sizeof(uint16_t) * P.a_end.size(), hipMemcpyHostToDevice, s));
  if (!P.t_end.empty())
    HIPOK(hipMemcpyAsync(D.t_end, P.t_end.data(), sizeof(uint16_t) * P.t_end.size(), hipMemcpyHostToDevice, s));
  HIPOK(hipStreamSynchronize(s));
  lp->uploaded = true;
  lp->setup_done = false;
  return UC_LP_OK;
}

static void release(uc_lp* lp) {
  if (lp->D.ar.base) {
    (void)hipFree(lp->D.ar.base);
    lp->D.ar.base = nullptr;
  }
  lp->uploaded = false;
  lp->setup_done = false;
}

static SlotDev make_slot(const HostProblem& P, const DevMem& D, double gamma) {
  SlotDev S;
  std::memset((void*)&S, 0, sizeof S);
  S.a_ptr = D.a_ptr;
  S.a_col = D.a_col;
  S.t_ptr = D.t_ptr;
  S.t_col = D.t_col;
  S.a_blk = D.a_blk;
  S.t_blk = D.t_blk;
  S.m = P.mi;
  S.n = P.ni;
  S.m_eq = P.m_eq;
  S.nscen = 1;
  S.gamma = gamma;
  S.active[0] = 1;
  S.a_nblk = (int)P.a_blk.size() - 1;
  S.t_nblk = (int)P.t_blk.size() - 1;
  S.dr = D.dr;
  S.dc = D.dc;
  S.f = D.f;
  S.d = D.d;
  S.f.av = D.a_v32;
  S.f.tv = D.t_v32;
  S.d.av = D.a_v64;
  S.d.tv = D.t_v64;
  S.f.avs = D.a_vs32;
  S.f.tvs = D.t_vs32;
  S.d.avs = D.a_vs64;
  S.d.tvs = D.t_vs64;
  S.a_cs = D.a_cs;
  S.t_cs = D.t_cs;
  S.a_dst = D.a_dst;
  S.t_dst = D.t_dst;
  S.a_pk = D.a_pk;
  S.t_pk = D.t_pk;
  S.a_end = D.a_end;
  S.t_end = D.t_end;
  S.ylo = D.ylo32;
  S.part_a = D.part_a;
  S.part_t = D.part_t;
  S.scal = D.scal;
  return S;
}

static SlotDev make_slot(const uc_lp* lp) { return make_slot(lp->P, lp->D, lp->opts.halpern_gamma); }

// Transpose, scaling, scaled data, power iteration.  Runs on `s`, synchronous.
static int setup_device(uc_lp* lp) {
  HostProblem& P = lp->P;
  DevMem& D = lp->D;
  hipStream_t s = lp->eng->stream;
  const int m = P.mi, n = P.ni;
  const int64_t z = P.nnzi;
  const int na = (int)P.a_blk.size() - 1, nt = (int)P.t_blk.size() - 1;
  // data (may have changed through uc_lp_update_data)
  HIPOK(hipMemcpyAsync(D.c_in, P.c.data(), sizeof(double) * n, hipMemcpyHostToDevice, s));
  HIPOK(hipMemcpyAsync(D.l_in, P.l.data(), sizeof(double) * n, hipMemcpyHostToDevice, s));
  HIPOK(hipMemcpyAsync(D.u_in, P.u.data(), sizeof(double) * n, hipMemcpyHostToDevice, s));
  if (m) HIPOK(hipMemcpyAsync(D.b_in, P.b.data(), sizeof(double) * m, hipMemcpyHostToDevice, s));
  // a1: A^T by a stable radix sort of the column indices
  {
    // an error left by an earlier call would otherwise be reported by the
    // sort's own final hipGetLastError(); name it here instead
    const hipError_t stale = hipGetLastError();
    if (stale != hipSuccess)
      return fail(UC_LP_EHIP, "an earlier HIP call failed before setup: %s", hipGetErrorName(stale));
  }
  launch_expand_rows(D.a_ptr, m, D.row_of, s);
  launch_iota(D.perm_in, z, s);
  HIPOK(hipGetLastError());
  {
    const int se = radix_sort_pairs(D.sort_temp, D.sort_bytes, D.keys_in, D.keys_out, D.perm_in, D.perm_out,
                                    z, n, s);
    if (se != 0)
      return fail(UC_LP_EHIP, "radix sort of %lld column indices failed: %s (temp %zu bytes)", (long long)z,
                  hipGetErrorName((hipError_t)se), D.sort_bytes);
  }
  launch_gather_transpose(D.perm_out, D.row_of, D.a_raw, z, D.t_col, D.t_raw, s);
  // a2: Ruiz equilibration then Pock-Chambolle (alpha = 1)
  launch_fill(D.dr, 1.0, m, s);
  launch_fill(D.dc, 1.0, n, s);
  for (int it = 0; it < lp->opts.ruiz_iters; ++it) {
    launch_scale_factor(0, D.a_ptr, D.a_col, D.a_raw, D.dr, D.dc, D.a_blk, na, m, D.fr, s);
    launch_scale_factor(0, D.t_ptr, D.t_col, D.t_raw, D.dc, D.dr, D.t_blk, nt, n, D.fc, s);
    launch_mul_inplace(D.dr, D.fr, m, s);
    launch_mul_inplace(D.dc, D.fc, n, s);
  }
  launch_scale_factor(1, D.a_ptr, D.a_col, D.a_raw, D.dr, D.dc, D.a_blk, na, m, D.fr, s);
  launch_scale_factor(1, D.t_ptr, D.t_col, D.t_raw, D.dc, D.dr, D.t_blk, nt, n, D.fc, s);
  launch_mul_inplace(D.dr, D.fr, m, s);
  launch_mul_inplace(D.dc, D.fc, n, s);
  launch_scale_values(D.a_ptr, D.a_col, D.a_raw, D.dr, D.dc, m, D.a_v64, D.a_v32, s);
  launch_scale_values(D.t_ptr, D.t_col, D.t_raw, D.dc, D.dr, n, D.t_v64, D.t_v32, s);
  // entries of each row block in column order, for the half-step gathers
  {
    HIPOK(hipGetLastError());
    int se = seg_sort_pairs(D.sort_temp, D.sort_bytes, D.a_col, D.a_cs, D.perm_in, D.perm_out, z, na, D.a_seg,
                            n, s);
    if (se == 0) {
      launch_gather_sorted(D.perm_out, D.a_seg, na, D.a_v64, D.a_v32, D.a_vs64, D.a_vs32, D.a_dst, D.a_cs,
                           D.a_base, D.a_pk, s);
      se = seg_sort_pairs(D.sort_temp, D.sort_bytes, D.t_col, D.t_cs, D.perm_in, D.perm_out, z, nt, D.t_seg, m,
                          s);
    }
    if (se == 0)
      launch_gather_sorted(D.perm_out, D.t_seg, nt, D.t_v64, D.t_v32, D.t_vs64, D.t_vs32, D.t_dst, D.t_cs,
                           D.t_base, D.t_pk, s);
    if (se != 0)
      return fail(UC_LP_EHIP, "segmented sort of the row blocks failed: %s", hipGetErrorName((hipError_t)se));
  }
  launch_scale_vectors(D.c_in, D.l_in, D.u_in, D.b_in, D.dc, D.dr, n, m, 1, (double*)D.d.c,
                       (double*)D.d.l, (double*)D.d.u, (double*)D.d.b, (float*)D.f.c, (float*)D.f.l,
                       (float*)D.f.u, (float*)D.f.b, s);
  // a3: ||A_hat||_2 by power iteration on A_hat' A_hat, and ||c_hat||, ||b_hat||
  launch_norm2(D.d.c, n, D.red_part, D.red_out + 1, s);
  if (m) launch_norm2(D.d.b, m, D.red_part, D.red_out + 2, s);
  else launch_fill(D.red_out + 2, 0.0, 1, s);
  launch_hash_vector(D.pv, n, 12345u, s);
  launch_norm2(D.pv, n, D.red_part, D.red_out, s);
  launch_normalize(D.pv, D.red_out, D.pv, n, s);
  for (int it = 0; it < lp->opts.power_iters; ++it) {
    launch_spmv64(D.a_ptr, D.a_col, D.a_v64, D.pv, D.pu, D.a_blk, na, s);
    launch_spmv64(D.t_ptr, D.t_col, D.t_v64, D.pu, D.pw, D.t_blk, nt, s);
    launch_norm2(D.pw, n, D.red_part, D.red_out, s);
    launch_normalize(D.pw, D.red_out, D.pv, n, s);
  }
  double h[3] = {0, 0, 0};
  HIPOK(hipMemcpyAsync(h, D.red_out, sizeof h, hipMemcpyDeviceToHost, s));
  HIPOK(hipStreamSynchronize(s));
  HIPOK(hipGetLastError());
  // the power-iteration estimate approaches ||A_hat||_2 from below, so it is
  // no safe step bound by itself; the step uses the Pock-Chambolle bound
  // ||A_hat||_2 <= 1 that the alpha = 1 scaling guarantees (Schur test), and
  // the estimate shows how tight that bound is
  const double norm_est = std::pow(std::max(h[0], 0.0), 0.25);
  const double norm_bound = 1.0;
  const double cn = std::sqrt(h[1]), bn = std::sqrt(h[2]);
  ChkState& st = lp->chk;
  st.eta = norm_bound > 0 ? lp->opts.step_scale / norm_bound : 1.0;
  st.omega = (cn > 0 && bn > 0) ? cn / bn : 1.0;
  {
    std::lock_guard<std::mutex> g(lp->mu);
    lp->info.norm_a_est = norm_est;
    lp->info.norm_a_bound = norm_bound;
    lp->info.eta = st.eta;
    lp->info.omega = st.omega;
  }
  SlotDev S = make_slot(lp);
  HIPOK(hipMemcpyAsync(D.slot_dev, &S, sizeof S, hipMemcpyHostToDevice, s));
  HIPOK(hipStreamSynchronize(s));
  lp->setup_done = true;
  return UC_LP_OK;
}

static int init_iterates(uc_lp* lp, int prec) {
  DevMem& D = lp->D;
  HostProblem& P = lp->P;
  hipStream_t s = lp->eng->stream;
  const double *xi = nullptr, *yi = nullptr;
  if (lp->has_warm) {
    HIPOK(hipMemcpyAsync(D.x_warm, lp->warm_x.data(), sizeof(double) * P.ni, hipMemcpyHostToDevice, s));
    if (P.mi) HIPOK(hipMemcpyAsync(D.y_warm, lp->warm_y.data(), sizeof(double) * P.mi, hipMemcpyHostToDevice, s));
    xi = D.x_warm;
    yi = D.y_warm;
  }
  launch_init_iterates(D.slot_dev, prec, xi, yi, P.ni, P.mi, P.m_eq, 1, s);
  HIPOK(hipGetLastError());
  return UC_LP_OK;
}

static int fetch_solution(uc_lp* lp, int prec) {
  DevMem& D = lp->D;
  HostProblem& P = lp->P;
  hipStream_t s = lp->eng->stream;
  launch_unscale(D.slot_dev, prec, D.x_out, D.y_out, P.ni, P.mi, 1, s);
  std::vector<double> xi(P.ni), yi(P.mi);
  HIPOK(hipMemcpyAsync(xi.data(), D.x_out, sizeof(double) * P.ni, hipMemcpyDeviceToHost, s));
  if (P.mi) HIPOK(hipMemcpyAsync(yi.data(), D.y_out, sizeof(double) * P.mi, hipMemcpyDeviceToHost, s));
  HIPOK(hipStreamSynchronize(s));
  lp->sol_x.assign(P.n, 0.0);
  lp->sol_y.assign(P.m, 0.0);
  for (int32_t j = 0; j < P.n; ++j)
    if (P.int_col[j] < 0) lp->sol_x[j] = P.o_lb[j];
  // x_hat lies in the scaled box; unscaling can overshoot a bound by an ulp,
  // so the original-space value is clamped back into [lb, ub]
  for (int j = 0; j < P.ni; ++j) lp->sol_x[P.col_map[j]] = std::min(std::max(xi[j], P.l[j]), P.u[j]);
  for (int i = 0; i < P.mi; ++i) {
    const int enc = P.row_map[i];
    if (enc >= 0) lp->sol_y[enc] = yi[i];
    else lp->sol_y[-enc - 1] = -yi[i];
  }
  return UC_LP_OK;
}

// ---- the KKT check: scalars -> info, restart / termination decisions -------

static void kkt_scalars(const double* q, double offset, double norm_b, double norm_c, uc_lp_info& in) {
  const double rho_p = std::sqrt(std::max(q[RQ_RES2], 0.0));
  const double rho_d = std::sqrt(std::max(q[RQ_N + CQ_DRES2] + q[RQ_YNEG2], 0.0));
  const double pobj = q[RQ_N + CQ_CX] - q[RQ_YLOR] + offset;
  const double dobj = q[RQ_BY] + q[RQ_N + CQ_LBUB] + offset;
  in.pobj = pobj;
  in.dobj = dobj;
  in.rel_primal = rho_p / (1.0 + norm_b);
  in.rel_dual = rho_d / (1.0 + norm_c);
  in.rel_gap = std::fabs(pobj - dobj) / (1.0 + std::fabs(pobj) + std::fabs(dobj));
  in.rel_kkt = std::max(in.rel_primal, std::max(in.rel_dual, in.rel_gap));
  in.abs_primal_inf = q[RQ_RESMAX];
}

static void kkt_from_scalars(const uc_lp* lp, const double* q, uc_lp_info& in) {
  kkt_scalars(q, lp->P.obj_offset, lp->P.norm_b, lp->P.norm_c, in);
}

// The decision parameters of a run of `o` on the data P.
static ChkParams make_params(const uc_lp_opts& o, const HostProblem& P) {
  ChkParams p;
  std::memset(&p, 0, sizeof p);
  p.mode = o.precision;
  p.K = o.kkt_every;
  p.restart_to_current = o.restart_to_current;
  p.fp32_stall_checks = o.fp32_stall_checks;
  p.iter_limit = o.iter_limit;
  p.eps_rel = o.eps_rel;
  p.eps_polish = o.eps_polish;
  p.eps_gap_rel = o.eps_gap_rel;
  p.eps_abs_feas = o.eps_abs_feas;
  p.eps_refine = o.eps_refine;
  p.restart_sufficient = o.restart_sufficient;
  p.restart_necessary = o.restart_necessary;
  p.restart_artificial = o.restart_artificial;
  p.pw_smoothing = o.pw_smoothing;
  p.pw_max_change = o.pw_max_change;
  p.pw_integral = o.pw_integral;
  p.pw_balance = o.precision == UC_LP_FP32_MIXED_POLISH ? o.pw_balance_polish : o.pw_balance;
  p.pw_balance_inner = o.pw_balance_refine;
  p.inner_diverge = o.refine_diverge;
  p.norm_b = P.norm_b;
  p.norm_c = P.norm_c;
  p.obj_offset = P.obj_offset;
  return p;
}

static ChkState fresh_state(int prec, double eta, double omega) {
  ChkState c;
  std::memset(&c, 0, sizeof c);
  c.prec = prec;
  c.status = UC_LP_RUNNING;
  c.eta = eta;
  c.omega = omega;
  return c;
}

// Run state -> the fields of uc_lp_info it determines.
static void info_from_state(const ChkState& c, uc_lp_info& in) {
  in.precision_now = c.prec == 1 ? UC_LP_FP32_MIXED : UC_LP_FP64;
  in.iters = c.iters;
  in.iters_fp64 = c.iters64;
  in.restarts = c.restarts;
  in.pobj = c.pobj;
  in.dobj = c.dobj;
  in.rel_primal = c.rel_primal;
  in.rel_dual = c.rel_dual;
  in.rel_gap = c.rel_gap;
  in.rel_kkt = c.rel_kkt;
  in.abs_primal_inf = c.abs_primal_inf;
  in.fp_residual = c.fp_residual;
  in.omega = c.omega;
  in.eta = c.eta;
  if (c.eps_reached) {
    in.pobj_at_eps = c.pobj_at_eps;
    in.rel_kkt_at_eps = c.rel_kkt_at_eps;
    in.rel_gap_at_eps = c.rel_gap_at_eps;
    in.iters_at_eps = c.iters_at_eps;
  }
}

static void print_check(const ChkState& c) {
  fprintf(stderr, "[uclp] it %lld prec %s kkt %.2e (p %.1e d %.1e g %.1e) pobj %.10g omega %.3g rfp %.3e rs %lld\n",
          (long long)c.iters, c.prec ? "fp32" : "fp64", c.rel_kkt, c.rel_primal, c.rel_dual, c.rel_gap, c.pobj,
          c.omega, c.fp_residual, (long long)c.restarts);
}

// Algorithmic bytes of one non-check half-step launch with vb-byte values:
// the matrix values and column indices, the 16-bit row ends, one read of the
// gathered vector, and per row of the block the streams its kernel touches
// (primal: xbar, x0 read and xbar written with full reflection, else x, x0
// read and x, xbar written, and c, l, u unless the block's flags supply them;
// dual: y, y0 read, y written, and b unless flagged).
static void half_step_bytes(const HostProblem& P, int vb, bool full, double* pb, double* db) {
  double p = (double)P.nnzi * (vb + 4) + 2.0 * P.ni + (double)vb * P.mi;
  for (size_t bk = 0; bk + 1 < P.t_blk.size(); ++bk) {
    const int f = P.t_flag[bk];
    const int per = (full ? 3 : 4) + !(f & kColC0) + !(f & kColUInf) + !(f & (kColL0 | kColLInf | kColLNegU));
    p += (double)(P.t_blk[bk + 1] - P.t_blk[bk]) * per * vb;
  }
  double d = (double)P.nnzi * (vb + 4) + 2.0 * P.mi + (double)vb * P.ni;
  for (size_t bk = 0; bk + 1 < P.a_blk.size(); ++bk)
    d += (double)(P.a_blk[bk + 1] - P.a_blk[bk]) * (3 + !(P.a_flag[bk] & kRowB0)) * vb;
  *pb = p;
  *db = d;
}

// The instance's info after a check whose run state is c (the engine's
// device clock dates the eps_rel milestone).
static void publish_state(uc_engine* E, uc_lp* lp, const ChkState& c, double tnow) {
  std::lock_guard<std::mutex> g(lp->mu);
  uc_lp_info& in = lp->info;
  info_from_state(c, in);
  const RefineRun& F = lp->ref;
  if (F.have_outer) {
    // refinement: the KKT fields describe the refined point, the running
    // correction problem reports its own error separately
    in.rel_kkt_inner = c.round > 0 && c.status == UC_LP_RUNNING ? c.rel_kkt : F.rel_kkt_inner;
    in.pobj = F.pobj;
    in.dobj = F.dobj;
    in.rel_primal = F.rel_primal;
    in.rel_dual = F.rel_dual;
    in.rel_gap = F.rel_gap;
    in.rel_kkt = F.rel_kkt;
    in.abs_primal_inf = F.abs_inf;
  }
  in.refine_rounds = F.round;
  in.t_total_s = tnow - lp->t_start;
  if (c.eps_reached && in.t_to_eps_s < 0 && E->tick_rate > 0)
    in.t_to_eps_s = (lp->t_stamp - lp->t_start) + (double)(int64_t)(c.tick_at_eps - lp->tick_start) / E->tick_rate;
  // report the FP32 launches when there are any (an FP32 solve that hands
  // over to FP64 near its end still reports its FP32 kernels), with the
  // algorithmic bytes of that precision
  const int tp = lp->timed_n[1] > 0 ? 1 : 0;
  if (lp->timed_n[tp] > 0) {
    in.primal_kernel_us = 1e3 * lp->timed_primal_ms[tp] / lp->timed_n[tp];
    in.dual_kernel_us = 1e3 * lp->timed_dual_ms[tp] / lp->timed_n[tp];
    in.timed_launches = lp->timed_n[tp];
  }
  const int bp = lp->timed_n[0] + lp->timed_n[1] > 0 ? tp : c.prec;
  in.primal_bytes = lp->hs_bytes[bp][0];
  in.dual_bytes = lp->hs_bytes[bp][1];
}

// ---- iterative refinement (UC_LP_FP32_REFINE) ---------------------------------
//
// At a round boundary the correction solve's FP32 point (x_hat, y_hat) is
// folded into the refined FP64 point (x*, y*) (held in the FP64 x_hat,
// y_hat), the residuals of (x*, y*) are formed and reduced in FP64, and the
// host decides: OPTIMAL when the original problem's relative KKT error at
// (x*, y*) meets eps_polish, else the next correction problem is written
// into the scaled data arrays and a fresh FP32 PDHG run starts on it from
// (0, 0).

static RefineArgs refine_args(const uc_lp* lp) {
  const DevMem& D = lp->D;
  const HostProblem& P = lp->P;
  RefineArgs R;
  std::memset((void*)&R, 0, sizeof R);
  R.a_ptr = D.a_ptr;
  R.a_col = D.a_col;
  R.t_ptr = D.t_ptr;
  R.t_col = D.t_col;
  R.a_blk = D.a_blk;
  R.t_blk = D.t_blk;
  R.a_v = D.a_v64;
  R.t_v = D.t_v64;
  R.c_in = D.c_in;
  R.b_in = D.b_in;
  R.l_in = D.l_in;
  R.u_in = D.u_in;
  R.dr = D.dr;
  R.dc = D.dc;
  R.m = P.mi;
  R.n = P.ni;
  R.m_eq = P.m_eq;
  R.a_nblk = (int)P.a_blk.size() - 1;
  R.t_nblk = (int)P.t_blk.size() - 1;
  R.inv_dp = R.inv_dd = R.dp = R.dd = 1.0;
  R.xs = D.d.xhat;
  R.ys = D.d.yhat;
  R.xc = D.f.xhat;
  R.yc = D.f.yhat;
  R.r = D.pu;
  R.d = D.pw;
  R.part_a = D.part_a;
  R.part_t = D.part_t;
  R.out = D.scal;
  R.c64 = const_cast<double*>(D.d.c);
  R.l64 = const_cast<double*>(D.d.l);
  R.u64 = const_cast<double*>(D.d.u);
  R.b64 = const_cast<double*>(D.d.b);
  R.c32 = const_cast<float*>(D.f.c);
  R.l32 = const_cast<float*>(D.f.l);
  R.u32 = const_cast<float*>(D.f.u);
  R.b32 = const_cast<float*>(D.f.b);
  R.ylo32 = D.ylo32;
  return R;
}

struct RefineFactors {
  double dp, dd, omega;
};

// D_P = min(1/||v||, growth D_P_prev) (growth D_P_prev when v = 0), D_D
// likewise; the primal weight carries over times the change of D_D / D_P.
static RefineFactors refine_factors(const double* q, double dp_prev, double dd_prev, double growth,
                                    double omega_prev) {
  const double ep = std::sqrt(std::max(q[FQ_VIOL2], 0.0));
  const double ed = std::sqrt(std::max(q[FQ_DRES2], 0.0));
  RefineFactors f;
  f.dp = ep > 0 ? std::min(1.0 / ep, growth * dp_prev) : growth * dp_prev;
  f.dd = ed > 0 ? std::min(1.0 / ed, growth * dd_prev) : growth * dd_prev;
  f.omega = omega_prev * (f.dd / f.dp) / (dd_prev / dp_prev);
  return f;
}

// Relative KKT error of the refined point on the original problem.
static void refine_outer(const double* q, const HostProblem& P, RefineRun& F) {
  const double rho_p = std::sqrt(std::max(q[FQ_VIOL2U], 0.0));
  const double rho_d = std::sqrt(std::max(q[FQ_DRES2U], 0.0));
  F.pobj = q[FQ_CX] + P.obj_offset;
  F.dobj = q[FQ_BY] + q[FQ_LBUB] + P.obj_offset;
  F.rel_primal = rho_p / (1.0 + P.norm_b);
  F.rel_dual = rho_d / (1.0 + P.norm_c);
  F.rel_gap = std::fabs(F.pobj - F.dobj) / (1.0 + std::fabs(F.pobj) + std::fabs(F.dobj));
  F.rel_kkt = std::max(F.rel_primal, std::max(F.rel_dual, F.rel_gap));
  F.abs_inf = q[FQ_VMAXU];
  F.have_outer = true;
}

// The KKT fields of the refined point to or from RefineRun::best.
static void save_best(RefineRun& F) {
  const double v[7] = {F.pobj, F.dobj, F.rel_primal, F.rel_dual, F.rel_gap, F.rel_kkt, F.abs_inf};
  std::memcpy(F.best, v, sizeof v);
  F.have_best = true;
}

static void load_best(RefineRun& F) {
  F.pobj = F.best[0];
  F.dobj = F.best[1];
  F.rel_primal = F.best[2];
  F.rel_dual = F.best[3];
  F.rel_gap = F.best[4];
  F.rel_kkt = F.best[5];
  F.abs_inf = F.best[6];
}

// The original scaled data back in the arrays a correction problem used.
static int restore_scaled_data(uc_lp* lp, hipStream_t s) {
  DevMem& D = lp->D;
  launch_scale_vectors(D.c_in, D.l_in, D.u_in, D.b_in, D.dc, D.dr, lp->P.ni, lp->P.mi, 1, (double*)D.d.c,
                       (double*)D.d.l, (double*)D.d.u, (double*)D.d.b, (float*)D.f.c, (float*)D.f.l,
                       (float*)D.f.u, (float*)D.f.b, s);
  HIPOK(hipGetLastError());
  HIPOK(hipStreamSynchronize(s));
  return UC_LP_OK;
}

// One round boundary of lp's run (stream idle).  `fold`: fold the FP32
// point of the running correction problem (or of the base solve) into
// (x*, y*) first.  `stop`: a terminal status the run ends with regardless
// (0 = none).  On return lp->chk either describes the next correction
// problem (status RUNNING) or carries the terminal status with prec = 0, so
// that the solution is read from (x*, y*).
static int refine_boundary(uc_lp* lp, hipStream_t s, bool fold, int stop) {
  RefineRun& F = lp->ref;
  ChkState& c = lp->chk;
  const uc_lp_opts& o = lp->opts;
  const HostProblem& P = lp->P;
  RefineArgs R = refine_args(lp);
  double q[FQ_N] = {};
  if (fold) {
    R.first = F.round == 0 ? 1 : 0;
    R.inv_dp = 1.0 / F.dp;
    R.inv_dd = 1.0 / F.dd;
    if (F.round > 0) F.rel_kkt_inner = c.rel_kkt;
    launch_refine_measure(R, s);
    HIPOK(hipGetLastError());
    HIPOK(hipMemcpyAsync(q, R.out, sizeof q, hipMemcpyDeviceToHost, s));
    HIPOK(hipStreamSynchronize(s));
    refine_outer(q, P, F);
    if (std::isfinite(F.rel_kkt) && (!F.have_best || F.rel_kkt < F.best[5])) {
      HIPOK(hipMemcpyAsync(lp->D.x_warm, lp->D.d.xhat, sizeof(double) * P.ni, hipMemcpyDeviceToDevice, s));
      if (P.mi)
        HIPOK(hipMemcpyAsync(lp->D.y_warm, lp->D.d.yhat, sizeof(double) * P.mi, hipMemcpyDeviceToDevice, s));
      save_best(F);
    }
    if (!c.eps_reached && F.rel_kkt <= o.eps_rel && (o.eps_abs_feas <= 0 || F.abs_inf <= o.eps_abs_feas)) {
      // the eps_rel milestone, reached by the refined point (host clock)
      c.eps_reached = 1;
      c.iters_at_eps = c.iters;
      c.pobj_at_eps = F.pobj;
      c.rel_kkt_at_eps = F.rel_kkt;
      c.rel_gap_at_eps = F.rel_gap;
      std::lock_guard<std::mutex> g(lp->mu);
      lp->info.t_to_eps_s = now_s() - lp->t_start;
    }
    if (o.verbose)
      fprintf(stderr, "[uclp] refine boundary %d at it %lld: kkt %.2e (p %.1e d %.1e g %.1e) pobj %.12g inner %.2e\n",
              F.round, (long long)c.iters, F.rel_kkt, F.rel_primal, F.rel_dual, F.rel_gap, F.pobj,
              F.round > 0 ? c.rel_kkt : 0.0);
  }
  int status = stop;
  if (status == 0) {
    const bool feas = o.eps_abs_feas <= 0 || F.abs_inf <= o.eps_abs_feas;
    if (!std::isfinite(F.rel_kkt)) status = UC_LP_NUMERICAL;
    else if (F.rel_kkt <= o.eps_polish && feas) status = UC_LP_OPTIMAL;
    else if (c.iters >= o.iter_limit || F.round >= o.refine_max_rounds) status = UC_LP_ITER_LIMIT;
  }
  if (status != 0) {
    c.status = status;
    c.promote = 0;
    if (status != UC_LP_OPTIMAL && F.have_best && !(F.rel_kkt <= F.best[5])) {
      // the run ends short of its target on a point worse than an earlier one
      HIPOK(hipMemcpyAsync(lp->D.d.xhat, lp->D.x_warm, sizeof(double) * P.ni, hipMemcpyDeviceToDevice, s));
      if (P.mi)
        HIPOK(hipMemcpyAsync(lp->D.d.yhat, lp->D.y_warm, sizeof(double) * P.mi, hipMemcpyDeviceToDevice, s));
      load_best(F);
      if (o.verbose) fprintf(stderr, "[uclp] refine: returning the best refined point, kkt %.2e\n", F.rel_kkt);
    }
    if (F.have_outer) c.prec = 0;  // the answer is (x*, y*)
    return restore_scaled_data(lp, s);
  }
  const RefineFactors f = refine_factors(q, F.dp, F.dd, o.refine_growth, c.omega);
  R.dp = f.dp;
  R.dd = f.dd;
  launch_refine_form(R, s);
  launch_init_iterates(lp->D.slot_dev, 1, nullptr, nullptr, P.ni, P.mi, P.m_eq, 1, s);
  HIPOK(hipGetLastError());
  HIPOK(hipStreamSynchronize(s));
  if (F.round == 0) {
    // tiles of the correction problems: infinite bounds stay infinite, no
    // other column value is known per block, and inequality duals are
    // bounded by ylo
    F.t_flag = P.t_flag;
    for (int& v : F.t_flag) v &= (kColLInf | kColUInf);
    F.a_flag.assign(P.a_flag.size(), kRowYlo);
  }
  if (o.verbose)
    fprintf(stderr, "[uclp] refine round %d: D_P %.3e D_D %.3e omega %.3e\n", F.round + 1, f.dp, f.dd, f.omega);
  F.dp = f.dp;
  F.dd = f.dd;
  ++F.round;
  // The correction problem's KKT error, measured on the scale of the refined
  // point it corrects: its residuals are D_P, D_D times those of
  // (x* + x~/D_P, y* + y~/D_D), and its duality gap D_P D_D times that
  // point's gap up to terms that vanish with the residuals.  So the check
  // normalises by D_P (1 + ||b||), D_D (1 + ||c||) and D_P D_D (1 + |pobj*|
  // + |dobj*|), and a round ends once this estimate of the refined point's
  // error has fallen to eps_refine times its value at the boundary (or to
  // eps_polish).
  lp->prm.norm_b = f.dp * (1.0 + P.norm_b) - 1.0;
  lp->prm.norm_c = f.dd * (1.0 + P.norm_c) - 1.0;
  lp->prm.gap_den = f.dp * f.dd * (1.0 + std::fabs(F.pobj) + std::fabs(F.dobj));
  lp->prm.eps_refine = std::max(o.eps_polish, o.eps_refine * F.rel_kkt);
  // before the refined point has met eps_rel, a round ends as soon as its
  // estimate says so, and the boundary dates the milestone
  if (!c.eps_reached) lp->prm.eps_refine = std::max(lp->prm.eps_refine, o.eps_rel);
  lp->prm.obj_offset = 0.0;
  // PDHG on the correction problem from (0, 0) takes the steps PDHG on the
  // original problem would take from (x*, y*) (in exact arithmetic): the run
  // continues as after a restart there.  The phase's step count carries on,
  // so the artificial restart rule does not fire again at once, and so do
  // the iteration counts and the eps_rel milestone.
  c.round = F.round;
  c.omega = f.omega;
  c.prec = 1;
  c.status = UC_LP_RUNNING;
  c.promote = 0;
  c.restart = 0;
  c.k_inner = 0;
  c.r_start_set = 0;
  c.r_prev_set = 0;
  c.gap_phase = 0;
  c.best_check = 0;
  c.best_kkt = 0;
  c.pw_int = 0;
  return UC_LP_OK;
}

// ---- engine worker -----------------------------------------------------------
//
// The worker admits queued instances, builds the tile layout of the active
// set and then runs epochs of K iterations with no host round-trip: each
// epoch ends with the FP64 check kernels, a check kernel that takes every
// instance's restart / primal-weight / termination decision on the device
// (one thread per instance, state in d_chk), the finish kernels, and an
// asynchronous copy of the run states into a pinned ring.  The next epoch is
// already enqueued when the worker reads an epoch's states.  An instance
// whose run ends (or that switches precision) is frozen by the check kernel,
// so later launches skip its tiles; the worker then drains the stream and
// retires, promotes and admits before it rebuilds the layout.

static int engine_tables(uc_engine* E, size_t ntiles) {
  if (ntiles > E->tile_cap) {
    if (E->d_tiles) (void)hipFree(E->d_tiles);
    E->d_tiles = nullptr;
    size_t cap = std::max<size_t>(ntiles, 2 * E->tile_cap);
    HIPOK(hipMalloc(&E->d_tiles, cap * sizeof(Tile)));
    E->tile_cap = cap;
  }
  return UC_LP_OK;
}

static void worker_fail(uc_engine* E, uc_lp* lp) {
  {
    std::lock_guard<std::mutex> g(lp->mu);
    lp->info.status = UC_LP_FAILED;
  }
  std::fprintf(stderr, "[uclp] solve failed: %s\n", g_err.c_str());
  E->err = g_err;
  lp->status.store(UC_LP_FAILED);
  lp->done_cv.notify_all();
}

static void start_instance(uc_engine* E, uc_lp* lp) {
  const double t0 = now_s();
  lp->t_start = t0;
  lp->host_stop = 0;
  for (int p = 0; p < 2; ++p) {
    lp->timed_primal_ms[p] = lp->timed_dual_ms[p] = 0;
    lp->timed_n[p] = 0;
  }
  {
    std::lock_guard<std::mutex> g(lp->mu);
    uc_lp_info in;
    std::memset(&in, 0, sizeof in);
    in.status = UC_LP_RUNNING;
    in.t_to_eps_s = -1;
    in.t_queue_s = t0 - lp->t_request;
    in.m_presolved = lp->P.mi;
    in.n_presolved = lp->P.ni;
    in.nnz_presolved = lp->P.nnzi;
    in.device_bytes = (int64_t)lp->need_bytes;
    lp->info = in;
  }
  lp->status.store(UC_LP_RUNNING);
  if (lp->P.infeasible) {
    finish_status(lp, UC_LP_INFEASIBLE);
    return;
  }
  int rc = UC_LP_OK;
  if (!lp->uploaded) rc = upload(lp);
  if (rc == UC_LP_OK) rc = setup_device(lp);
  const int prec = lp->opts.precision == UC_LP_FP64 ? 0 : 1;
  lp->chk = fresh_state(prec, lp->chk.eta, lp->chk.omega);
  lp->ref = RefineRun();
  lp->prm = make_params(lp->opts, lp->P);
  for (int p = 0; p < 2; ++p)
    half_step_bytes(lp->P, p ? 4 : 8, lp->opts.halpern_gamma == 1.0, &lp->hs_bytes[p][0], &lp->hs_bytes[p][1]);
  if (rc == UC_LP_OK) rc = init_iterates(lp, prec);
  if (rc == UC_LP_OK) {
    // device clock at the start of the iterations (the stream is idle here)
    launch_stamp(lp->D.tick, E->stream);
    unsigned long long tk = 0;
    hipError_t e = hipMemcpyAsync(&tk, lp->D.tick, sizeof tk, hipMemcpyDeviceToHost, E->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(E->stream);
    if (e != hipSuccess) rc = fail(UC_LP_EHIP, "clock stamp: %s", hipGetErrorString(e));
    lp->tick_start = tk;
    lp->t_stamp = now_s();
  }
  if (rc != UC_LP_OK) {
    worker_fail(E, lp);
    return;
  }
  {
    std::lock_guard<std::mutex> g(lp->mu);
    lp->info.t_setup_s = now_s() - t0;
    lp->info.omega = lp->chk.omega;
    lp->info.eta = lp->chk.eta;
  }
  E->active.push_back(lp);
  E->layout_valid = false;
}

static void retire(uc_engine* E, uc_lp* lp, int status) {
  int rc = fetch_solution(lp, lp->chk.prec);
  if (!E->private_engine) {
    release(lp);
    std::lock_guard<std::mutex> g(E->mu);
    E->used -= lp->need_bytes;
  }
  {
    std::lock_guard<std::mutex> g(lp->mu);
    lp->info.t_total_s = now_s() - lp->t_start;
  }
  if (rc != UC_LP_OK) worker_fail(E, lp);
  else finish_status(lp, status);
}

static void fail_all(uc_engine* E, const char* what, hipError_t e) {
  fail(UC_LP_EHIP, "%s: %s", what, hipGetErrorString(e));
  for (auto* lp : E->active) worker_fail(E, lp);
  E->active.clear();
  E->layout_valid = false;
}

// Slot table, tiles, run states and parameters of the active set.  Called
// with nothing in flight.
static hipError_t build_layout(uc_engine* E) {
  hipStream_t s = E->stream;
  const int A = (int)E->active.size();
  int K = 1 << 30;
  bool timing = false;
  for (auto* lp : E->active) {
    K = std::min(K, lp->opts.kkt_every);
    timing |= lp->opts.timing != 0;
  }
  E->K = K;
  E->timing = timing;
  std::vector<Tile> tt[2], at[2];
  std::vector<int> ids(A);
  std::vector<ChkState> chk(A);
  std::vector<ChkParams> prm(A);
  for (int a = 0; a < A; ++a) {
    uc_lp* lp = E->active[a];
    lp->slot = a;
    ids[a] = a;
    const int p = lp->chk.prec;
    const bool corr = lp->ref.round > 0;  // correction data loaded (refinement)
    push_tiles(tt[p], a, lp->P.t_blk, lp->P.t_ptr, corr ? &lp->ref.t_flag : &lp->P.t_flag, &lp->P.t_base);
    push_tiles(at[p], a, lp->P.a_blk, lp->P.a_ptr, corr ? &lp->ref.a_flag : &lp->P.a_flag, &lp->P.a_base);
    SlotDev S = make_slot(lp);
    S.scal = E->d_scal + (size_t)a * kScal;
    S.tau[0] = lp->chk.eta / lp->chk.omega;
    S.sigma[0] = lp->chk.eta * lp->chk.omega;
    S.k0[0] = lp->chk.k_inner;
    S.restart[0] = 0;
    S.active[0] = 1;
    E->h_slots[a] = S;
    chk[a] = lp->chk;
    prm[a] = lp->prm;
    prm[a].K = K;
  }
  E->nT1 = (int)tt[1].size();
  E->nT0 = (int)tt[0].size();
  E->nA1 = (int)at[1].size();
  E->nA0 = (int)at[0].size();
  E->off_t0 = tt[1].size();
  E->off_a1 = E->off_t0 + tt[0].size();
  E->off_a0 = E->off_a1 + at[1].size();
  const size_t total = E->off_a0 + at[0].size();
  if (engine_tables(E, total) != UC_LP_OK) return hipErrorOutOfMemory;
  std::vector<Tile> all;
  all.reserve(total);
  all.insert(all.end(), tt[1].begin(), tt[1].end());
  all.insert(all.end(), tt[0].begin(), tt[0].end());
  all.insert(all.end(), at[1].begin(), at[1].end());
  all.insert(all.end(), at[0].begin(), at[0].end());
  hipError_t e = hipSuccess;
  if (total) e = hipMemcpyAsync(E->d_tiles, all.data(), total * sizeof(Tile), hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipMemcpyAsync(E->d_ids, ids.data(), A * sizeof(int), hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipMemcpyAsync(E->d_slots, E->h_slots, A * sizeof(SlotDev), hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipMemcpyAsync(E->d_chk, chk.data(), A * sizeof(ChkState), hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipMemcpyAsync(E->d_prm, prm.data(), A * sizeof(ChkParams), hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);  // the host vectors die at scope end
  E->layout_valid = e == hipSuccess;
  return e;
}

// One epoch of K iterations over the active set, its check and the copy of
// the run states into ring entry r.
static void enqueue_epoch(uc_engine* E, int r) {
  hipStream_t s = E->stream;
  const int A = (int)E->active.size(), K = E->K;
  const Tile* T1 = E->d_tiles;
  const Tile* T0 = E->d_tiles + E->off_t0;
  const Tile* A1 = E->d_tiles + E->off_a1;
  const Tile* A0 = E->d_tiles + E->off_a0;
  const int nT1 = E->nT1, nT0 = E->nT0, nA1 = E->nA1, nA0 = E->nA0;
  hipEvent_t* ev = E->tev[r];
  for (int j = 0; j < K; ++j) {
    const bool check = j == K - 1;
    // the middle iteration carries dispatch-attached timing events on the
    // first non-empty precision group
    const bool tj = E->timing && j == K / 2;
    const bool t1 = tj && nT1 > 0, t0 = tj && nT1 == 0;
    launch_primal(1, check, E->d_slots, T1, nT1, j, 1, s, t1 ? ev[0] : nullptr, t1 ? ev[1] : nullptr);
    launch_primal(0, check, E->d_slots, T0, nT0, j, 1, s, t0 ? ev[0] : nullptr, t0 ? ev[1] : nullptr);
    launch_dual(1, check, E->d_slots, A1, nA1, j, 1, s, t1 ? ev[2] : nullptr, t1 ? ev[3] : nullptr);
    launch_dual(0, check, E->d_slots, A0, nA0, j, 1, s, t0 ? ev[2] : nullptr, t0 ? ev[3] : nullptr);
  }
  launch_kkt(1, E->d_slots, T1, nT1, A1, nA1, 1, s);
  launch_kkt(0, E->d_slots, T0, nT0, A0, nA0, 1, s);
  launch_reduce(E->d_slots, E->d_ids, A, 1, E->d_red2, s);
  launch_engine_check(E->d_slots, E->d_chk, E->d_prm, A, s);
  launch_finish(1, E->d_slots, T1, nT1, A1, nA1, 0, 1, s);
  launch_finish(0, E->d_slots, T0, nT0, A0, nA0, 0, 1, s);
  (void)hipMemcpyAsync(E->h_ring + (size_t)r * E->max_slots, E->d_chk, A * sizeof(ChkState), hipMemcpyDeviceToHost,
                       s);
  (void)hipEventRecord(E->ring_ev[r], s);
}

// Reads ring entry r (its epoch has completed): publishes every instance's
// state and timing; true when the active set has to change (a run ended or
// switches precision, the host stops one, a queued request fits, shutdown).
static bool process_epoch(uc_engine* E, int r) {
  const int A = (int)E->active.size();
  const double tnow = now_s();
  if (E->timing) {
    float t01 = 0, t23 = 0;
    if (hipEventElapsedTime(&t01, E->tev[r][0], E->tev[r][1]) == hipSuccess &&
        hipEventElapsedTime(&t23, E->tev[r][2], E->tev[r][3]) == hipSuccess) {
      const int tp = E->nT1 > 0 ? 1 : 0;  // the group that carried the events
      for (auto* lp : E->active)
        if (lp->opts.timing) {
          lp->timed_primal_ms[tp] += t01;
          lp->timed_dual_ms[tp] += t23;
          ++lp->timed_n[tp];
        }
    }
  }
  bool change = false;
  for (int a = 0; a < A; ++a) {
    uc_lp* lp = E->active[a];
    const ChkState& c = E->h_ring[(size_t)r * E->max_slots + a];
    publish_state(E, lp, c, tnow);
    if (lp->opts.verbose) print_check(c);
    if (c.status != UC_LP_RUNNING || c.promote) change = true;
    if (lp->cancel.load()) {
      lp->host_stop = UC_LP_CANCELLED;
      change = true;
    } else if (tnow - lp->t_start >= lp->opts.time_limit_s) {
      lp->host_stop = UC_LP_TIME_LIMIT;
      change = true;
    }
  }
  std::lock_guard<std::mutex> g(E->mu);
  if (E->shutdown) change = true;
  if (!E->queue.empty() && (int)E->active.size() < E->max_slots &&
      (E->private_engine || E->used + E->queue.front()->need_bytes <= E->budget))
    change = true;
  return change;
}

// Epochs until the active set has to change, then a drain: every instance's
// device state is read back; finished runs retire, FP32 runs that reached
// their hand-over switch to FP64 (promote kernels), host-stopped runs end.
static void run_epochs(uc_engine* E) {
  hipStream_t s = E->stream;
  if (!E->layout_valid) {
    const hipError_t e = build_layout(E);
    if (e != hipSuccess) return fail_all(E, "layout upload", e);
  }
  long long issued = 0, done = 0;
  bool change = false;
  while (!change) {
    while (issued - done < kRing) enqueue_epoch(E, (int)(issued++ % kRing));
    const hipError_t e = hipEventSynchronize(E->ring_ev[done % kRing]);
    if (e != hipSuccess) return fail_all(E, "epoch", e);
    change = process_epoch(E, (int)(done++ % kRing));
  }
  const int A = (int)E->active.size();
  std::vector<ChkState> chk(A);
  hipError_t e = hipMemcpyAsync(chk.data(), E->d_chk, A * sizeof(ChkState), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e == hipSuccess) e = hipGetLastError();
  if (e != hipSuccess) return fail_all(E, "epoch", e);
  const double tnow = now_s();
  std::vector<Tile> pt, pa;
  for (int a = 0; a < A; ++a) {
    uc_lp* lp = E->active[a];
    lp->chk = chk[a];
    publish_state(E, lp, chk[a], tnow);
    if (lp->opts.precision == UC_LP_FP32_REFINE) {
      // a round boundary of iterative refinement, or the end of a run that
      // is inside a correction problem (its point is folded in unless it
      // went non-finite)
      const int dev = lp->chk.status;
      int rc = UC_LP_OK;
      if (dev == UC_LP_RUNNING && lp->chk.promote && !lp->host_stop) {
        rc = refine_boundary(lp, s, true, 0);
      } else if (lp->ref.round > 0 && (dev != UC_LP_RUNNING || lp->host_stop)) {
        const int st = dev != UC_LP_RUNNING ? dev : lp->host_stop;
        rc = refine_boundary(lp, s, st != UC_LP_NUMERICAL, st);
      }
      if (rc != UC_LP_OK) {
        std::fprintf(stderr, "[uclp] refinement step failed: %s\n", g_err.c_str());
        lp->chk.status = UC_LP_FAILED;
      }
      publish_state(E, lp, lp->chk, now_s());
      continue;
    }
    if (lp->chk.status == UC_LP_RUNNING && lp->chk.promote && !lp->host_stop) {
      // FP32 x_hat, y_hat -> FP64 iterates of the same slot
      push_tiles(pt, a, lp->P.t_blk, lp->P.t_ptr);
      push_tiles(pa, a, lp->P.a_blk, lp->P.a_ptr);
      lp->chk.promote = 0;
    }
  }
  E->layout_valid = false;
  if (!pt.empty() || !pa.empty()) {
    std::vector<Tile> both = pt;
    both.insert(both.end(), pa.begin(), pa.end());
    if (engine_tables(E, both.size()) != UC_LP_OK) return fail_all(E, "promote tiles", hipErrorOutOfMemory);
    e = hipMemcpyAsync(E->d_tiles, both.data(), both.size() * sizeof(Tile), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) launch_promote(E->d_slots, E->d_tiles, (int)pt.size(), E->d_tiles + pt.size(), (int)pa.size(), 1, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return fail_all(E, "promote", e);
  }
  std::vector<uc_lp*> keep;
  for (auto* lp : E->active) {
    const int st = lp->chk.status != UC_LP_RUNNING ? lp->chk.status : lp->host_stop;
    if (st != 0 && st != UC_LP_RUNNING) retire(E, lp, st);
    else keep.push_back(lp);
  }
  E->active.swap(keep);
}

static void worker_main(uc_engine* E) {
  (void)hipSetDevice(E->device);
  for (;;) {
    std::vector<uc_lp*> admit;
    {
      std::unique_lock<std::mutex> g(E->mu);
      if (E->active.empty())
        E->cv.wait(g, [&] { return E->shutdown || !E->queue.empty(); });
      if (E->shutdown && E->queue.empty() && E->active.empty()) break;
      // drop cancelled queued requests
      for (auto it = E->queue.begin(); it != E->queue.end();) {
        if ((*it)->cancel.load()) {
          uc_lp* lp = *it;
          it = E->queue.erase(it);
          if (!E->private_engine) E->used -= lp->need_bytes;
          g.unlock();
          finish_status(lp, UC_LP_CANCELLED);
          g.lock();
        } else {
          ++it;
        }
      }
      while (!E->queue.empty() && (int)(E->active.size() + admit.size()) < E->max_slots) {
        uc_lp* lp = E->queue.front();
        if (!E->private_engine && E->used + lp->need_bytes > E->budget) break;
        if (!E->private_engine) E->used += lp->need_bytes;
        E->queue.pop_front();
        admit.push_back(lp);
      }
      if (E->shutdown) {
        for (auto* lp : E->active) lp->cancel.store(true);
      }
    }
    for (auto* lp : admit) start_instance(E, lp);
    if (!E->active.empty()) run_epochs(E);
  }
}

// ---------------------------------------------------------------------------
// C ABI: engine
// ---------------------------------------------------------------------------

static int engine_init(uc_engine* E) {
  HIPOK(hipSetDevice(E->device));
  HIPOK(hipStreamCreate(&E->stream));
  HIPOK(hipMalloc(&E->d_slots, sizeof(SlotDev) * E->max_slots));
  HIPOK(hipMalloc(&E->d_ids, sizeof(int) * E->max_slots));
  HIPOK(hipHostMalloc((void**)&E->h_slots, sizeof(SlotDev) * E->max_slots, hipHostMallocDefault));
  HIPOK(hipHostMalloc((void**)&E->h_ring, sizeof(ChkState) * kRing * E->max_slots, hipHostMallocDefault));
  HIPOK(hipMalloc(&E->d_scal, sizeof(double) * kScal * E->max_slots));
  HIPOK(hipMalloc(&E->d_red2, sizeof(double) * kRedChunks * (RQ_N + CQ_N) * E->max_slots));
  HIPOK(hipMalloc(&E->d_chk, sizeof(ChkState) * E->max_slots));
  HIPOK(hipMalloc(&E->d_prm, sizeof(ChkParams) * E->max_slots));
  for (int r = 0; r < kRing; ++r) {
    HIPOK(hipEventCreate(&E->ring_ev[r]));
    for (auto& ev : E->tev[r]) HIPOK(hipEventCreate(&ev));
  }
  int khz = 0;
  HIPOK(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, E->device));
  E->tick_rate = 1e3 * (double)khz;
  E->worker = std::thread(worker_main, E);
  return UC_LP_OK;
}

static void engine_free(uc_engine* E) {
  if (!E) return;
  {
    std::lock_guard<std::mutex> g(E->mu);
    E->shutdown = true;
  }
  E->cv.notify_all();
  if (E->worker.joinable()) E->worker.join();
  (void)hipSetDevice(E->device);
  for (void* p : {(void*)E->d_slots, (void*)E->d_ids, (void*)E->d_tiles, (void*)E->d_scal, (void*)E->d_red2,
                  (void*)E->d_chk, (void*)E->d_prm})
    if (p) (void)hipFree(p);
  if (E->h_slots) (void)hipHostFree(E->h_slots);
  if (E->h_ring) (void)hipHostFree(E->h_ring);
  for (int r = 0; r < kRing; ++r) {
    if (E->ring_ev[r]) (void)hipEventDestroy(E->ring_ev[r]);
    for (auto ev : E->tev[r])
      if (ev) (void)hipEventDestroy(ev);
  }
  if (E->stream) (void)hipStreamDestroy(E->stream);
  delete E;
}

extern "C" int uc_engine_create(int device, size_t hbm_budget_bytes, int32_t max_slots, uc_engine** out) {
  g_err.clear();
  if (!out) return fail(UC_LP_EINVAL, "out is NULL");
  *out = nullptr;
  if (max_slots < 1 || max_slots > 1024) return fail(UC_LP_EINVAL, "max_slots %d not in 1..1024", max_slots);
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || count <= 0) return fail(UC_LP_EHIP, "no HIP device");
  if (device < 0 || device >= count) return fail(UC_LP_EINVAL, "device %d of %d", device, count);
  uc_engine* E = new (std::nothrow) uc_engine();
  if (!E) return fail(UC_LP_ENOMEM, "engine allocation");
  E->device = device;
  E->max_slots = max_slots;
  if (hipSetDevice(device) != hipSuccess) {
    delete E;
    return fail(UC_LP_EHIP, "hipSetDevice");
  }
  size_t fr = 0, tot = 0;
  (void)hipMemGetInfo(&fr, &tot);
  E->budget = hbm_budget_bytes ? hbm_budget_bytes : (size_t)(0.9 * (double)fr);
  int rc = engine_init(E);
  if (rc != UC_LP_OK) {
    engine_free(E);
    return rc;
  }
  *out = E;
  return UC_LP_OK;
}

extern "C" void uc_engine_destroy(uc_engine* eng) {
  if (!eng) return;
  {
    std::lock_guard<std::mutex> g(eng->mu);
    for (auto* lp : eng->queue) lp->cancel.store(true);
    for (auto* lp : eng->active) lp->cancel.store(true);
  }
  engine_free(eng);
}

// ---------------------------------------------------------------------------
// C ABI: instances
// ---------------------------------------------------------------------------

extern "C" int uc_lp_create(uc_engine* eng, int32_t m, int32_t n, int64_t nnz, const int32_t* row_ptr,
                            const int32_t* col_idx, const double* val, const double* c, const double* b,
                            const char* sense, const double* lb, const double* ub, const uc_lp_opts* opts,
                            uc_lp** out) {
  g_err.clear();
  if (!out) return fail(UC_LP_EINVAL, "out is NULL");
  *out = nullptr;
  uc_lp_opts o;
  uc_lp_opts_default(&o);
  if (opts) o = *opts;
  int rc = check_opts(o);
  if (rc) return rc;
  if ((rc = validate_csr(m, n, nnz, row_ptr, col_idx, val))) return rc;
  if ((rc = validate_data(m, n, c, b, sense, lb, ub))) return rc;
  std::unique_ptr<uc_lp> lp(new (std::nothrow) uc_lp());
  if (!lp) return fail(UC_LP_ENOMEM, "instance allocation");
  lp->opts = o;
  HostProblem& P = lp->P;
  P.m = m;
  P.n = n;
  P.nnz = nnz;
  P.o_ptr.assign(row_ptr, row_ptr + m + 1);
  P.o_col.assign(col_idx, col_idx + nnz);
  P.o_val.assign(val, val + nnz);
  P.o_c.assign(c, c + n);
  P.o_b.assign(b, b + m);
  P.o_sense.assign(sense, sense + m);
  P.o_lb.assign(lb, lb + n);
  P.o_ub.assign(ub, ub + n);
  presolve_structure(P);
  presolve_data(P, P);
  if (P.ni == 0) return fail(UC_LP_ENOTSUP, "every column is fixed; nothing to solve");
  if (P.mi == 0) return fail(UC_LP_ENOTSUP, "no row has an entry in a free column; nothing for PDHG to solve");
  lp->need_bytes = arena_bytes(P, 1);
  std::memset(&lp->info, 0, sizeof lp->info);
  lp->info.t_to_eps_s = -1;
  lp->info.m_presolved = P.mi;
  lp->info.n_presolved = P.ni;
  lp->info.nnz_presolved = P.nnzi;
  lp->info.device_bytes = (int64_t)lp->need_bytes;
  if (eng) {
    if (lp->need_bytes > eng->budget)
      return fail(UC_LP_EBUDGET, "instance needs %zu bytes, engine budget is %zu", lp->need_bytes, eng->budget);
    lp->eng = eng;
  } else {
    uc_engine* E = nullptr;
    rc = uc_engine_create(0, 0, 1, &E);
    if (rc) return rc;
    E->private_engine = true;
    lp->eng = E;
    lp->owns_engine = true;
    rc = upload(lp.get());
    if (rc) {
      uc_engine_destroy(E);
      return rc;
    }
  }
  *out = lp.release();
  return UC_LP_OK;
}

extern "C" int uc_lp_update_data(uc_lp* lp, const double* c, const double* b, const double* lb,
                                 const double* ub) {
  g_err.clear();
  if (!lp) return fail(UC_LP_EINVAL, "NULL handle");
  const int s = lp->status.load();
  if (s == UC_LP_QUEUED || s == UC_LP_RUNNING) return fail(UC_LP_ESTATE, "solve in progress");
  HostProblem& P = lp->P;
  std::vector<double> nc = c ? std::vector<double>(c, c + P.n) : P.o_c;
  std::vector<double> nb = b ? std::vector<double>(b, b + P.m) : P.o_b;
  std::vector<double> nl = lb ? std::vector<double>(lb, lb + P.n) : P.o_lb;
  std::vector<double> nu = ub ? std::vector<double>(ub, ub + P.n) : P.o_ub;
  int rc = validate_data(P.m, P.n, nc.data(), nb.data(), P.o_sense.data(), nl.data(), nu.data());
  if (rc) return rc;
  for (int32_t j = 0; j < P.n; ++j)
    if ((nl[j] == nu[j]) != (P.int_col[j] < 0))
      return fail(UC_LP_ENOTSUP, "column %d changes between fixed and free; create a new instance", j);
  P.o_c.swap(nc);
  P.o_b.swap(nb);
  P.o_lb.swap(nl);
  P.o_ub.swap(nu);
  presolve_data(P, P);
  ++lp->data_gen;
  lp->setup_done = false;
  return UC_LP_OK;
}

extern "C" int uc_lp_solve(uc_lp* lp, const double* x0, const double* y0) {
  g_err.clear();
  if (!lp) return fail(UC_LP_EINVAL, "NULL handle");
  const int s = lp->status.load();
  if (s == UC_LP_QUEUED || s == UC_LP_RUNNING) return fail(UC_LP_ESTATE, "solve already in progress");
  HostProblem& P = lp->P;
  lp->has_warm = x0 || y0;
  if (lp->has_warm) {
    lp->warm_x.assign(P.ni, 0.0);
    lp->warm_y.assign(P.mi, 0.0);
    if (x0)
      for (int j = 0; j < P.ni; ++j) lp->warm_x[j] = x0[P.col_map[j]];
    if (y0)
      for (int i = 0; i < P.mi; ++i) {
        const int enc = P.row_map[i];
        lp->warm_y[i] = enc >= 0 ? y0[enc] : -y0[-enc - 1];
      }
    for (double v : lp->warm_x)
      if (!std::isfinite(v)) return fail(UC_LP_EINVAL, "non-finite warm start");
    for (double v : lp->warm_y)
      if (!std::isfinite(v)) return fail(UC_LP_EINVAL, "non-finite warm start");
  }
  lp->cancel.store(false);
  lp->t_request = now_s();
  uc_engine* E = lp->eng;
  {
    std::lock_guard<std::mutex> g(lp->mu);
    lp->info.status = UC_LP_QUEUED;
    lp->info.t_to_eps_s = -1;
  }
  lp->status.store(UC_LP_QUEUED);
  {
    std::lock_guard<std::mutex> g(E->mu);
    E->queue.push_back(lp);
  }
  E->cv.notify_all();
  return UC_LP_OK;
}

extern "C" int uc_lp_status(const uc_lp* lp, uc_lp_info* out) {
  g_err.clear();
  if (!lp || !out) return fail(UC_LP_EINVAL, "NULL argument");
  *out = get_info(lp);
  out->status = lp->status.load();
  if (out->status == UC_LP_RUNNING && lp->t_start > 0) out->t_total_s = now_s() - lp->t_start;
  return UC_LP_OK;
}

extern "C" int uc_lp_wait(uc_lp* lp, double timeout_s) {
  g_err.clear();
  if (!lp) return fail(UC_LP_EINVAL, "NULL handle");
  std::unique_lock<std::mutex> g(lp->mu);
  auto pending = [&] {
    const int s = lp->status.load();
    return s == UC_LP_QUEUED || s == UC_LP_RUNNING;
  };
  if (timeout_s < 0) {
    lp->done_cv.wait(g, [&] { return !pending(); });
    return UC_LP_OK;
  }
  if (!lp->done_cv.wait_for(g, std::chrono::duration<double>(timeout_s), [&] { return !pending(); }))
    return fail(UC_LP_ETIMEOUT, "wait timed out");
  return UC_LP_OK;
}

extern "C" int uc_lp_cancel(uc_lp* lp) {
  g_err.clear();
  if (!lp) return fail(UC_LP_EINVAL, "NULL handle");
  lp->cancel.store(true);
  lp->eng->cv.notify_all();
  return UC_LP_OK;
}

extern "C" int uc_lp_get_solution(const uc_lp* lp, double* x, double* y) {
  g_err.clear();
  if (!lp) return fail(UC_LP_EINVAL, "NULL handle");
  const int s = lp->status.load();
  if (!(s == UC_LP_OPTIMAL || s == UC_LP_ITER_LIMIT || s == UC_LP_TIME_LIMIT || s == UC_LP_CANCELLED ||
        s == UC_LP_NUMERICAL))
    return fail(UC_LP_ESTATE, "no solution in status %d", s);
  if (lp->sol_x.size() != (size_t)lp->P.n) return fail(UC_LP_ESTATE, "solution not available");
  if (x) std::memcpy(x, lp->sol_x.data(), sizeof(double) * lp->P.n);
  if (y) std::memcpy(y, lp->sol_y.data(), sizeof(double) * lp->P.m);
  return UC_LP_OK;
}

extern "C" void uc_lp_destroy(uc_lp* lp) {
  if (!lp) return;
  lp->cancel.store(true);
  uc_engine* E = lp->eng;
  E->cv.notify_all();
  {
    std::unique_lock<std::mutex> g(lp->mu);
    lp->done_cv.wait(g, [&] {
      const int s = lp->status.load();
      return s != UC_LP_QUEUED && s != UC_LP_RUNNING;
    });
  }
  if (lp->owns_engine) {
    engine_free(E);  // joins the worker before the instance memory goes
    (void)hipSetDevice(0);
    release(lp);
  } else {
    (void)hipSetDevice(E->device);
    if (lp->uploaded) {
      release(lp);
    }
  }
  delete lp;
}

extern "C" const char* uc_lp_last_error(void) { return g_err.c_str(); }

// ---------------------------------------------------------------------------
// step-level entry points
// ---------------------------------------------------------------------------

static int debug_ready(uc_lp* lp) {
  if (!lp) return fail(UC_LP_EINVAL, "NULL handle");
  if (!lp->owns_engine) return fail(UC_LP_ESTATE, "step-level calls need a handle created with eng == NULL");
  const int s = lp->status.load();
  if (s == UC_LP_QUEUED || s == UC_LP_RUNNING) return fail(UC_LP_ESTATE, "solve in progress");
  HIPOK(hipSetDevice(lp->eng->device));
  if (!lp->uploaded) {
    int rc = upload(lp);
    if (rc) return rc;
  }
  if (!lp->setup_done) return setup_device(lp);
  return UC_LP_OK;
}

extern "C" int uc_lp_internal_dims(uc_lp* lp, int32_t* m_int, int32_t* n_int, int64_t* nnz_int, int32_t* m_eq,
                                   int32_t* row_map, int32_t* col_map) {
  g_err.clear();
  if (!lp) return fail(UC_LP_EINVAL, "NULL handle");
  const HostProblem& P = lp->P;
  if (m_int) *m_int = P.mi;
  if (n_int) *n_int = P.ni;
  if (nnz_int) *nnz_int = P.nnzi;
  if (m_eq) *m_eq = P.m_eq;
  if (row_map) std::memcpy(row_map, P.row_map.data(), sizeof(int) * P.mi);
  if (col_map) std::memcpy(col_map, P.col_map.data(), sizeof(int) * P.ni);
  return UC_LP_OK;
}

extern "C" int uc_lp_get_transpose(uc_lp* lp, int32_t* t_row_ptr, int32_t* t_col, double* t_val) {
  g_err.clear();
  int rc = debug_ready(lp);
  if (rc) return rc;
  hipStream_t s = lp->eng->stream;
  const HostProblem& P = lp->P;
  if (t_row_ptr) HIPOK(hipMemcpyAsync(t_row_ptr, lp->D.t_ptr, sizeof(int) * (P.ni + 1), hipMemcpyDeviceToHost, s));
  if (t_col && P.nnzi) HIPOK(hipMemcpyAsync(t_col, lp->D.t_col, sizeof(int) * P.nnzi, hipMemcpyDeviceToHost, s));
  if (t_val && P.nnzi) HIPOK(hipMemcpyAsync(t_val, lp->D.t_raw, sizeof(double) * P.nnzi, hipMemcpyDeviceToHost, s));
  HIPOK(hipStreamSynchronize(s));
  return UC_LP_OK;
}

extern "C" int uc_lp_get_scaling(uc_lp* lp, double* d_row, double* d_col, double* norm_est) {
  g_err.clear();
  int rc = debug_ready(lp);
  if (rc) return rc;
  hipStream_t s = lp->eng->stream;
  const HostProblem& P = lp->P;
  if (d_row && P.mi) HIPOK(hipMemcpyAsync(d_row, lp->D.dr, sizeof(double) * P.mi, hipMemcpyDeviceToHost, s));
  if (d_col) HIPOK(hipMemcpyAsync(d_col, lp->D.dc, sizeof(double) * P.ni, hipMemcpyDeviceToHost, s));
  HIPOK(hipStreamSynchronize(s));
  if (norm_est) *norm_est = get_info(lp).norm_a_est;
  return UC_LP_OK;
}

template <typename T>
static int put_vec(T* dst, const double* src, size_t n, hipStream_t s) {
  std::vector<T> tmp(src, src + n);
  HIPOK(hipMemcpyAsync(dst, tmp.data(), sizeof(T) * n, hipMemcpyHostToDevice, s));
  HIPOK(hipStreamSynchronize(s));
  return UC_LP_OK;
}

template <typename T>
static int get_vec(double* dst, const T* src, size_t n, hipStream_t s) {
  std::vector<T> tmp(n);
  HIPOK(hipMemcpyAsync(tmp.data(), src, sizeof(T) * n, hipMemcpyDeviceToHost, s));
  HIPOK(hipStreamSynchronize(s));
  for (size_t i = 0; i < n; ++i) dst[i] = (double)tmp[i];
  return UC_LP_OK;
}

template <typename T>
static int debug_iterate_t(uc_lp* lp, int iters, int threads, const double* x, const double* y, const double* x0,
                           const double* y0, int64_t k, double tau, double sigma, double* xh, double* yh, double* xn,
                           double* yn, double* rfp) {
  const HostProblem& P = lp->P;
  DevMem& D = lp->D;
  uc_engine* E = lp->eng;
  hipStream_t s = E->stream;
  const int prec = sizeof(T) == 4 ? 1 : 0;
  Vecs<T>& V = prec ? *(Vecs<T>*)&D.f : *(Vecs<T>*)&D.d;
  int rc;
  if ((rc = put_vec<T>(V.x, x, P.ni, s)) || (rc = put_vec<T>(V.x0, x0, P.ni, s)) ||
      (rc = put_vec<T>(V.y, y, P.mi, s)) || (rc = put_vec<T>(V.y0, y0, P.mi, s)))
    return rc;
  SlotDev S = make_slot(lp);
  S.tau[0] = tau;
  S.sigma[0] = sigma;
  S.k0[0] = k;
  S.kfin = k + iters - 1;
  S.restart[0] = 0;
  S.active[0] = 1;
  std::vector<Tile> tl;
  push_tiles(tl, 0, P.t_blk, P.t_ptr, &P.t_flag, &P.t_base);
  push_tiles(tl, 0, P.a_blk, P.a_ptr, &P.a_flag, &P.a_base);
  E->layout_valid = false;  // the engine's tile and slot tables are overwritten below
  if ((rc = engine_tables(E, tl.size()))) return rc;
  HIPOK(hipMemcpyAsync(E->d_slots, &S, sizeof S, hipMemcpyHostToDevice, s));
  HIPOK(hipMemcpyAsync(E->d_tiles, tl.data(), tl.size() * sizeof(Tile), hipMemcpyHostToDevice, s));
  int zero = 0;
  HIPOK(hipMemcpyAsync(E->d_ids, &zero, sizeof zero, hipMemcpyHostToDevice, s));
  const Tile* TT = E->d_tiles;
  const Tile* TA = E->d_tiles + S.t_nblk;
  // the launch sequence of one check interval of the solve (run_epochs)
  for (int j = 0; j < iters; ++j) {
    const bool check = j == iters - 1;
    launch_primal(prec, check, E->d_slots, TT, S.t_nblk, j, 1, s, nullptr, nullptr, threads);
    launch_dual(prec, check, E->d_slots, TA, S.a_nblk, j, 1, s, nullptr, nullptr, threads);
  }
  launch_kkt(prec, E->d_slots, TT, S.t_nblk, TA, S.a_nblk, 1, s);
  launch_reduce(E->d_slots, E->d_ids, 1, 1, E->d_red2, s);
  launch_finish(prec, E->d_slots, TT, S.t_nblk, TA, S.a_nblk, 0, 1, s);
  double q[kScal];
  HIPOK(hipMemcpyAsync(q, D.scal, sizeof q, hipMemcpyDeviceToHost, s));
  HIPOK(hipGetLastError());
  HIPOK(hipStreamSynchronize(s));
  if ((rc = get_vec<T>(xh, V.xhat, P.ni, s)) || (rc = get_vec<T>(yh, V.yhat, P.mi, s)) ||
      (rc = get_vec<T>(xn, V.x, P.ni, s)) || (rc = get_vec<T>(yn, V.y, P.mi, s)))
    return rc;
  if (rfp) {
    // the same scalars and metric as the restart test of a solve
    const double r2 = q[RQ_N + CQ_DX2] / tau + q[RQ_DY2] / sigma + 2.0 * q[RQ_DYADX];
    *rfp = std::sqrt(std::max(r2, 0.0));
  }
  return UC_LP_OK;
}

extern "C" int uc_lp_debug_iterate(uc_lp* lp, int32_t precision, int32_t iters, int32_t block_threads,
                                   const double* x, const double* y, const double* x0, const double* y0, int64_t k,
                                   double tau, double sigma, double* x_hat, double* y_hat, double* x_next,
                                   double* y_next, double* fp_residual) {
  g_err.clear();
  int rc = debug_ready(lp);
  if (rc) return rc;
  if (!x || !y || !x0 || !y0 || !x_hat || !y_hat || !x_next || !y_next)
    return fail(UC_LP_EINVAL, "NULL vector");
  if (k < 0 || !(tau > 0) || !(sigma > 0)) return fail(UC_LP_EINVAL, "k, tau, sigma");
  if (iters < 1 || iters > 4096) return fail(UC_LP_EINVAL, "iters %d not in 1..4096", iters);
  if (block_threads != 0 && block_threads != kThreads && block_threads != kRowsPerBlock)
    return fail(UC_LP_EINVAL, "block_threads %d: 0, %d or %d", block_threads, kThreads, kRowsPerBlock);
  if (precision == UC_LP_FP64)
    return debug_iterate_t<double>(lp, iters, block_threads, x, y, x0, y0, k, tau, sigma, x_hat, y_hat, x_next,
                                   y_next, fp_residual);
  if (precision == UC_LP_FP32_MIXED)
    return debug_iterate_t<float>(lp, iters, block_threads, x, y, x0, y0, k, tau, sigma, x_hat, y_hat, x_next,
                                  y_next, fp_residual);
  return fail(UC_LP_ENOTSUP, "precision %d", precision);
}

extern "C" int uc_lp_debug_step(uc_lp* lp, int32_t precision, const double* x, const double* y,
                                const double* x0, const double* y0, int64_t k, double tau, double sigma,
                                double* x_hat, double* y_hat, double* x_next, double* y_next) {
  return uc_lp_debug_iterate(lp, precision, 1, 0, x, y, x0, y0, k, tau, sigma, x_hat, y_hat, x_next, y_next,
                             nullptr);
}

extern "C" int uc_lp_eval_kkt(uc_lp* lp, const double* x, const double* y, uc_lp_info* out) {
  g_err.clear();
  int rc = debug_ready(lp);
  if (rc) return rc;
  if (!x || !y || !out) return fail(UC_LP_EINVAL, "NULL argument");
  const HostProblem& P = lp->P;
  DevMem& D = lp->D;
  uc_engine* E = lp->eng;
  hipStream_t s = E->stream;
  // internal scaled point: x_hat = x / D_c, y_hat = y / D_r (sign of 'L' rows flipped)
  std::vector<double> dr(P.mi), dc(P.ni), xi(P.ni), yi(P.mi);
  if (P.mi) HIPOK(hipMemcpyAsync(dr.data(), D.dr, sizeof(double) * P.mi, hipMemcpyDeviceToHost, s));
  HIPOK(hipMemcpyAsync(dc.data(), D.dc, sizeof(double) * P.ni, hipMemcpyDeviceToHost, s));
  HIPOK(hipStreamSynchronize(s));
  for (int j = 0; j < P.ni; ++j) xi[j] = x[P.col_map[j]] / dc[j];
  for (int i = 0; i < P.mi; ++i) {
    const int enc = P.row_map[i];
    yi[i] = (enc >= 0 ? y[enc] : -y[-enc - 1]) / dr[i];
  }
  Vecs<double>& V = D.d;
  for (double* dst : {V.x, V.x0, V.xhat})
    if ((rc = put_vec<double>(dst, xi.data(), P.ni, s))) return rc;
  for (double* dst : {V.y, V.y0, V.yhat})
    if ((rc = put_vec<double>(dst, yi.data(), P.mi, s))) return rc;
  SlotDev S = make_slot(lp);
  std::vector<Tile> tl;
  push_tiles(tl, 0, P.t_blk, P.t_ptr, &P.t_flag, &P.t_base);
  push_tiles(tl, 0, P.a_blk, P.a_ptr, &P.a_flag, &P.a_base);
  E->layout_valid = false;  // the engine's tile and slot tables are overwritten below
  if ((rc = engine_tables(E, tl.size()))) return rc;
  HIPOK(hipMemcpyAsync(E->d_slots, &S, sizeof S, hipMemcpyHostToDevice, s));
  HIPOK(hipMemcpyAsync(E->d_tiles, tl.data(), tl.size() * sizeof(Tile), hipMemcpyHostToDevice, s));
  int zero = 0;
  HIPOK(hipMemcpyAsync(E->d_ids, &zero, sizeof zero, hipMemcpyHostToDevice, s));
  launch_kkt(0, E->d_slots, E->d_tiles, S.t_nblk, E->d_tiles + S.t_nblk, S.a_nblk, 1, s);
  launch_reduce(E->d_slots, E->d_ids, 1, 1, E->d_red2, s);
  double q[kScal];
  HIPOK(hipMemcpyAsync(q, D.scal, sizeof q, hipMemcpyDeviceToHost, s));
  HIPOK(hipStreamSynchronize(s));
  HIPOK(hipGetLastError());
  uc_lp_info in;
  std::memset(&in, 0, sizeof in);
  kkt_from_scalars(lp, q, in);
  // fixed columns and removed rows contribute nothing to the residuals when
  // x sits at the fixed value; report violations of those separately
  for (int32_t j = 0; j < P.n; ++j)
    if (P.int_col[j] < 0 && x[j] != P.o_lb[j]) in.abs_primal_inf = std::max(in.abs_primal_inf, std::fabs(x[j] - P.o_lb[j]));
  in.status = lp->status.load();
  *out = in;
  return UC_LP_OK;
}

extern "C" int uc_lp_debug_refine(uc_lp* lp, const double* x_star, const double* y_star, const float* x_corr,
                                  const float* y_corr, int32_t first, const double* par, double* x_new,
                                  double* y_new, double* data64, float* data32, double* scal) {
  g_err.clear();
  int rc = debug_ready(lp);
  if (rc) return rc;
  if (!x_corr || !y_corr || !par || (!first && (!x_star || !y_star))) return fail(UC_LP_EINVAL, "NULL argument");
  for (int k = 0; k < 6; ++k)
    if (!std::isfinite(par[k])) return fail(UC_LP_EINVAL, "par[%d] is not finite", k);
  if (!(par[0] > 0 && par[1] > 0 && par[2] > 0 && par[3] > 0 && par[4] > 1 && par[5] > 0))
    return fail(UC_LP_EINVAL, "refinement factors must be positive (growth > 1)");
  const HostProblem& P = lp->P;
  DevMem& D = lp->D;
  hipStream_t s = lp->eng->stream;
  const size_t n = P.ni, m = P.mi;
  if (!first) {
    HIPOK(hipMemcpyAsync(D.d.xhat, x_star, 8 * n, hipMemcpyHostToDevice, s));
    if (m) HIPOK(hipMemcpyAsync(D.d.yhat, y_star, 8 * m, hipMemcpyHostToDevice, s));
  }
  HIPOK(hipMemcpyAsync(D.f.xhat, x_corr, 4 * n, hipMemcpyHostToDevice, s));
  if (m) HIPOK(hipMemcpyAsync(D.f.yhat, y_corr, 4 * m, hipMemcpyHostToDevice, s));
  RefineArgs R = refine_args(lp);
  R.first = first ? 1 : 0;
  R.inv_dp = par[0];
  R.inv_dd = par[1];
  launch_refine_measure(R, s);
  HIPOK(hipGetLastError());
  double q[FQ_N];
  HIPOK(hipMemcpyAsync(q, R.out, sizeof q, hipMemcpyDeviceToHost, s));
  HIPOK(hipStreamSynchronize(s));
  const RefineFactors f = refine_factors(q, par[2], par[3], par[4], par[5]);
  R.dp = f.dp;
  R.dd = f.dd;
  launch_refine_form(R, s);
  HIPOK(hipGetLastError());
  if (x_new) HIPOK(hipMemcpyAsync(x_new, D.d.xhat, 8 * n, hipMemcpyDeviceToHost, s));
  if (y_new && m) HIPOK(hipMemcpyAsync(y_new, D.d.yhat, 8 * m, hipMemcpyDeviceToHost, s));
  if (data64) {
    HIPOK(hipMemcpyAsync(data64, D.d.c, 8 * n, hipMemcpyDeviceToHost, s));
    HIPOK(hipMemcpyAsync(data64 + n, D.d.l, 8 * n, hipMemcpyDeviceToHost, s));
    HIPOK(hipMemcpyAsync(data64 + 2 * n, D.d.u, 8 * n, hipMemcpyDeviceToHost, s));
    if (m) HIPOK(hipMemcpyAsync(data64 + 3 * n, D.d.b, 8 * m, hipMemcpyDeviceToHost, s));
  }
  if (data32) {
    HIPOK(hipMemcpyAsync(data32, D.f.c, 4 * n, hipMemcpyDeviceToHost, s));
    HIPOK(hipMemcpyAsync(data32 + n, D.f.l, 4 * n, hipMemcpyDeviceToHost, s));
    HIPOK(hipMemcpyAsync(data32 + 2 * n, D.f.u, 4 * n, hipMemcpyDeviceToHost, s));
    if (m) {
      HIPOK(hipMemcpyAsync(data32 + 3 * n, D.f.b, 4 * m, hipMemcpyDeviceToHost, s));
      HIPOK(hipMemcpyAsync(data32 + 3 * n + m, D.ylo32, 4 * m, hipMemcpyDeviceToHost, s));
    }
  }
  HIPOK(hipStreamSynchronize(s));
  RefineRun F;
  refine_outer(q, P, F);
  if (scal) {
    const double v[14] = {f.dp, f.dd, f.omega, q[FQ_VIOL2], q[FQ_DRES2], q[FQ_VIOL2U], q[FQ_BY], q[FQ_VMAXU],
                          q[FQ_DRES2U], q[FQ_LBUB], q[FQ_CX], f.dp * std::sqrt(std::max(q[FQ_R2U], 0.0)),
                          f.dd * std::sqrt(std::max(q[FQ_D2U], 0.0)), F.rel_kkt};
    std::memcpy(scal, v, sizeof v);
  }
  // the scaled data arrays held the correction problem
  return restore_scaled_data(lp, s);
}

// ---------------------------------------------------------------------------
// standalone SpMV and bandwidth probes
// ---------------------------------------------------------------------------

struct SpmvDev {
  int *ptr = nullptr, *col = nullptr, *blk = nullptr, *crow = nullptr;
  void *val = nullptr, *x = nullptr, *y = nullptr, *cval = nullptr;
  int2* coord = nullptr;
  int nblk = 0;
  bool fixup = true;  // some merge tile ends inside a row
};

static void spmv_free(SpmvDev& S) {
  for (void* p : {(void*)S.ptr, (void*)S.col, (void*)S.blk, (void*)S.crow, S.val, S.x, S.y, S.cval, (void*)S.coord})
    if (p) (void)hipFree(p);
}

static int spmv_prepare(int32_t m, int32_t n, int64_t nnz, const int32_t* rp, const int32_t* ci, const double* v,
                        int prec, const double* x, SpmvDev& S, hipStream_t s) {
  std::vector<int> ptr(rp, rp + m + 1), blk;
  partition_rows(ptr, m, blk);
  S.nblk = (int)blk.size() - 1;
  const size_t vs = prec == UC_LP_FP64 ? 8 : 4;
  HIPOK(hipMalloc(&S.ptr, sizeof(int) * (m + 1)));
  HIPOK(hipMalloc(&S.col, sizeof(int) * std::max<int64_t>(nnz, 1)));
  HIPOK(hipMalloc(&S.blk, sizeof(int) * blk.size()));
  HIPOK(hipMalloc(&S.val, vs * std::max<int64_t>(nnz, 1)));
  HIPOK(hipMalloc(&S.x, vs * n));
  HIPOK(hipMalloc(&S.y, vs * m));
  const int nc = merge_workgroups(m, nnz);
  HIPOK(hipMalloc(&S.crow, sizeof(int) * std::max(nc, 1)));
  HIPOK(hipMalloc(&S.cval, vs * std::max(nc, 1)));
  HIPOK(hipMalloc(&S.coord, sizeof(int2) * (nc + 1)));
  HIPOK(hipMemcpyAsync(S.ptr, rp, sizeof(int) * (m + 1), hipMemcpyHostToDevice, s));
  if (nnz) HIPOK(hipMemcpyAsync(S.col, ci, sizeof(int) * nnz, hipMemcpyHostToDevice, s));
  HIPOK(hipMemcpyAsync(S.blk, blk.data(), sizeof(int) * blk.size(), hipMemcpyHostToDevice, s));
  if (prec == UC_LP_FP64) {
    if (nnz) HIPOK(hipMemcpyAsync(S.val, v, 8 * nnz, hipMemcpyHostToDevice, s));
    if (x) HIPOK(hipMemcpyAsync(S.x, x, 8 * n, hipMemcpyHostToDevice, s));
    HIPOK(hipStreamSynchronize(s));
  } else {
    std::vector<float> fv(v, v + nnz);
    std::vector<float> fx(n, 0.0f);
    if (x)
      for (int j = 0; j < n; ++j) fx[j] = (float)x[j];
    else
      for (int j = 0; j < n; ++j) fx[j] = 1.0f;
    if (nnz) HIPOK(hipMemcpyAsync(S.val, fv.data(), 4 * nnz, hipMemcpyHostToDevice, s));
    HIPOK(hipMemcpyAsync(S.x, fx.data(), 4 * n, hipMemcpyHostToDevice, s));
    HIPOK(hipStreamSynchronize(s));
  }
  if (prec == UC_LP_FP64 && !x) {
    std::vector<double> ones(n, 1.0);
    HIPOK(hipMemcpy(S.x, ones.data(), 8 * n, hipMemcpyHostToDevice));
  }
  // the merge-path coordinates depend on the row pointers only: computed
  // once here, as the row-split partition is; the fix-up is needed only if
  // a tile ends inside a row
  launch_merge_coords(S.ptr, m, nnz, S.coord, s);
  HIPOK(hipGetLastError());
  std::vector<int2> cd((size_t)nc + 1);
  HIPOK(hipMemcpyAsync(cd.data(), S.coord, sizeof(int2) * (nc + 1), hipMemcpyDeviceToHost, s));
  HIPOK(hipStreamSynchronize(s));
  S.fixup = false;
  for (int g = 1; g < nc; ++g)
    if (cd[g].x < m && cd[g].y > rp[cd[g].x]) S.fixup = true;
  return UC_LP_OK;
}

static void spmv_launch(const SpmvDev& S, int32_t m, int64_t nnz, int prec, int algo, hipStream_t s) {
  if (prec == UC_LP_FP64) {
    if (algo == UC_LP_SPMV_MERGEPATH)
      launch_spmv_merge64(S.ptr, S.col, (const double*)S.val, (const double*)S.x, (double*)S.y, m, nnz, S.coord,
                          S.crow, (double*)S.cval, s, true, S.fixup);
    else
      launch_spmv64(S.ptr, S.col, (const double*)S.val, (const double*)S.x, (double*)S.y, S.blk, S.nblk, s);
  } else {
    if (algo == UC_LP_SPMV_MERGEPATH)
      launch_spmv_merge32(S.ptr, S.col, (const float*)S.val, (const float*)S.x, (float*)S.y, m, nnz, S.coord,
                          S.crow, (float*)S.cval, s, true, S.fixup);
    else
      launch_spmv32(S.ptr, S.col, (const float*)S.val, (const float*)S.x, (float*)S.y, S.blk, S.nblk, s);
  }
}

extern "C" int uc_spmv(int device, int32_t m, int32_t n, int64_t nnz, const int32_t* row_ptr,
                       const int32_t* col_idx, const double* val, const double* x, double* y, int32_t precision,
                       int32_t algo) {
  g_err.clear();
  int rc = validate_csr(m, n, nnz, row_ptr, col_idx, val);
  if (rc) return rc;
  if (!x || !y) return fail(UC_LP_EINVAL, "NULL vector");
  if (precision != UC_LP_FP64 && precision != UC_LP_FP32_MIXED) return fail(UC_LP_ENOTSUP, "precision");
  if (algo != UC_LP_SPMV_ROWSPLIT && algo != UC_LP_SPMV_MERGEPATH) return fail(UC_LP_ENOTSUP, "algo");
  HIPOK(hipSetDevice(device));
  hipStream_t s;
  HIPOK(hipStreamCreate(&s));
  SpmvDev S;
  rc = spmv_prepare(m, n, nnz, row_ptr, col_idx, val, precision, x, S, s);
  if (rc == UC_LP_OK) {
    spmv_launch(S, m, nnz, precision, algo, s);
    hipError_t e = hipStreamSynchronize(s);
    if (e == hipSuccess) e = hipGetLastError();
    if (e != hipSuccess) rc = fail(UC_LP_EHIP, "spmv: %s", hipGetErrorString(e));
  }
  if (rc == UC_LP_OK) {
    if (precision == UC_LP_FP64) {
      if (hipMemcpy(y, S.y, 8 * m, hipMemcpyDeviceToHost) != hipSuccess) rc = fail(UC_LP_EHIP, "copy y");
    } else {
      std::vector<float> fy(m);
      if (hipMemcpy(fy.data(), S.y, 4 * m, hipMemcpyDeviceToHost) != hipSuccess) rc = fail(UC_LP_EHIP, "copy y");
      for (int i = 0; i < m; ++i) y[i] = fy[i];
    }
  }
  spmv_free(S);
  (void)hipStreamDestroy(s);
  return rc;
}

extern "C" int uc_spmv_bench(int device, int32_t m, int32_t n, int64_t nnz, const int32_t* row_ptr,
                             const int32_t* col_idx, const double* val, int32_t precision, int32_t algo,
                             int32_t copies, int32_t reps, double* us_per_spmv) {
  g_err.clear();
  int rc = validate_csr(m, n, nnz, row_ptr, col_idx, val);
  if (rc) return rc;
  if (!us_per_spmv || copies < 1 || copies > 64 || reps < 1) return fail(UC_LP_EINVAL, "copies/reps/out");
  if (precision != UC_LP_FP64 && precision != UC_LP_FP32_MIXED) return fail(UC_LP_ENOTSUP, "precision");
  if (algo != UC_LP_SPMV_ROWSPLIT && algo != UC_LP_SPMV_MERGEPATH) return fail(UC_LP_ENOTSUP, "algo");
  HIPOK(hipSetDevice(device));
  hipStream_t s;
  HIPOK(hipStreamCreate(&s));
  std::vector<SpmvDev> C(copies);
  for (int i = 0; i < copies && rc == UC_LP_OK; ++i)
    rc = spmv_prepare(m, n, nnz, row_ptr, col_idx, val, precision, nullptr, C[i], s);
  if (rc == UC_LP_OK) {
    hipEvent_t a, b;
    (void)hipEventCreate(&a);
    (void)hipEventCreate(&b);
    for (int i = 0; i < copies; ++i) spmv_launch(C[i], m, nnz, precision, algo, s);  // warm-up
    (void)hipEventRecord(a, s);
    for (int r = 0; r < reps; ++r) spmv_launch(C[r % copies], m, nnz, precision, algo, s);
    (void)hipEventRecord(b, s);
    hipError_t e = hipEventSynchronize(b);
    float ms = 0;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, a, b);
    if (e == hipSuccess) e = hipGetLastError();
    if (e != hipSuccess) rc = fail(UC_LP_EHIP, "spmv bench: %s", hipGetErrorString(e));
    else *us_per_spmv = 1e3 * ms / reps;
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
  }
  for (auto& S : C) spmv_free(S);
  (void)hipStreamDestroy(s);
  return rc;
}

extern "C" int uc_copy_bench(int device, size_t bytes, int32_t reps, double* gbps) {
  g_err.clear();
  if (!gbps || reps < 1 || bytes < 16) return fail(UC_LP_EINVAL, "bytes/reps/out");
  HIPOK(hipSetDevice(device));
  const size_t n4 = bytes / 16;
  void *a = nullptr, *b = nullptr;
  HIPOK(hipMalloc(&a, n4 * 16));
  if (hipMalloc(&b, n4 * 16) != hipSuccess) {
    (void)hipFree(a);
    return fail(UC_LP_ENOMEM, "copy buffer");
  }
  hipStream_t s;
  HIPOK(hipStreamCreate(&s));
  (void)hipMemsetAsync(a, 0, n4 * 16, s);
  hipEvent_t e0, e1;
  (void)hipEventCreate(&e0);
  (void)hipEventCreate(&e1);
  launch_copy_kernel((const float4*)a, (float4*)b, (int64_t)n4, s);
  (void)hipEventRecord(e0, s);
  for (int r = 0; r < reps; ++r)
    launch_copy_kernel((const float4*)((r & 1) ? b : a), (float4*)((r & 1) ? a : b), (int64_t)n4, s);
  (void)hipEventRecord(e1, s);
  hipError_t e = hipEventSynchronize(e1);
  float ms = 0;
  if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
  int rc = UC_LP_OK;
  if (e != hipSuccess) rc = fail(UC_LP_EHIP, "copy bench: %s", hipGetErrorString(e));
  else *gbps = 2.0 * (double)n4 * 16.0 * reps / (ms * 1e-3) / 1e9;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  (void)hipStreamDestroy(s);
  (void)hipFree(a);
  (void)hipFree(b);
  return rc;
}

extern "C" int uc_lp_bench_half_steps(uc_lp* lp, int32_t precision, int32_t copies, int32_t reps,
                                      double* primal_us, double* dual_us, double* primal_bytes,
                                      double* dual_bytes) {
  g_err.clear();
  if (!primal_us || !dual_us) return fail(UC_LP_EINVAL, "NULL output");
  if (copies < 1 || copies > 64 || reps < 1 || reps > 4096) return fail(UC_LP_EINVAL, "copies 1..64, reps 1..4096");
  if (precision != UC_LP_FP64 && precision != UC_LP_FP32_MIXED) return fail(UC_LP_ENOTSUP, "precision %d", precision);
  int rc = debug_ready(lp);
  if (rc) return rc;
  const int prec = precision == UC_LP_FP32_MIXED ? 1 : 0;
  const HostProblem& P = lp->P;
  uc_engine* E = lp->eng;
  hipStream_t s = E->stream;
  if ((rc = init_iterates(lp, prec))) return rc;
  HIPOK(hipStreamSynchronize(s));
  const size_t bytes = lp->D.ar.bytes;
  std::vector<void*> mem(copies, nullptr);
  SlotDev* d_slots = nullptr;
  Tile* d_tiles = nullptr;
  std::vector<hipEvent_t> ev;
  auto cleanup = [&]() {
    for (void* p : mem)
      if (p) (void)hipFree(p);
    if (d_slots) (void)hipFree(d_slots);
    if (d_tiles) (void)hipFree(d_tiles);
    for (auto e : ev) (void)hipEventDestroy(e);
  };
#define BENCH_HIP(call)                                                                      \
  do {                                                                                       \
    hipError_t e_ = (call);                                                                  \
    if (e_ != hipSuccess) {                                                                  \
      cleanup();                                                                             \
      return fail(UC_LP_EHIP, "%s failed: %s", #call, hipGetErrorString(e_));                \
    }                                                                                        \
  } while (0)
  // each copy is the instance's whole arena (matrix, scaled data, iterates),
  // so its slot descriptor is carved the same way at another base
  std::vector<SlotDev> slots(copies);
  std::vector<Tile> tiles;
  for (int c = 0; c < copies; ++c) {
    if (hipMalloc(&mem[c], bytes) != hipSuccess) {
      (void)hipGetLastError();
      cleanup();
      return fail(UC_LP_ENOMEM, "copy %d of %zu bytes", c, bytes);
    }
    BENCH_HIP(hipMemcpyAsync(mem[c], lp->D.ar.base, bytes, hipMemcpyDeviceToDevice, s));
    DevMem Dc;
    std::memset((void*)&Dc, 0, sizeof Dc);
    Dc.ar.base = (char*)mem[c];
    Dc.ar.bytes = bytes;
    carve(Dc, P, 1);
    SlotDev S = make_slot(P, Dc, lp->opts.halpern_gamma);
    S.tau[0] = lp->chk.eta / lp->chk.omega;
    S.sigma[0] = lp->chk.eta * lp->chk.omega;
    S.k0[0] = 0;
    S.active[0] = 1;
    slots[c] = S;
    push_tiles(tiles, c, P.t_blk, P.t_ptr, &P.t_flag, &P.t_base);
  }
  const size_t nt = P.t_blk.size() - 1, na = P.a_blk.size() - 1;
  for (int c = 0; c < copies; ++c) push_tiles(tiles, c, P.a_blk, P.a_ptr, &P.a_flag, &P.a_base);
  BENCH_HIP(hipMalloc(&d_slots, sizeof(SlotDev) * copies));
  BENCH_HIP(hipMalloc(&d_tiles, sizeof(Tile) * tiles.size()));
  BENCH_HIP(hipMemcpyAsync(d_slots, slots.data(), sizeof(SlotDev) * copies, hipMemcpyHostToDevice, s));
  BENCH_HIP(hipMemcpyAsync(d_tiles, tiles.data(), sizeof(Tile) * tiles.size(), hipMemcpyHostToDevice, s));
  BENCH_HIP(hipStreamSynchronize(s));
  ev.resize(4 * (size_t)reps, nullptr);
  for (auto& e : ev) BENCH_HIP(hipEventCreate(&e));
  auto tt = [&](int c) { return d_tiles + (size_t)c * nt; };
  auto ta = [&](int c) { return d_tiles + (size_t)copies * nt + (size_t)c * na; };
  // warm-up: one iteration on every copy
  for (int c = 0; c < copies; ++c) {
    launch_primal(prec, false, d_slots, tt(c), (int)nt, 1, 1, s);
    launch_dual(prec, false, d_slots, ta(c), (int)na, 1, 1, s);
  }
  // iterations round-robin over the copies: launch r reads copy r % copies,
  // as a solve's non-check launches (inner index 1..62, primal iterate rebuilt
  // at full reflection); each launch carries its own start / stop events
  for (int r = 0; r < reps; ++r) {
    const int c = r % copies, j = 1 + r % 62;
    launch_primal(prec, false, d_slots, tt(c), (int)nt, j, 1, s, ev[4 * r], ev[4 * r + 1]);
    launch_dual(prec, false, d_slots, ta(c), (int)na, j, 1, s, ev[4 * r + 2], ev[4 * r + 3]);
  }
  BENCH_HIP(hipGetLastError());
  BENCH_HIP(hipStreamSynchronize(s));
  double tp = 0, td = 0;
  for (int r = 0; r < reps; ++r) {
    float a = 0, b = 0;
    BENCH_HIP(hipEventElapsedTime(&a, ev[4 * r], ev[4 * r + 1]));
    BENCH_HIP(hipEventElapsedTime(&b, ev[4 * r + 2], ev[4 * r + 3]));
    tp += a;
    td += b;
  }
  *primal_us = 1e3 * tp / reps;
  *dual_us = 1e3 * td / reps;
  double pb = 0, db = 0;
  half_step_bytes(P, prec ? 4 : 8, lp->opts.halpern_gamma == 1.0, &pb, &db);
  if (primal_bytes) *primal_bytes = pb;
  if (dual_bytes) *dual_bytes = db;
  cleanup();
#undef BENCH_HIP
  return UC_LP_OK;
}

// ---------------------------------------------------------------------------
// merge-path SpMV on caller-owned device arrays, without allocation
// ---------------------------------------------------------------------------

// Scratch of the allocation-free SpMV (workgroup coordinates and carries of
// the merge-path kernels): one static array per device, held until the
// process ends.  Host code never passes the array's name to a kernel (on the
// host it is a stand-in, not a device address); it passes the device address
// that hipGetSymbolAddress returns for each device, looked up once per device
// with that device current.
constexpr size_t kNoAllocScratchBytes = size_t(4) << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];
constexpr int kMaxScratchDevices = 64;
static std::mutex g_scratch_mu;
static void* g_scratch_dev[kMaxScratchDevices];

// Device address of `scratch` on `device`, which must be current.
static int scratch_address(int device, void** out) {
  std::lock_guard<std::mutex> g(g_scratch_mu);
  if (!g_scratch_dev[device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(UC_LP_EHIP, "hipGetSymbolAddress(scratch) on device %d: %s", device, hipGetErrorString(e));
    g_scratch_dev[device] = p;
  }
  *out = g_scratch_dev[device];
  return UC_LP_OK;
}

static size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

// Offsets of the merge-path scratch for nwg workgroups with vb-byte values:
// coord[nwg + 1] (int2), carry_row[nwg], carry_val[nwg].
static size_t merge_scratch_layout(int nwg, size_t vb, size_t* off_row, size_t* off_val) {
  *off_row = align256((size_t)(nwg + 1) * sizeof(int2));
  *off_val = align256(*off_row + (size_t)nwg * sizeof(int));
  return *off_val + (size_t)nwg * vb;
}

// The memory behind p must be device (or managed) memory of `device`.
static int check_device_pointer(const void* p, int device, const char* what) {
  hipPointerAttribute_t a;
  std::memset(&a, 0, sizeof a);
  const hipError_t e = hipPointerGetAttributes(&a, p);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return fail(UC_LP_EINVAL, "%s is not device memory (%s)", what, hipGetErrorString(e));
  }
  if (!(a.type == hipMemoryTypeDevice || a.type == hipMemoryTypeManaged) || a.device != device)
    return fail(UC_LP_EINVAL, "%s is not device memory of device %d (type %d, device %d)", what, device, (int)a.type,
                a.device);
  return UC_LP_OK;
}

extern "C" int uc_spmv_merge_noalloc(int device, int32_t m, int32_t n, int64_t nnz, const int32_t* row_ptr,
                                     const int32_t* col_idx, const void* val, const void* x, void* y,
                                     int32_t precision, void* hip_stream) {
  g_err.clear();
  if (m < 1 || n < 1) return fail(UC_LP_EINVAL, "m=%d n=%d must be >= 1", m, n);
  if (nnz < 0 || nnz > INT32_MAX) return fail(UC_LP_EINVAL, "nnz=%lld out of range", (long long)nnz);
  if (!row_ptr || !x || !y || (nnz > 0 && (!col_idx || !val))) return fail(UC_LP_EINVAL, "NULL array");
  if (precision != UC_LP_FP64 && precision != UC_LP_FP32_MIXED) return fail(UC_LP_ENOTSUP, "precision %d", precision);
  const size_t vb = precision == UC_LP_FP64 ? 8 : 4;
  const int64_t items = (int64_t)m + nnz;
  const int64_t nwg64 = (items + kMergeStep - 1) / kMergeStep;  // merge_workgroups without its int range
  size_t off_row = 0, off_val = 0;
  const size_t need = nwg64 < INT32_MAX ? merge_scratch_layout((int)nwg64, vb, &off_row, &off_val) : SIZE_MAX;
  if (need > kNoAllocScratchBytes)
    return fail(UC_LP_ENOTSUP, "m + nnz = %lld needs %zu bytes of scratch; the static scratch holds %zu bytes",
                (long long)items, need, kNoAllocScratchBytes);
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || count <= 0) return fail(UC_LP_EHIP, "no HIP device");
  if (device < 0 || device >= count || device >= kMaxScratchDevices)
    return fail(UC_LP_EINVAL, "device %d of %d", device, count);
  int prev = 0;
  HIPOK(hipGetDevice(&prev));
  HIPOK(hipSetDevice(device));
  int rc = UC_LP_OK;
  const void* ptrs[5] = {row_ptr, col_idx, val, x, y};
  const char* names[5] = {"row_ptr", "col_idx", "val", "x", "y"};
  for (int i = 0; i < 5 && rc == UC_LP_OK; ++i)
    if (ptrs[i]) rc = check_device_pointer(ptrs[i], device, names[i]);
  void* sp = nullptr;
  if (rc == UC_LP_OK) rc = scratch_address(device, &sp);
  if (rc == UC_LP_OK) {
    char* base = (char*)sp;
    int2* coord = (int2*)base;
    int* crow = (int*)(base + off_row);
    hipStream_t s = (hipStream_t)hip_stream;
    if (precision == UC_LP_FP64)
      launch_spmv_merge64(row_ptr, col_idx, (const double*)val, (const double*)x, (double*)y, m, nnz, coord, crow,
                          (double*)(base + off_val), s);
    else
      launch_spmv_merge32(row_ptr, col_idx, (const float*)val, (const float*)x, (float*)y, m, nnz, coord, crow,
                          (float*)(base + off_val), s);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) rc = fail(UC_LP_EHIP, "merge-path launch: %s", hipGetErrorString(e));
  }
  (void)hipSetDevice(prev);
  return rc;
}

// ---------------------------------------------------------------------------
// scenario batches over one matrix
// ---------------------------------------------------------------------------

// Lanes of an interleaved scenario array (element j of lane L at j * lanes +
// L) kept by a batch after some of its scenarios have finished.
struct LaneMap {
  int src_lanes, dst_lanes;
  int lane[kMaxScen];  // dst lane k <- src lane lane[k]
};

// dst[j * dst_lanes + k] = src[j * src_lanes + lane[k]] for j < rows.
template <typename T>
__global__ void k_compact_lanes(const T* __restrict__ src, T* __restrict__ dst, int64_t rows, LaneMap mp) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= rows * mp.dst_lanes) return;
  const int64_t j = e / mp.dst_lanes;
  const int k = (int)(e - j * mp.dst_lanes);
  dst[e] = src[j * mp.src_lanes + mp.lane[k]];
}

template <typename T>
static void launch_compact_lanes(const T* src, T* dst, int64_t rows, const LaneMap& mp, hipStream_t s) {
  const int64_t total = rows * mp.dst_lanes;
  if (total <= 0) return;
  const int threads = 256;
  k_compact_lanes<T><<<(unsigned)((total + threads - 1) / threads), threads, 0, s>>>(src, dst, rows, mp);
}

struct ScenArena {
  Arena ar;
  double *c_in, *l_in, *u_in, *b_in, *x_out, *y_out, *x_warm, *y_warm;
  double *part_a, *part_t, *scal, *red2;
  Vecs<float> f;
  Vecs<double> d;
  SlotDev* slot_dev;
  Tile* tiles;
};

static void carve_scen(ScenArena& A, const HostProblem& P, int S) {
  Arena& a = A.ar;
  const int n = P.ni, m = P.mi;
  A.c_in = a.take<double>((size_t)n * S);
  A.l_in = a.take<double>((size_t)n * S);
  A.u_in = a.take<double>((size_t)n * S);
  A.b_in = a.take<double>((size_t)m * S);
  A.x_out = a.take<double>((size_t)n * S);
  A.y_out = a.take<double>((size_t)m * S);
  A.x_warm = a.take<double>((size_t)n * S);
  A.y_warm = a.take<double>((size_t)m * S);
  A.part_a = a.take<double>(P.a_blk.size() * RQ_N * kMaxScen);
  A.part_t = a.take<double>(P.t_blk.size() * CQ_N * kMaxScen);
  A.scal = a.take<double>((size_t)kScal * kMaxScen);
  A.red2 = a.take<double>(red2_ms_doubles());
  carve_vecs(a, A.f, n, m, S);
  carve_vecs(a, A.d, n, m, S);
  A.slot_dev = a.take<SlotDev>(1);
  A.tiles = a.take<Tile>(P.a_blk.size() + P.t_blk.size());
}

// The batched half-steps can serve 16 bytes of consecutive scenarios per
// access (4 FP32 or 2 FP64 lanes) when the batch width is a multiple of that
// and every vector they touch starts on a 16-byte boundary.
template <typename T>
static bool vecs_aligned16(const Vecs<T>& V) {
  const void* p[11] = {V.x, V.x0, V.xbar, V.xhat, V.y, V.y0, V.yhat, V.c, V.l, V.u, V.b};
  for (const void* q : p)
    if (((uintptr_t)q & 15) != 0) return false;
  return true;
}

static bool ms_vector_lanes(const SlotDev& S, int prec, int lanes) {
  if (prec == 1) return lanes % 4 == 0 && vecs_aligned16(S.f);
  return lanes % 2 == 0 && vecs_aligned16(S.d);
}

extern "C" int uc_lp_solve_scenarios(uc_lp* base, int32_t n_scen, const double* c, const double* b,
                                     const double* lb, const double* ub, const double* x0, const double* y0,
                                     double* x, double* y, uc_lp_info* info) {
  g_err.clear();
  if (!base) return fail(UC_LP_EINVAL, "NULL handle");
  if (n_scen < 1 || n_scen > kMaxScen) return fail(UC_LP_ENOTSUP, "n_scen %d not in 1..%d", n_scen, kMaxScen);
  if (!c || !b || !lb || !ub || !info) return fail(UC_LP_EINVAL, "NULL scenario array");
  if (base->opts.precision == UC_LP_FP32_REFINE)
    return fail(UC_LP_ENOTSUP, "scenario batches do not run UC_LP_FP32_REFINE");
  const HostProblem& P = base->P;
  const int S = n_scen, n = P.n, m = P.m, ni = P.ni, mi = P.mi;
  // per-scenario validation and minimal presolve (same fixed-column structure as the base)
  std::vector<HostProblem> SP(S);
  // each scenario's checks and presolve on a host thread of its own; an
  // error is reported for the lowest-numbered failing scenario
  std::vector<int> prc(S, UC_LP_OK);
  std::vector<std::string> pmsg(S);
  fork_join(S, [&](int s) {
    const double *cs = c + (size_t)s * n, *bs = b + (size_t)s * m, *ls = lb + (size_t)s * n, *us = ub + (size_t)s * n;
    int rc = validate_data(m, n, cs, bs, P.o_sense.data(), ls, us);
    if (rc) {
      prc[s] = rc;
      pmsg[s] = g_err;
      return;
    }
    for (int32_t j = 0; j < n; ++j)
      if ((ls[j] == us[j]) != (P.int_col[j] < 0)) {
        prc[s] = fail(UC_LP_ENOTSUP, "scenario %d: column %d differs from the base in being fixed", s, j);
        pmsg[s] = g_err;
        return;
      }
    HostProblem& Q = SP[s];  // data only; the structure is the base's
    Q.m = m;
    Q.n = n;
    Q.o_c.assign(cs, cs + n);
    Q.o_b.assign(bs, bs + m);
    Q.o_lb.assign(ls, ls + n);
    Q.o_ub.assign(us, us + n);
    Q.ni = ni;
    Q.mi = mi;
    Q.b.assign(mi, 0.0);
    Q.c.assign(ni, 0.0);
    Q.l.assign(ni, 0.0);
    Q.u.assign(ni, 0.0);
    presolve_data(Q, P);
    if (Q.infeasible) {
      prc[s] = fail(UC_LP_EINVAL, "scenario %d is infeasible by its empty rows", s);
      pmsg[s] = g_err;
    }
  });
  for (int s = 0; s < S; ++s)
    if (prc[s] != UC_LP_OK) return fail(prc[s], "%s", pmsg[s].c_str());
  // a block flag holds for the batch when it holds for every scenario
  std::vector<int> tflag = SP[0].t_flag, aflag = SP[0].a_flag;
  for (int s = 1; s < S; ++s) {
    for (size_t k = 0; k < tflag.size(); ++k) tflag[k] &= SP[s].t_flag[k];
    for (size_t k = 0; k < aflag.size(); ++k) aflag[k] &= SP[s].a_flag[k];
  }
  int rc = debug_ready(base);
  if (rc) return rc;
  base->cancel.store(false);  // uc_lp_cancel from another thread stops the batch
  uc_engine* E = base->eng;
  hipStream_t st = E->stream;
  const uc_lp_opts& o = base->opts;
  ScenArena A;
  std::memset((void*)&A, 0, sizeof A);
  carve_scen(A, P, S);
  const size_t bytes = A.ar.used + 256;
  void* mem = nullptr;
  if (hipMalloc(&mem, bytes) != hipSuccess) {
    (void)hipGetLastError();
    return fail(UC_LP_ENOMEM, "scenario arena of %zu bytes", bytes);
  }
  A.ar = Arena();
  A.ar.base = (char*)mem;
  A.ar.bytes = bytes;
  carve_scen(A, P, S);
  void* cmem = nullptr;  // FP64 arrays of the scenarios still running after the FP64 hand-over
  auto cleanup = [&]() {
    (void)hipFree(mem);
    if (cmem) (void)hipFree(cmem);
  };
#define SCEN_HIP(call)                                                                           \
  do {                                                                                           \
    hipError_t e_ = (call);                                                                      \
    if (e_ != hipSuccess) {                                                                      \
      cleanup();                                                                                 \
      return fail(UC_LP_EHIP, "%s failed: %s", #call, hipGetErrorString(e_));                    \
    }                                                                                            \
  } while (0)
  // scenario-major internal data -> interleaved scaled data on the device
  {
    for (int s = 0; s < S; ++s) {  // scenario-major, straight from each scenario's arrays
      SCEN_HIP(hipMemcpyAsync(A.c_in + (size_t)s * ni, SP[s].c.data(), (size_t)ni * 8, hipMemcpyHostToDevice, st));
      SCEN_HIP(hipMemcpyAsync(A.l_in + (size_t)s * ni, SP[s].l.data(), (size_t)ni * 8, hipMemcpyHostToDevice, st));
      SCEN_HIP(hipMemcpyAsync(A.u_in + (size_t)s * ni, SP[s].u.data(), (size_t)ni * 8, hipMemcpyHostToDevice, st));
      if (mi)
        SCEN_HIP(hipMemcpyAsync(A.b_in + (size_t)s * mi, SP[s].b.data(), (size_t)mi * 8, hipMemcpyHostToDevice, st));
    }
    launch_scale_vectors(A.c_in, A.l_in, A.u_in, A.b_in, base->D.dc, base->D.dr, ni, mi, S, (double*)A.d.c,
                         (double*)A.d.l, (double*)A.d.u, (double*)A.d.b, (float*)A.f.c, (float*)A.f.l,
                         (float*)A.f.u, (float*)A.f.b, st);
    SCEN_HIP(hipStreamSynchronize(st));
  }
  // primal weights from the scaled data
  std::vector<double> dr(mi), dc(ni);
  if (mi) SCEN_HIP(hipMemcpyAsync(dr.data(), base->D.dr, 8 * mi, hipMemcpyDeviceToHost, st));
  SCEN_HIP(hipMemcpyAsync(dc.data(), base->D.dc, 8 * ni, hipMemcpyDeviceToHost, st));
  SCEN_HIP(hipStreamSynchronize(st));
  std::vector<ChkState> ps(S);
  std::vector<ChkParams> pp(S);
  std::vector<uc_lp_info> inf(S);
  std::vector<int> done(S, 0), status(S, UC_LP_RUNNING);
  const double t0 = now_s();
  std::vector<double> cnorm(S), bnorm(S);
  fork_join(S, [&](int s) {
    double cn = 0, bn = 0;
    for (int j = 0; j < ni; ++j) cn += (SP[s].c[j] * dc[j]) * (SP[s].c[j] * dc[j]);
    for (int i = 0; i < mi; ++i) bn += (SP[s].b[i] * dr[i]) * (SP[s].b[i] * dr[i]);
    cnorm[s] = cn;
    bnorm[s] = bn;
  });
  for (int s = 0; s < S; ++s) {
    const double cn = cnorm[s], bn = bnorm[s];
    ps[s] = fresh_state(o.precision == UC_LP_FP64 ? 0 : 1, base->chk.eta,
                        (cn > 0 && bn > 0) ? std::sqrt(cn) / std::sqrt(bn) : 1.0);
    pp[s] = make_params(o, SP[s]);
    std::memset(&inf[s], 0, sizeof inf[s]);
    inf[s].t_to_eps_s = -1;
    const uc_lp_info bi = get_info(base);
    inf[s].norm_a_est = bi.norm_a_est;
    inf[s].norm_a_bound = bi.norm_a_bound;
    inf[s].eta = bi.eta;
    inf[s].m_presolved = mi;
    inf[s].n_presolved = ni;
    inf[s].nnz_presolved = P.nnzi;
    inf[s].device_bytes = (int64_t)bytes;
  }
  SlotDev SD = make_slot(base);
  SD.nscen = S;
  SD.f = A.f;
  SD.d = A.d;
  SD.f.av = base->D.a_v32;
  SD.f.tv = base->D.t_v32;
  SD.d.av = base->D.a_v64;
  SD.d.tv = base->D.t_v64;
  SD.f.avs = base->D.a_vs32;
  SD.f.tvs = base->D.t_vs32;
  SD.d.avs = base->D.a_vs64;
  SD.d.tvs = base->D.t_vs64;
  SD.part_a = A.part_a;
  SD.part_t = A.part_t;
  SD.scal = A.scal;
  SCEN_HIP(hipMemcpyAsync(A.slot_dev, &SD, sizeof SD, hipMemcpyHostToDevice, st));
  // warm start (the same point for every scenario), interleaved
  const double *xin = nullptr, *yin = nullptr;
  std::vector<double> wx, wy;
  if (x0 || y0) {
    wx.assign((size_t)ni * S, 0.0);
    wy.assign((size_t)mi * S, 0.0);
    for (int j = 0; j < ni; ++j)
      for (int s = 0; s < S; ++s) wx[(size_t)j * S + s] = x0 ? x0[P.col_map[j]] : 0.0;
    for (int i = 0; i < mi; ++i) {
      const int enc = P.row_map[i];
      const double v = y0 ? (enc >= 0 ? y0[enc] : -y0[-enc - 1]) : 0.0;
      for (int s = 0; s < S; ++s) wy[(size_t)i * S + s] = v;
    }
    SCEN_HIP(hipMemcpyAsync(A.x_warm, wx.data(), wx.size() * 8, hipMemcpyHostToDevice, st));
    if (mi) SCEN_HIP(hipMemcpyAsync(A.y_warm, wy.data(), wy.size() * 8, hipMemcpyHostToDevice, st));
    xin = A.x_warm;
    yin = A.y_warm;
  }
  int phase = o.precision == UC_LP_FP64 ? 0 : 1;
  launch_init_iterates(A.slot_dev, phase, xin, yin, ni, mi, P.m_eq, S, st);
  std::vector<Tile> tl;
  const int nt = (int)P.t_blk.size() - 1, na = (int)P.a_blk.size() - 1;
  push_tiles(tl, 0, P.t_blk, P.t_ptr, &tflag);
  push_tiles(tl, 0, P.a_blk, P.a_ptr, &aflag);
  SCEN_HIP(hipMemcpyAsync(A.tiles, tl.data(), tl.size() * sizeof(Tile), hipMemcpyHostToDevice, st));
  SCEN_HIP(hipStreamSynchronize(st));
  const Tile* TT = A.tiles;
  const Tile* TA = A.tiles + nt;
  const int K = o.kkt_every;
  // lane L of the interleaved arrays holds scenario lane[L]; all S at first
  std::vector<int> lane(S);
  for (int s = 0; s < S; ++s) lane[s] = s;
  int SL = S;
  int64_t NX = (int64_t)ni * S, NY = (int64_t)mi * S;
  std::vector<double> q((size_t)kScal * S);
  // final points of finished scenarios, unscaled, in the presolved numbering
  std::vector<std::vector<double>> px(S), py(S);
  std::vector<double> hx, hy;
  // at the end the last lanes are read from hx / hy in place (end_lane)
  std::vector<int> end_lane(S, -1);
  auto take_points = [&](int lanes, bool at_end) -> hipError_t {
    launch_unscale(A.slot_dev, phase, A.x_out, A.y_out, ni, mi, lanes, st);
    hx.resize((size_t)ni * lanes);
    hy.resize((size_t)mi * lanes);
    hipError_t e = hipMemcpyAsync(hx.data(), A.x_out, hx.size() * 8, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess && mi) e = hipMemcpyAsync(hy.data(), A.y_out, hy.size() * 8, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return e;
    std::vector<int> take;  // lanes whose scenario finished and has no point yet
    for (int L = 0; L < lanes; ++L) {
      const int s = lane[L];
      if (done[s] != 1 || !px[s].empty()) continue;
      if (at_end) {
        end_lane[s] = L;
        continue;
      }
      px[s].resize(ni);
      py[s].resize(mi);
      take.push_back(L);
    }
    if (take.empty()) return hipSuccess;
    const int nth = std::max(1, std::min(16, (int)std::thread::hardware_concurrency()));
    fork_join(nth, [&](int t) {  // each thread reads one range of the interleaved arrays in order
      const int j0 = (int)((int64_t)ni * t / nth), j1 = (int)((int64_t)ni * (t + 1) / nth);
      for (int j = j0; j < j1; ++j)
        for (int L : take) px[lane[L]][j] = hx[(size_t)j * lanes + L];
      const int i0 = (int)((int64_t)mi * t / nth), i1 = (int)((int64_t)mi * (t + 1) / nth);
      for (int i = i0; i < i1; ++i)
        for (int L : take) py[lane[L]][i] = hy[(size_t)i * lanes + L];
    });
    return hipSuccess;
  };
  // Moves the lanes `keep` of the current layout into new arrays holding
  // only them.  In the FP32 phase the FP32 iterates and data move, the FP64
  // data move and FP64 iterates are allocated for the hand-over; in the FP64
  // phase the FP64 iterates and data move.  Without device memory for the
  // new arrays the batch simply keeps its layout.
  bool no_compact = false;  // set when the device had no memory for it
  auto compact = [&](const std::vector<int>& keep) -> hipError_t {
    const int SC = (int)keep.size();
    const bool fp32 = phase == 1;
    Arena ar;
    Vecs<float> fn = SD.f;
    Vecs<double> dn = SD.d;
    float *fc = nullptr, *fl = nullptr, *fu = nullptr, *fb = nullptr;
    double *dc_ = nullptr, *dl = nullptr, *du = nullptr, *db = nullptr;
    void* nmem = nullptr;
    for (int pass = 0; pass < 2; ++pass) {
      if (pass == 1) {
        const size_t cbytes = ar.used + 256;
        if (hipMalloc(&nmem, cbytes) != hipSuccess) {
          (void)hipGetLastError();
          no_compact = true;
          return hipSuccess;
        }
        ar = Arena();
        ar.base = (char*)nmem;
        ar.bytes = cbytes;
      }
      dn.x = ar.take<double>((size_t)ni * SC);
      dn.x0 = ar.take<double>((size_t)ni * SC);
      dn.xbar = ar.take<double>((size_t)ni * SC);
      dn.xhat = ar.take<double>((size_t)ni * SC);
      dn.y = ar.take<double>((size_t)mi * SC);
      dn.y0 = ar.take<double>((size_t)mi * SC);
      dn.yhat = ar.take<double>((size_t)mi * SC);
      dc_ = ar.take<double>((size_t)ni * SC);
      dl = ar.take<double>((size_t)ni * SC);
      du = ar.take<double>((size_t)ni * SC);
      db = ar.take<double>((size_t)mi * SC);
      if (fp32) {
        fn.x = ar.take<float>((size_t)ni * SC);
        fn.x0 = ar.take<float>((size_t)ni * SC);
        fn.xbar = ar.take<float>((size_t)ni * SC);
        fn.xhat = ar.take<float>((size_t)ni * SC);
        fn.y = ar.take<float>((size_t)mi * SC);
        fn.y0 = ar.take<float>((size_t)mi * SC);
        fn.yhat = ar.take<float>((size_t)mi * SC);
        fc = ar.take<float>((size_t)ni * SC);
        fl = ar.take<float>((size_t)ni * SC);
        fu = ar.take<float>((size_t)ni * SC);
        fb = ar.take<float>((size_t)mi * SC);
      }
    }
    LaneMap mp;
    std::memset(&mp, 0, sizeof mp);
    mp.src_lanes = SL;
    mp.dst_lanes = SC;
    for (int k = 0; k < SC; ++k) mp.lane[k] = keep[k];
    // x and y carry the Halpern state; xhat and yhat the last check's point;
    // xbar is rewritten by the next primal half-step before it is read
    if (fp32) {
      launch_compact_lanes(SD.f.x, fn.x, ni, mp, st);
      launch_compact_lanes(SD.f.x0, fn.x0, ni, mp, st);
      launch_compact_lanes(SD.f.xhat, fn.xhat, ni, mp, st);
      launch_compact_lanes(SD.f.c, fc, ni, mp, st);
      launch_compact_lanes(SD.f.l, fl, ni, mp, st);
      launch_compact_lanes(SD.f.u, fu, ni, mp, st);
      launch_compact_lanes(SD.f.y, fn.y, mi, mp, st);
      launch_compact_lanes(SD.f.y0, fn.y0, mi, mp, st);
      launch_compact_lanes(SD.f.yhat, fn.yhat, mi, mp, st);
      launch_compact_lanes(SD.f.b, fb, mi, mp, st);
    } else {
      launch_compact_lanes(SD.d.x, dn.x, ni, mp, st);
      launch_compact_lanes(SD.d.x0, dn.x0, ni, mp, st);
      launch_compact_lanes(SD.d.xhat, dn.xhat, ni, mp, st);
      launch_compact_lanes(SD.d.y, dn.y, mi, mp, st);
      launch_compact_lanes(SD.d.y0, dn.y0, mi, mp, st);
      launch_compact_lanes(SD.d.yhat, dn.yhat, mi, mp, st);
    }
    launch_compact_lanes(SD.d.c, dc_, ni, mp, st);
    launch_compact_lanes(SD.d.l, dl, ni, mp, st);
    launch_compact_lanes(SD.d.u, du, ni, mp, st);
    launch_compact_lanes(SD.d.b, db, mi, mp, st);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipStreamSynchronize(st);  // the old arrays and slot table are released below
    if (e != hipSuccess) {
      (void)hipFree(nmem);
      return e;
    }
    if (cmem) (void)hipFree(cmem);
    cmem = nmem;
    dn.c = dc_;
    dn.l = dl;
    dn.u = du;
    dn.b = db;
    if (fp32) {
      fn.c = fc;
      fn.l = fl;
      fn.u = fu;
      fn.b = fb;
    } else {  // the FP32 arrays are not read again
      fn.x = fn.x0 = fn.xbar = fn.xhat = fn.y = fn.y0 = fn.yhat = nullptr;
      fn.c = fn.l = fn.u = fn.b = nullptr;
    }
    SD.f = fn;
    SD.d = dn;
    SD.nscen = SC;
    std::vector<int> nl(SC);
    for (int k = 0; k < SC; ++k) nl[k] = lane[keep[k]];
    lane = nl;
    SL = SC;
    NX = (int64_t)ni * SL;
    NY = (int64_t)mi * SL;
    return hipSuccess;
  };
  for (;;) {
    for (int L = 0; L < SL; ++L) {
      const int s = lane[L];
      SD.tau[L] = ps[s].eta / ps[s].omega;
      SD.sigma[L] = ps[s].eta * ps[s].omega;
      SD.k0[L] = ps[s].k_inner;
      SD.restart[L] = 0;
      SD.active[L] = done[s] ? 0 : 1;
    }
    SCEN_HIP(hipMemcpyAsync(A.slot_dev, &SD, sizeof SD, hipMemcpyHostToDevice, st));
    const bool vec = ms_vector_lanes(SD, phase, SL);
    for (int j = 0; j < K; ++j) {
      const bool check = j == K - 1;
      launch_primal_ms(phase, check, vec, A.slot_dev, TT, nt, j, st);
      launch_dual_ms(phase, check, vec, A.slot_dev, TA, na, j, st);
    }
    launch_kkt_ms(phase, A.slot_dev, TT, nt, TA, na, A.red2, st);
    SCEN_HIP(hipMemcpyAsync(q.data(), A.scal, (size_t)kScal * SL * 8, hipMemcpyDeviceToHost, st));
    SCEN_HIP(hipStreamSynchronize(st));
    SCEN_HIP(hipGetLastError());
    const double tnow = now_s();
    bool promote_ready = true, all_done = true;
    for (int L = 0; L < SL; ++L) {
      const int s = lane[L];
      if (done[s]) continue;
      const bool had_eps = ps[s].eps_reached != 0;
      int32_t stop = 0;
      if (base->cancel.load()) stop = UC_LP_CANCELLED;
      else if (tnow - t0 >= o.time_limit_s) stop = UC_LP_TIME_LIMIT;
      check_step(ps[s], pp[s], &q[(size_t)L * kScal], stop, 0);
      info_from_state(ps[s], inf[s]);
      inf[s].t_total_s = tnow - t0;
      if (!had_eps && ps[s].eps_reached) inf[s].t_to_eps_s = tnow - t0;
      if (o.verbose) print_check(ps[s]);
      SD.restart[L] = ps[s].restart;
      if (ps[s].status != UC_LP_RUNNING) {
        done[s] = 1;
        status[s] = ps[s].status;
      } else if (ps[s].promote) {
        done[s] = 2;  // waits, frozen, for the other scenarios of this phase
      }
    }
    // scenarios without a lane have finished (done = 1)
    for (int L = 0; L < SL; ++L) {
      const int s = lane[L];
      SD.active[L] = done[s] ? 0 : 1;
      promote_ready &= done[s] != 0;
      all_done &= done[s] == 1;
    }
    SCEN_HIP(hipMemcpyAsync(A.slot_dev, &SD, sizeof SD, hipMemcpyHostToDevice, st));
    launch_finish_ms(phase, A.slot_dev, NX, NY, K - 1, st);
    if (all_done) break;
    if (promote_ready) {
      // every scenario finished its FP32 phase: continue all waiting ones in FP64
      launch_promote_ms(A.slot_dev, NX, NY, st);
      phase = 0;
      for (int L = 0; L < SL; ++L)
        if (done[lane[L]] == 2) done[lane[L]] = 0;
    }
    // Once at most half the lanes hold a scenario that has not finished
    // (running, or waiting for the FP64 hand-over), the finished scenarios'
    // points are taken and the others continue on arrays that hold only
    // their lanes, so a batch iteration reads those lanes only.
    std::vector<int> keep;
    for (int L = 0; L < SL; ++L)
      if (done[lane[L]] != 1) keep.push_back(L);
    if (!no_compact && !keep.empty() && 2 * (int)keep.size() <= SL) {
      SCEN_HIP(take_points(SL, false));
      SCEN_HIP(compact(keep));
    }
  }
  SCEN_HIP(take_points(SL, true));
  for (int s = 0; s < S; ++s)
    if (end_lane[s] < 0 && (px[s].size() != (size_t)ni || py[s].size() != (size_t)mi)) {
      cleanup();
      return fail(UC_LP_EHIP, "scenario %d: no final point was taken", s);
    }
  const int SE = SL;
  auto xres = [&](int j, int s) {
    return end_lane[s] >= 0 ? hx[(size_t)j * SE + end_lane[s]] : px[s][j];
  };
  auto yres = [&](int i, int s) {
    return end_lane[s] >= 0 ? hy[(size_t)i * SE + end_lane[s]] : py[s][i];
  };
  cleanup();
#undef SCEN_HIP
  const double t_end = now_s();
  for (int s = 0; s < S; ++s) {
    inf[s].status = status[s];
    inf[s].t_total_s = t_end - t0;
    info[s] = inf[s];
  }
  // interleaved device order -> one array per scenario in the original
  // numbering: each host thread reads a contiguous range of the interleaved
  // results once and writes the S scenarios' entries of that range
  const int nth = std::max(1, std::min(16, (int)std::thread::hardware_concurrency()));
  fork_join(nth, [&](int t) {
    if (x) {
      const int j0 = (int)((int64_t)ni * t / nth), j1 = (int)((int64_t)ni * (t + 1) / nth);
      for (int j = j0; j < j1; ++j) {
        const int oj = P.col_map[j];
        for (int s = 0; s < S; ++s)
          x[(size_t)s * n + oj] = std::min(std::max(xres(j, s), SP[s].l[j]), SP[s].u[j]);
      }
      const int f0 = (int)((int64_t)n * t / nth), f1 = (int)((int64_t)n * (t + 1) / nth);
      for (int32_t j = f0; j < f1; ++j)
        if (P.int_col[j] < 0)
          for (int s = 0; s < S; ++s) x[(size_t)s * n + j] = SP[s].o_lb[j];
    }
    if (y) {
      const int r0 = (int)((int64_t)m * t / nth), r1 = (int)((int64_t)m * (t + 1) / nth);
      for (int s = 0; s < S; ++s) std::fill(y + (size_t)s * m + r0, y + (size_t)s * m + r1, 0.0);
    }
  });
  if (y)  // after every thread has cleared its rows: the presolved rows scatter anywhere
    fork_join(nth, [&](int t) {
      const int i0 = (int)((int64_t)mi * t / nth), i1 = (int)((int64_t)mi * (t + 1) / nth);
      for (int i = i0; i < i1; ++i) {
        const int enc = P.row_map[i];
        for (int s = 0; s < S; ++s) {
          const double v = yres(i, s);
          if (enc >= 0) y[(size_t)s * m + enc] = v;
          else y[(size_t)s * m + (-enc - 1)] = -v;
        }
      }
    });
  return UC_LP_OK;
}

// ---------------------------------------------------------------------------
// problem and solution in caller-owned device memory
// ---------------------------------------------------------------------------

// D2H copy of n elements on s (n = 0: nothing).
template <typename T>
static int read_device(std::vector<T>& dst, const T* src, size_t n, hipStream_t s) {
  dst.resize(n);
  if (n) HIPOK(hipMemcpyAsync(dst.data(), src, sizeof(T) * n, hipMemcpyDeviceToHost, s));
  return UC_LP_OK;
}

extern "C" int uc_lp_create_device(uc_engine* eng, int32_t m, int32_t n, int64_t nnz, const int32_t* row_ptr,
                                   const int32_t* col_idx, const double* val, const double* c, const double* b,
                                   const char* sense, const double* lb, const double* ub, const uc_lp_opts* opts,
                                   void* hip_stream, uc_lp** out) {
  g_err.clear();
  if (!out) return fail(UC_LP_EINVAL, "out is NULL");
  *out = nullptr;
  if (m < 1 || n < 1 || nnz < 0) return fail(UC_LP_EINVAL, "m=%d n=%d nnz=%lld", m, n, (long long)nnz);
  if (!row_ptr || !c || !b || !sense || !lb || !ub || (nnz > 0 && (!col_idx || !val)))
    return fail(UC_LP_EINVAL, "NULL array");
  const int device = eng ? eng->device : 0;
  int prev = 0;
  HIPOK(hipGetDevice(&prev));
  HIPOK(hipSetDevice(device));
  int rc = UC_LP_OK;
  const void* ptrs[8] = {row_ptr, col_idx, val, c, b, sense, lb, ub};
  const char* names[8] = {"row_ptr", "col_idx", "val", "c", "b", "sense", "lb", "ub"};
  for (int i = 0; i < 8 && rc == UC_LP_OK; ++i)
    if (ptrs[i]) rc = check_device_pointer(ptrs[i], device, names[i]);
  // deep copies to the host (the presolve and the row-block partition are
  // host work), read after what the caller enqueued on its stream
  std::vector<int32_t> hp, hc;
  std::vector<double> hv, hcst, hb, hl, hu;
  std::vector<char> hs;
  hipStream_t s = (hipStream_t)hip_stream;
  if (rc == UC_LP_OK) rc = read_device(hp, row_ptr, (size_t)m + 1, s);
  if (rc == UC_LP_OK && nnz) rc = read_device(hc, col_idx, (size_t)nnz, s);
  if (rc == UC_LP_OK && nnz) rc = read_device(hv, val, (size_t)nnz, s);
  if (rc == UC_LP_OK) rc = read_device(hcst, c, (size_t)n, s);
  if (rc == UC_LP_OK) rc = read_device(hb, b, (size_t)m, s);
  if (rc == UC_LP_OK) rc = read_device(hs, sense, (size_t)m, s);
  if (rc == UC_LP_OK) rc = read_device(hl, lb, (size_t)n, s);
  if (rc == UC_LP_OK) rc = read_device(hu, ub, (size_t)n, s);
  if (rc == UC_LP_OK) {
    const hipError_t e = hipStreamSynchronize(s);
    if (e != hipSuccess) rc = fail(UC_LP_EHIP, "reading the device arrays: %s", hipGetErrorString(e));
  }
  (void)hipSetDevice(prev);
  if (rc) return rc;
  return uc_lp_create(eng, m, n, nnz, hp.data(), nnz ? hc.data() : nullptr, nnz ? hv.data() : nullptr, hcst.data(),
                      hb.data(), hs.data(), hl.data(), hu.data(), opts, out);
}

extern "C" int uc_lp_get_solution_device(const uc_lp* lp, double* x, double* y, void* hip_stream) {
  g_err.clear();
  if (!lp) return fail(UC_LP_EINVAL, "NULL handle");
  const int s = lp->status.load();
  if (!(s == UC_LP_OPTIMAL || s == UC_LP_ITER_LIMIT || s == UC_LP_TIME_LIMIT || s == UC_LP_CANCELLED ||
        s == UC_LP_NUMERICAL))
    return fail(UC_LP_ESTATE, "no solution in status %d", s);
  if (lp->sol_x.size() != (size_t)lp->P.n) return fail(UC_LP_ESTATE, "solution not available");
  const int device = lp->eng->device;
  int prev = 0;
  HIPOK(hipGetDevice(&prev));
  HIPOK(hipSetDevice(device));
  int rc = UC_LP_OK;
  if (x) rc = check_device_pointer(x, device, "x");
  if (rc == UC_LP_OK && y) rc = check_device_pointer(y, device, "y");
  hipStream_t st = (hipStream_t)hip_stream;
  if (rc == UC_LP_OK && x) {
    const hipError_t e = hipMemcpyAsync(x, lp->sol_x.data(), sizeof(double) * lp->P.n, hipMemcpyHostToDevice, st);
    if (e != hipSuccess) rc = fail(UC_LP_EHIP, "copy of x: %s", hipGetErrorString(e));
  }
  if (rc == UC_LP_OK && y) {
    const hipError_t e = hipMemcpyAsync(y, lp->sol_y.data(), sizeof(double) * lp->P.m, hipMemcpyHostToDevice, st);
    if (e != hipSuccess) rc = fail(UC_LP_EHIP, "copy of y: %s", hipGetErrorString(e));
  }
  (void)hipSetDevice(prev);
  return rc;
}
