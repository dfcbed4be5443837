// Device kernels of libuclp (gfx950, wave64).
//
// Every hot kernel walks a list of tiles (slot, row block).  A row block is a
// run of consecutive CSR rows holding at most kRowsPerBlock rows and
// kNnzTile entries (or one longer row).  The kThreads threads of a workgroup
// first load the block's entries with coalesced reads, multiply them by the
// gathered vector entries and stage the products in LDS; then thread t sums
// row r0 + t from LDS in CSR order and runs the per-row epilogue
// (projection, extrapolation, Halpern averaging or KKT terms).  The
// summation order of a row therefore depends only on the matrix, so results
// are bitwise reproducible and independent of which other instances share a
// launch.
//
// Workgroups are dispatched round-robin over the 8 XCDs of the MI355X; the
// tile index is remapped so that each XCD walks one contiguous eighth of the
// tiles, which keeps the gathered vector window of that range in its own L2.

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>
#include <hipcub/hipcub.hpp>
#include <math.h>
#include <stdint.h>

#include "check.h"
#include "uclp_dev.h"

namespace uclp {

// ---------------------------------------------------------------------------
// helpers
// ---------------------------------------------------------------------------

constexpr int kXcd = 8;

__host__ __device__ inline int xcd_grid(int ntiles) {
  int per = (ntiles + kXcd - 1) / kXcd;
  return per * kXcd;
}

__device__ inline int xcd_tile(int ntiles) {
  int per = (ntiles + kXcd - 1) / kXcd;
  int w = blockIdx.x;
  int t = (w % kXcd) * per + (w / kXcd);
  return t < ntiles ? t : -1;
}

template <typename T>
__device__ inline T clampv(T v, T lo, T hi) {
  return v < lo ? lo : (v > hi ? hi : v);
}

template <typename T>
__device__ inline const Vecs<T>& vecs(const SlotDev& s);
template <>
__device__ inline const Vecs<float>& vecs<float>(const SlotDev& s) { return s.f; }
template <>
__device__ inline const Vecs<double>& vecs<double>(const SlotDev& s) { return s.d; }

// Block-wide sum (or max) of NQ doubles per thread; result valid in thread 0.
template <int NQ>
__device__ inline void block_reduce(double (&v)[NQ], const bool (&is_max)[NQ], double* red) {
  // red: LDS scratch of (kThreads / 64) * NQ doubles
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    double x = v[q];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      double o = __shfl_down(x, off, 64);
      x = is_max[q] ? fmax(x, o) : x + o;
    }
    v[q] = x;
  }
  if (lane == 0) {
#pragma unroll
    for (int q = 0; q < NQ; ++q) red[wave * NQ + q] = v[q];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      double x = red[q];
      for (int w = 1; w < kThreads / 64; ++w) x = is_max[q] ? fmax(x, red[w * NQ + q]) : x + red[w * NQ + q];
      v[q] = x;
    }
  }
}

// Row sums of one row block: products val[k] * g(k) staged in LDS, then summed
// per row in CSR order.  Thread t owns rows r0 + t + q * kThreads; f(row, sum)
// runs once per owned row.  A long row (one row above kNnzTile) is reduced by
// the whole block and reported to thread 0.
template <typename ACC, typename Prod, typename F>
__device__ inline void block_rows(const int* __restrict__ ptr, int r0, int r1, ACC* lds, ACC* red,
                                  Prod prod, F f) {
  const int k0 = ptr[r0];
  const int k1 = ptr[r1];
  const int nz = k1 - k0;
  if (nz <= kNnzTile) {
    if (nz > 0) {
      // all products' loads are issued before the first LDS store
      ACC v[kNnzTile / kThreads];
#pragma unroll
      for (int u = 0; u < kNnzTile / kThreads; ++u) v[u] = prod(k0 + min((int)threadIdx.x + u * kThreads, nz - 1));
#pragma unroll
      for (int u = 0; u < kNnzTile / kThreads; ++u)
        if ((int)threadIdx.x + u * kThreads < nz) lds[threadIdx.x + u * kThreads] = v[u];
    }
    __syncthreads();
    for (int r = r0 + threadIdx.x; r < r1; r += kThreads) {
      const int a = ptr[r] - k0;
      const int b = ptr[r + 1] - k0;
      ACC s = 0;
      for (int k = a; k < b; ++k) s += lds[k];
      f(r, s);
    }
    return;
  }
  // one long row
  ACC s = 0;
  for (int k = k0 + threadIdx.x; k < k1; k += kThreads) s += prod(k);
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    ACC t = red[0];
    for (int w = 1; w < kThreads / 64; ++w) t += red[w];
    f(r0, t);
  }
}

// ---------------------------------------------------------------------------
// PDHG half-steps (one scenario per slot)
// ---------------------------------------------------------------------------

// Pointers that the half-steps read through are cast to the global address
// space: loaded from the slot descriptor they are generic, and generic loads
// may alias LDS, which makes the compiler wait for each gather before the
// next product is written to LDS.
#define UCLP_GLOBAL __attribute__((address_space(1)))
template <typename T>
__device__ __forceinline__ const UCLP_GLOBAL T* gld(const T* p) {
  return (const UCLP_GLOBAL T*)p;
}
template <typename T>
__device__ __forceinline__ UCLP_GLOBAL T* gst(T* p) {
  return (UCLP_GLOBAL T*)p;
}

// Staging of one row block's products into LDS: every thread issues all of
// its (at most kNnzTile / NT) entry loads, then all gathers, so each wave
// keeps many independent loads in flight before the block barrier.
constexpr int kItems = kNnzTile / kThreads;

// The staging reads the block's entries in column order: the gathers of
// neighbouring lanes fall on neighbouring cache lines, and each product is
// written to its CSR position dst[k] so the per-row sums keep CSR order.
template <typename T, typename G, int NT = kThreads>
__device__ inline void stage_sorted(const int* cs_, const T* vs_, const unsigned short* dst_, const G* g_, int nz,
                                    T* lds) {
  // straight-line loads: items past the block's end re-read its last entry
  // and are not written, so all gathers of a thread are in flight together
  constexpr int kIt = kNnzTile / NT;
  if (nz <= 0) return;
  const UCLP_GLOBAL int* cs = gld(cs_);
  const UCLP_GLOBAL T* vs = gld(vs_);
  const UCLP_GLOBAL unsigned short* dst = gld(dst_);
  const UCLP_GLOBAL G* g = gld(g_);
  int c[kIt], d[kIt];
  T v[kIt], gv[kIt];
#pragma unroll
  for (int u = 0; u < kIt; ++u) {
    const int k = min((int)threadIdx.x + u * NT, nz - 1);
    c[u] = cs[k];
    v[u] = vs[k];
    d[u] = dst[k];
  }
#pragma unroll
  for (int u = 0; u < kIt; ++u) gv[u] = (T)g[c[u]];
#pragma unroll
  for (int u = 0; u < kIt; ++u)
    if ((int)threadIdx.x + u * NT < nz) lds[d[u]] = v[u] * gv[u];
}

// The same from the packed words: one 4-byte read per entry for index and slot.
template <typename T, typename G, int NT = kThreads>
__device__ inline void stage_packed(const unsigned* pk_, const T* vs_, int base, const G* g_, int nz, T* lds) {
  constexpr int kIt = kNnzTile / NT;
  if (nz <= 0) return;
  const UCLP_GLOBAL unsigned* pk = gld(pk_);
  const UCLP_GLOBAL T* vs = gld(vs_);
  const UCLP_GLOBAL G* gb = gld(g_) + base;
  unsigned p[kIt];
  T v[kIt], gv[kIt];
#pragma unroll
  for (int u = 0; u < kIt; ++u) {
    const int k = min((int)threadIdx.x + u * NT, nz - 1);
    p[u] = pk[k];
    v[u] = vs[k];
  }
#pragma unroll
  for (int u = 0; u < kIt; ++u) gv[u] = (T)gb[p[u] & kPackMask];
#pragma unroll
  for (int u = 0; u < kIt; ++u)
    if ((int)threadIdx.x + u * NT < nz) lds[p[u] >> kPackShift] = v[u] * gv[u];
}

// The entries of a row block that fits the LDS tile, in column order, kItems
// per thread: load(k, g) gets an entry's position k in the column-ordered
// arrays and its gathered index g and returns its value(s); store(slot, v)
// then writes them at the entry's CSR position.  All loads of a thread are
// issued before its first store (items past the block's end repeat its last
// entry and are not stored).
template <typename V, typename Load, typename Store>
__device__ inline void for_sorted(const Tile& tl, const unsigned* pk_, const int* cs_, const unsigned short* dst_,
                                  Load load, Store store) {
  const int k0 = tl.k0, nz = tl.k1 - tl.k0;
  if (nz <= 0) return;
  int kk[kItems], g[kItems], sl[kItems];
  if (tl.base >= 0) {
    const UCLP_GLOBAL unsigned* pk = gld(pk_);
#pragma unroll
    for (int u = 0; u < kItems; ++u) {
      kk[u] = k0 + min((int)threadIdx.x + u * kThreads, nz - 1);
      const unsigned p = pk[kk[u]];
      g[u] = tl.base + (int)(p & kPackMask);
      sl[u] = (int)(p >> kPackShift);
    }
  } else {
    const UCLP_GLOBAL int* cs = gld(cs_);
    const UCLP_GLOBAL unsigned short* dst = gld(dst_);
#pragma unroll
    for (int u = 0; u < kItems; ++u) {
      kk[u] = k0 + min((int)threadIdx.x + u * kThreads, nz - 1);
      g[u] = cs[kk[u]];
      sl[u] = (int)dst[kk[u]];
    }
  }
  V v[kItems];
#pragma unroll
  for (int u = 0; u < kItems; ++u) v[u] = load(kk[u], g[u]);
#pragma unroll
  for (int u = 0; u < kItems; ++u)
    if ((int)threadIdx.x + u * kThreads < nz) store(sl[u], v[u]);
}

// block_rows over a tile whose entries are also stored in column order: a
// block that fits the LDS tile stages psorted(k, g) (position k of the
// column-ordered arrays, gathered index g) at each entry's CSR position; a
// long row takes pcsr(k) in CSR order.  f(row, sum) runs for every row, with
// the row's products summed in CSR order either way.
template <typename ACC, typename PS, typename PC, typename F>
__device__ inline void block_rows_sorted(const Tile& tl, const int* __restrict__ ptr, const unsigned* pk,
                                         const int* cs, const unsigned short* dst, ACC* lds, ACC* red,
                                         PS psorted, PC pcsr, F f) {
  const int r0 = tl.r0, r1 = tl.r1, k0 = tl.k0, k1 = tl.k1;
  if (k1 - k0 <= kNnzTile) {
    for_sorted<ACC>(tl, pk, cs, dst, psorted, [&](int slot, ACC v) { lds[slot] = v; });
    __syncthreads();
    for (int r = r0 + threadIdx.x; r < r1; r += kThreads) {
      const int a = ptr[r] - k0;
      const int b = ptr[r + 1] - k0;
      ACC s = 0;
      for (int k = a; k < b; ++k) s += lds[k];
      f(r, s);
    }
    return;
  }
  ACC s = 0;
  for (int k = k0 + threadIdx.x; k < k1; k += kThreads) s += pcsr(k);
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    ACC t = red[0];
    for (int w = 1; w < kThreads / 64; ++w) t += red[w];
    f(r0, t);
  }
}

// Sum of one long row (above kNnzTile entries) by the whole block; valid in thread 0.
template <typename T, typename G, int NT = kThreads>
__device__ inline T long_row_sum(const int* __restrict__ col, const T* __restrict__ val,
                                 const G* __restrict__ g, int nz, T* red) {
  T s = 0;
  for (int k = threadIdx.x; k < nz; k += NT) s += val[k] * (T)g[col[k]];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  T t = red[0];
  for (int w = 1; w < NT / 64; ++w) t += red[w];
  return t;
}

// Primal half-step over the rows of A^T (= columns j of A):
//   g = c_j - (A^T y)_j ; x_hat = clamp(x - tau g, l, u) ; xbar = 2 x_hat - x
//   non-check: x <- w ((1+gamma) x_hat - gamma x) + (1 - w) x0 (w xbar at gamma = 1),
//              w = (k + 1)/(k + 2), 1 - w = 1/(k + 2)
//   check:     x_hat stored, x kept for the residuals
// At gamma = 1 the Halpern iterate is not stored between checks: x is read
// only by this kernel (the dual half-step gathers xbar), so the launch after
// another rebuilds it as w' xbar + (1 - w') x0 from the stored xbar and the
// anchor, with the previous launch's w'.  The first launch after a check
// reads x itself, and a check launch stores the rebuilt x for the KKT and
// finish kernels.
// NT threads per workgroup; thread t handles rows r0 + t + q * NT, q < kRowsPerBlock / NT.
template <typename T, bool CHECK, int NT>
__global__ __launch_bounds__(NT) void k_primal(const SlotDev* __restrict__ slots,
                                                     const Tile* __restrict__ tiles, int ntiles,
                                                     int jiter) {
  __shared__ T lds[kNnzTile];
  __shared__ T red[NT / 64];
  constexpr int kRpt = kRowsPerBlock / NT;
  const int t = xcd_tile(ntiles);
  if (t < 0) return;
  const Tile tl = tiles[t];
  const SlotDev& S = slots[tl.slot];
  if (!S.active[0]) return;  // frozen slot: finished or waiting for a precision switch
  const Vecs<T>& V = vecs<T>(S);
  const int r0 = tl.r0, r1 = tl.r1;
  const UCLP_GLOBAL unsigned short* rend = gld(S.t_end);
  const int k0 = tl.k0;
  const int nz = tl.k1 - k0;
  const int fl = tl.flags;
  const bool full = S.gamma == 1.0;  // full reflection: 2 x_hat - x is xbar itself
  const bool rebuild = full && jiter > 0;
  T wp = 0, wap = 0;
  if (rebuild) {
    const double kp = (double)(S.k0[0] + jiter - 1);
    wp = (T)((kp + 1.0) / (kp + 2.0));
    wap = (T)(1.0 / (kp + 2.0));
  }
  // epilogue operands first, so their loads overlap the gathers.  The loads
  // are straight-line: a thread past the block's last row loads that row
  // and skips the epilogue; values that depend on loads (x rebuilt, l = -u)
  // are formed after the barrier.
  int a[kRpt], b[kRpt];
  T c[kRpt], lr[kRpt], u[kRpt], xv[kRpt], xa[kRpt];
#pragma unroll
  for (int q = 0; q < kRpt; ++q) {
    const int j = min(r0 + (int)threadIdx.x + q * NT, r1 - 1);
    const int ap = rend[max(j - 1, r0)];
    a[q] = j == r0 ? 0 : ap;
    b[q] = rend[j];
    c[q] = (fl & kColC0) ? (T)0 : gld(V.c)[j];
    u[q] = (fl & kColUInf) ? (T)INFINITY : gld(V.u)[j];
    lr[q] = (fl & (kColL0 | kColLInf | kColLNegU)) ? (T)0 : gld(V.l)[j];
    xa[q] = 0;
    if (rebuild) {
      xa[q] = gld(V.x0)[j];
      xv[q] = gld(V.xbar)[j];
    } else {
      xv[q] = gld(V.x)[j];
      if (!CHECK) xa[q] = gld(V.x0)[j];
    }
  }
  T s[kRpt];
  if (nz <= kNnzTile) {
    if (tl.base >= 0)
      stage_packed<T, T, NT>(S.t_pk + k0, V.tvs + k0, tl.base, V.y, nz, lds);
    else
      stage_sorted<T, T, NT>(S.t_cs + k0, V.tvs + k0, S.t_dst + k0, V.y, nz, lds);
    __syncthreads();
#pragma unroll
    for (int q = 0; q < kRpt; ++q) {
      T acc = 0;
      for (int k = a[q]; k < b[q]; ++k) acc += lds[k];
      s[q] = acc;
    }
  } else {
    s[0] = long_row_sum<T, T, NT>(S.t_col + k0, V.tv + k0, V.y, nz, red);
    if (threadIdx.x != 0) return;
  }
  const T tau = (T)S.tau[0];
  const double kk = (double)(S.k0[0] + jiter);
  const T w = (T)((kk + 1.0) / (kk + 2.0));
  const T wa = (T)(1.0 / (kk + 2.0));
#pragma unroll
  for (int q = 0; q < kRpt; ++q) {
    const int j = r0 + threadIdx.x + q * NT;
    if (j >= r1) break;
    const T x = rebuild ? wp * xv[q] + wap * xa[q] : xv[q];
    const T l = (fl & kColL0) ? (T)0 : (fl & kColLInf) ? -(T)INFINITY : (fl & kColLNegU) ? -u[q] : lr[q];
    const T xh = clampv<T>(x - tau * (c[q] - s[q]), l, u[q]);
    const T xb = (T)2 * xh - x;
    gst(V.xbar)[j] = xb;
    if (CHECK) {
      gst(V.xhat)[j] = xh;
      if (rebuild) gst(V.x)[j] = x;
    } else if (!full) {
      gst(V.x)[j] = w * ((T)(1.0 + S.gamma) * xh - (T)S.gamma * x) + wa * xa[q];
    }
  }
}

// Dual half-step over the rows of A:
//   y_hat = y + sigma (b - A xbar), projected to y >= 0 on rows i >= m_eq
//   (y >= ylo in tiles flagged kRowYlo: the correction problems of
//   iterative refinement)
//   non-check: y <- w ((1+gamma) y_hat - gamma y) + (1 - w) y0 ; check: y_hat stored
template <typename T, bool CHECK, int NT>
__global__ __launch_bounds__(NT) void k_dual(const SlotDev* __restrict__ slots,
                                                   const Tile* __restrict__ tiles, int ntiles,
                                                   int jiter) {
  __shared__ T lds[kNnzTile];
  __shared__ T red[NT / 64];
  constexpr int kRpt = kRowsPerBlock / NT;
  const int t = xcd_tile(ntiles);
  if (t < 0) return;
  const Tile tl = tiles[t];
  const SlotDev& S = slots[tl.slot];
  if (!S.active[0]) return;
  const Vecs<T>& V = vecs<T>(S);
  const int r0 = tl.r0, r1 = tl.r1;
  const UCLP_GLOBAL unsigned short* rend = gld(S.a_end);
  const int k0 = tl.k0;
  const int nz = tl.k1 - k0;
  // straight-line epilogue loads, as in k_primal
  int a[kRpt], b[kRpt];
  T bi[kRpt], y[kRpt], ya[kRpt], lo[kRpt];
  const bool ylo = tl.flags & kRowYlo;
#pragma unroll
  for (int q = 0; q < kRpt; ++q) {
    const int i = min(r0 + (int)threadIdx.x + q * NT, r1 - 1);
    const int ap = rend[max(i - 1, r0)];
    a[q] = i == r0 ? 0 : ap;
    b[q] = rend[i];
    bi[q] = (tl.flags & kRowB0) ? (T)0 : gld(V.b)[i];
    y[q] = gld(V.y)[i];
    ya[q] = CHECK ? (T)0 : gld(V.y0)[i];
    lo[q] = ylo ? (T)gld(S.ylo)[i] : (T)0;
  }
  T s[kRpt];
  if (nz <= kNnzTile) {
    if (tl.base >= 0)
      stage_packed<T, T, NT>(S.a_pk + k0, V.avs + k0, tl.base, V.xbar, nz, lds);
    else
      stage_sorted<T, T, NT>(S.a_cs + k0, V.avs + k0, S.a_dst + k0, V.xbar, nz, lds);
    __syncthreads();
#pragma unroll
    for (int q = 0; q < kRpt; ++q) {
      T acc = 0;
      for (int k = a[q]; k < b[q]; ++k) acc += lds[k];
      s[q] = acc;
    }
  } else {
    s[0] = long_row_sum<T, T, NT>(S.a_col + k0, V.av + k0, V.xbar, nz, red);
    if (threadIdx.x != 0) return;
  }
  const T sigma = (T)S.sigma[0];
  const double kk = (double)(S.k0[0] + jiter);
  const T w = (T)((kk + 1.0) / (kk + 2.0));
  const T wa = (T)(1.0 / (kk + 2.0));
  const T g1 = (T)(1.0 + S.gamma), g = (T)S.gamma;
#pragma unroll
  for (int q = 0; q < kRpt; ++q) {
    const int i = r0 + threadIdx.x + q * NT;
    if (i >= r1) break;
    T yh = y[q] + sigma * (bi[q] - s[q]);
    if (i >= S.m_eq) yh = yh > lo[q] ? yh : lo[q];
    if (CHECK) gst(V.yhat)[i] = yh;
    else gst(V.y)[i] = w * (g1 * yh - g * y[q]) + wa * ya[q];
  }
}

// KKT check over the rows of A (FP64 values, FP64 accumulation):
//   s1 = (A x_hat)_i, s2 = (A (x_hat - x))_i
//   unscaled violation r_i = (b_i - s1)/D_r,i (G rows: max(0, .))
template <typename T>
__global__ __launch_bounds__(kThreads) void k_kkt_rows(const SlotDev* __restrict__ slots,
                                                       const Tile* __restrict__ tiles, int ntiles) {
  __shared__ double lds1[kNnzTile];
  __shared__ double lds2[kNnzTile];
  __shared__ double red[(kThreads / 64) * RQ_N];
  const int t = xcd_tile(ntiles);
  if (t < 0) return;
  const Tile tl = tiles[t];
  const SlotDev& S = slots[tl.slot];
  if (!S.active[0]) return;
  const Vecs<T>& V = vecs<T>(S);
  const int r0 = tl.r0, r1 = tl.r1;
  const int* __restrict__ ptr = S.a_ptr;
  const int* __restrict__ col = S.a_col;
  const double* __restrict__ val = S.d.av;
  const T* __restrict__ xh = V.xhat;
  const T* __restrict__ x = V.x;
  const int k0 = tl.k0;
  const int k1 = tl.k1;
  const int nz = k1 - k0;
  double q[RQ_N] = {0, 0, 0, 0, 0, 0, 0, 0};
  const bool is_max[RQ_N] = {false, false, false, false, false, false, true, false};
  const bool ylo = tl.flags & kRowYlo;
  auto row_terms = [&](int row, double s1, double s2) {
    const bool ineq = row >= S.m_eq;
    double r = S.d.b[row] - s1;
    if (ineq) r = r > 0.0 ? r : 0.0;
    const double ru = r / S.dr[row];
    const double yh = (double)V.yhat[row];
    const double dy = yh - (double)V.y[row];
    const double d0 = yh - (double)V.y0[row];
    const double lo = ineq && ylo ? (double)S.ylo[row] : 0.0;
    q[RQ_RES2] += ru * ru;
    q[RQ_BY] += S.d.b[row] * yh;
    q[RQ_DY2] += dy * dy;
    q[RQ_DYADX] += dy * s2;
    q[RQ_DY0] += d0 * d0;
    // dual sign violation of an inequality row, unscaled (zero for projected iterates)
    const double yneg = ineq && yh < lo ? (yh - lo) * S.dr[row] : 0.0;
    q[RQ_YNEG2] += yneg * yneg;
    q[RQ_RESMAX] = fmax(q[RQ_RESMAX], fabs(ru));
    q[RQ_YLOR] += lo * (s1 - S.d.b[row]);
  };
  if (nz <= kNnzTile) {
    const UCLP_GLOBAL double* vs = gld(S.d.avs);
    const UCLP_GLOBAL T* gxh = gld(xh);
    const UCLP_GLOBAL T* gx = gld(x);
    struct P2 {
      double p1, p2;
    };
    for_sorted<P2>(
        tl, S.a_pk, S.a_cs, S.a_dst,
        [&](int k, int c) {
          const double v = vs[k];
          const double a = (double)gxh[c];
          return P2{v * a, v * (a - (double)gx[c])};
        },
        [&](int slot, P2 p) {
          lds1[slot] = p.p1;
          lds2[slot] = p.p2;
        });
    __syncthreads();
    for (int r = r0 + threadIdx.x; r < r1; r += kThreads) {
      double s1 = 0, s2 = 0;
      for (int k = ptr[r] - k0; k < ptr[r + 1] - k0; ++k) {
        s1 += lds1[k];
        s2 += lds2[k];
      }
      row_terms(r, s1, s2);
    }
  } else {
    double s1 = 0, s2 = 0;
    for (int k = k0 + threadIdx.x; k < k1; k += kThreads) {
      const int c = col[k];
      const double a = (double)xh[c];
      s1 += val[k] * a;
      s2 += val[k] * (a - (double)x[c]);
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      s1 += __shfl_down(s1, off, 64);
      s2 += __shfl_down(s2, off, 64);
    }
    if ((threadIdx.x & 63) == 0) {
      lds1[threadIdx.x >> 6] = s1;
      lds2[threadIdx.x >> 6] = s2;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      s1 = lds1[0];
      s2 = lds2[0];
      for (int w = 1; w < kThreads / 64; ++w) {
        s1 += lds1[w];
        s2 += lds2[w];
      }
      row_terms(r0, s1, s2);
    }
  }
  __syncthreads();
  block_reduce<RQ_N>(q, is_max, red);
  if (threadIdx.x == 0) {
    double* out = S.part_a + (size_t)tl.blk * RQ_N;
#pragma unroll
    for (int k = 0; k < RQ_N; ++k) out[k] = q[k];
  }
}

// KKT check over the rows of A^T: reduced cost d_hat = c_j - (A^T y_hat)_j,
// bound multiplier by finiteness of the bounds, unscaled by 1/D_c.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_kkt_cols(const SlotDev* __restrict__ slots,
                                                       const Tile* __restrict__ tiles, int ntiles) {
  __shared__ double lds[kNnzTile];
  __shared__ double red[(kThreads / 64) * RQ_N];
  const int t = xcd_tile(ntiles);
  if (t < 0) return;
  const Tile tl = tiles[t];
  const SlotDev& S = slots[tl.slot];
  if (!S.active[0]) return;
  const Vecs<T>& V = vecs<T>(S);
  const int r0 = tl.r0, r1 = tl.r1;
  const int* __restrict__ col = S.t_col;
  const double* __restrict__ val = S.d.tv;
  const T* __restrict__ yh = V.yhat;
  double q[CQ_N] = {0, 0, 0, 0, 0};
  const bool is_max[CQ_N] = {false, false, false, false, false};
  const double* __restrict__ vs = S.d.tvs;
  const UCLP_GLOBAL double* gvs = gld(vs);
  const UCLP_GLOBAL T* gyh = gld(yh);
  block_rows_sorted<double>(tl, S.t_ptr, S.t_pk, S.t_cs, S.t_dst, lds, red,
                     [&](int k, int c) { return gvs[k] * (double)gyh[c]; },
                     [&](int k) { return val[k] * (double)yh[col[k]]; },
                     [&](int j, double s) {
                       const double c = S.d.c[j];
                       const double l = S.d.l[j];
                       const double u = S.d.u[j];
                       const double dh = c - s;
                       const bool fl = isfinite(l);
                       const bool fu = isfinite(u);
                       double lam = 0.0;
                       if (fl && fu) lam = dh;
                       else if (fl) lam = dh > 0.0 ? dh : 0.0;
                       else if (fu) lam = dh < 0.0 ? dh : 0.0;
                       const double dres = (dh - lam) / S.dc[j];
                       const double xhv = (double)V.xhat[j];
                       const double dx = xhv - (double)V.x[j];
                       const double d0 = xhv - (double)V.x0[j];
                       q[CQ_DRES2] += dres * dres;
                       q[CQ_LBUB] += (lam > 0.0 ? l * lam : 0.0) + (lam < 0.0 ? u * lam : 0.0);
                       q[CQ_CX] += c * xhv;
                       q[CQ_DX2] += dx * dx;
                       q[CQ_DX0] += d0 * d0;
                     });
  __syncthreads();
  block_reduce<CQ_N>(q, is_max, red);
  if (threadIdx.x == 0) {
    double* out = S.part_t + (size_t)tl.blk * CQ_N;
#pragma unroll
    for (int k = 0; k < CQ_N; ++k) out[k] = q[k];
  }
}

// Final reduction of the block partials of one slot, in block order.
__global__ __launch_bounds__(kThreads) void k_reduce_part(const SlotDev* __restrict__ slots,
                                                          const int* __restrict__ ids,
                                                          double* __restrict__ red2) {
  constexpr int NQ = RQ_N + CQ_N;
  __shared__ double red[(kThreads / 64) * NQ];
  const SlotDev& S = slots[ids[blockIdx.y]];
  const int g = blockIdx.x;
  double q[NQ];
  bool is_max[NQ];
#pragma unroll
  for (int k = 0; k < NQ; ++k) {
    q[k] = 0.0;
    is_max[k] = (k == RQ_RESMAX);
  }
  const int a0 = (int)((int64_t)S.a_nblk * g / kRedChunks), a1 = (int)((int64_t)S.a_nblk * (g + 1) / kRedChunks);
  for (int b = a0 + (int)threadIdx.x; b < a1; b += kThreads) {
    const double* p = S.part_a + (size_t)b * RQ_N;
#pragma unroll
    for (int k = 0; k < RQ_N; ++k) q[k] = is_max[k] ? fmax(q[k], p[k]) : q[k] + p[k];
  }
  const int t0 = (int)((int64_t)S.t_nblk * g / kRedChunks), t1 = (int)((int64_t)S.t_nblk * (g + 1) / kRedChunks);
  for (int b = t0 + (int)threadIdx.x; b < t1; b += kThreads) {
    const double* p = S.part_t + (size_t)b * CQ_N;
#pragma unroll
    for (int k = 0; k < CQ_N; ++k) q[RQ_N + k] += p[k];
  }
  block_reduce<NQ>(q, is_max, red);
  if (threadIdx.x == 0) {
    double* out = red2 + ((size_t)blockIdx.y * kRedChunks + g) * NQ;
#pragma unroll
    for (int k = 0; k < NQ; ++k) out[k] = q[k];
  }
}

__global__ __launch_bounds__(kThreads) void k_reduce(const SlotDev* __restrict__ slots,
                                                     const int* __restrict__ ids,
                                                     const double* __restrict__ red2) {
  constexpr int NQ = RQ_N + CQ_N;
  __shared__ double red[(kThreads / 64) * NQ];
  const SlotDev& S = slots[ids[blockIdx.x]];
  double q[NQ];
  bool is_max[NQ];
#pragma unroll
  for (int k = 0; k < NQ; ++k) {
    q[k] = 0.0;
    is_max[k] = (k == RQ_RESMAX);
  }
  for (int g = threadIdx.x; g < kRedChunks; g += kThreads) {
    const double* p = red2 + ((size_t)blockIdx.x * kRedChunks + g) * NQ;
#pragma unroll
    for (int k = 0; k < NQ; ++k) q[k] = is_max[k] ? fmax(q[k], p[k]) : q[k] + p[k];
  }
  block_reduce<NQ>(q, is_max, red);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < NQ; ++k) S.scal[k] = q[k];
  }
}

// After a check: restart at (x_hat, y_hat) (flag 1), take the Halpern step and
// restart there (flag 2), or take the Halpern step (flag 0).
template <typename T>
__global__ __launch_bounds__(kThreads) void k_finish_x(const SlotDev* __restrict__ slots,
                                                       const Tile* __restrict__ tiles, int ntiles,
                                                       int kk) {
  const int t = xcd_tile(ntiles);
  if (t < 0) return;
  const Tile tl = tiles[t];
  const SlotDev& S = slots[tl.slot];
  if (!S.active[0]) return;
  const Vecs<T>& V = vecs<T>(S);
  const double k = (double)(S.kfin + kk);
  const T w = (T)((k + 1.0) / (k + 2.0));
  const T wa = (T)(1.0 / (k + 2.0));
  for (int j = tl.r0 + threadIdx.x; j < tl.r1; j += kThreads) {
    if (S.restart[0] == 1) {
      const T xh = V.xhat[j];
      V.x[j] = xh;
      V.x0[j] = xh;
    } else {
      const T refl = S.gamma == 1.0 ? V.xbar[j] : (T)(1.0 + S.gamma) * V.xhat[j] - (T)S.gamma * V.x[j];
      const T xn = w * refl + wa * V.x0[j];
      V.x[j] = xn;
      if (S.restart[0] == 2) V.x0[j] = xn;
    }
  }
}

template <typename T>
__global__ __launch_bounds__(kThreads) void k_finish_y(const SlotDev* __restrict__ slots,
                                                       const Tile* __restrict__ tiles, int ntiles,
                                                       int kk) {
  const int t = xcd_tile(ntiles);
  if (t < 0) return;
  const Tile tl = tiles[t];
  const SlotDev& S = slots[tl.slot];
  if (!S.active[0]) return;
  const Vecs<T>& V = vecs<T>(S);
  const double k = (double)(S.kfin + kk);
  const T w = (T)((k + 1.0) / (k + 2.0));
  const T wa = (T)(1.0 / (k + 2.0));
  for (int i = tl.r0 + threadIdx.x; i < tl.r1; i += kThreads) {
    if (S.restart[0] == 1) {
      const T yh = V.yhat[i];
      V.y[i] = yh;
      V.y0[i] = yh;
    } else {
      const T yn = w * ((T)(1.0 + S.gamma) * V.yhat[i] - (T)S.gamma * V.y[i]) + wa * V.y0[i];
      V.y[i] = yn;
      if (S.restart[0] == 2) V.y0[i] = yn;
    }
  }
}

// FP32 -> FP64 switch: the FP64 phase starts (as a restart) at the FP32 x_hat, y_hat.
__global__ __launch_bounds__(kThreads) void k_promote_x(const SlotDev* __restrict__ slots,
                                                        const Tile* __restrict__ tiles, int ntiles) {
  const int t = xcd_tile(ntiles);
  if (t < 0) return;
  const Tile tl = tiles[t];
  const SlotDev& S = slots[tl.slot];
  for (int j = tl.r0 + threadIdx.x; j < tl.r1; j += kThreads) {
    const double v = (double)S.f.xhat[j];
    S.d.x[j] = v;
    S.d.x0[j] = v;
    S.d.xhat[j] = v;
  }
}

__global__ __launch_bounds__(kThreads) void k_promote_y(const SlotDev* __restrict__ slots,
                                                        const Tile* __restrict__ tiles, int ntiles) {
  const int t = xcd_tile(ntiles);
  if (t < 0) return;
  const Tile tl = tiles[t];
  const SlotDev& S = slots[tl.slot];
  for (int i = tl.r0 + threadIdx.x; i < tl.r1; i += kThreads) {
    const double v = (double)S.f.yhat[i];
    S.d.y[i] = v;
    S.d.y0[i] = v;
    S.d.yhat[i] = v;
  }
}

// The engine's per-check decisions on the device: one thread per slot runs
// the check of its run on the reduced scalars, then sets what the finish
// kernel and the next epoch read (restart flag, Halpern index, steps).  A run
// that ends, or whose FP32 phase ends, is frozen (active = 0) until the host
// retires or switches it.
__global__ void k_engine_check(SlotDev* __restrict__ slots, ChkState* __restrict__ chk,
                               const ChkParams* __restrict__ prm, int nslots) {
  const int a = blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= nslots) return;
  SlotDev& S = slots[a];
  if (!S.active[0]) return;
  ChkState st = chk[a];
  if (st.status != UC_LP_RUNNING) return;
  const ChkParams p = prm[a];
  const long long k0 = S.k0[0];
  check_step(st, p, S.scal, 0, wall_clock64());
  S.kfin = k0 + p.K - 1;  // the check step the finish kernel completes
  S.restart[0] = st.restart;
  S.k0[0] = st.k_inner;
  S.tau[0] = st.eta / st.omega;
  S.sigma[0] = st.eta * st.omega;
  if (st.status != UC_LP_RUNNING || st.promote) S.active[0] = 0;
  chk[a] = st;
}

__global__ void k_stamp(unsigned long long* t) {
  if (blockIdx.x == 0 && threadIdx.x == 0) *t = wall_clock64();
}

// ---------------------------------------------------------------------------
// iterative refinement: the round boundary of one instance (FP64, scaled space)
// ---------------------------------------------------------------------------

// Smallest float >= v and largest float <= v (infinities pass through).
__device__ inline float f32_up(double v) {
  float f = (float)v;
  if ((double)f < v) f = nextafterf(f, INFINITY);
  return f;
}
__device__ inline float f32_down(double v) {
  float f = (float)v;
  if ((double)f > v) f = nextafterf(f, -INFINITY);
  return f;
}

// x* <- clamp(x* + x~ / D_P, l_hat, u_hat), y* <- y* + y~ / D_D (>= 0 on
// inequality rows); `first`: x* = y* = 0 before.
__global__ void k_refine_fold(RefineArgs R) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < R.n) {
    const double d = R.dc[i];
    const double l = R.l_in[i] / d, u = R.u_in[i] / d;
    const double v = (R.first ? 0.0 : R.xs[i]) + (double)R.xc[i] * R.inv_dp;
    R.xs[i] = fmin(fmax(v, l), u);
  } else if (i < (int64_t)R.n + R.m) {
    const int r = (int)(i - R.n);
    double v = (R.first ? 0.0 : R.ys[r]) + (double)R.yc[r] * R.inv_dd;
    if (r >= R.m_eq) v = fmax(v, 0.0);
    R.ys[r] = v;
  }
}

constexpr int kFq = 5;  // FQ partials per row block (rows: FQ_VIOL2.., cols: FQ_DRES2..)

// r = b_hat - A_hat x* over one row block of A, with the row FQ partials.
__global__ __launch_bounds__(kThreads) void k_refine_rows(RefineArgs R) {
  __shared__ double lds[kNnzTile];
  __shared__ double red[(kThreads / 64) * kFq];
  const int bk = blockIdx.x;
  double q[kFq] = {0, 0, 0, 0, 0};
  const bool is_max[kFq] = {false, false, false, false, true};
  block_rows<double>(
      R.a_ptr, R.a_blk[bk], R.a_blk[bk + 1], lds, red, [&](int k) { return R.a_v[k] * R.xs[R.a_col[k]]; },
      [&](int i, double s) {
        const double dr = R.dr[i];
        const double bh = R.b_in[i] * dr;
        const double r = bh - s;
        const double v = i >= R.m_eq ? fmax(r, 0.0) : r;
        const double ru = r / dr, vu = v / dr;
        R.r[i] = r;
        q[0] += v * v;
        q[1] += ru * ru;
        q[2] += vu * vu;
        q[3] += bh * R.ys[i];
        q[4] = fmax(q[4], fabs(vu));
      });
  __syncthreads();
  block_reduce<kFq>(q, is_max, red);
  if (threadIdx.x == 0)
    for (int k = 0; k < kFq; ++k) R.part_a[(size_t)bk * kFq + k] = q[k];
}

// d = c_hat - A_hat' y* over one row block of A^T, with the column FQ partials.
__global__ __launch_bounds__(kThreads) void k_refine_cols(RefineArgs R) {
  __shared__ double lds[kNnzTile];
  __shared__ double red[(kThreads / 64) * kFq];
  const int bk = blockIdx.x;
  double q[kFq] = {0, 0, 0, 0, 0};
  const bool is_max[kFq] = {false, false, false, false, false};
  block_rows<double>(
      R.t_ptr, R.t_blk[bk], R.t_blk[bk + 1], lds, red, [&](int k) { return R.t_v[k] * R.ys[R.t_col[k]]; },
      [&](int j, double s) {
        const double dc = R.dc[j];
        const double c = R.c_in[j] * dc, l = R.l_in[j] / dc, u = R.u_in[j] / dc;
        const double dh = c - s;
        const bool fl = isfinite(l), fu = isfinite(u);
        double lam = 0.0;
        if (fl && fu) lam = dh;
        else if (fl) lam = dh > 0.0 ? dh : 0.0;
        else if (fu) lam = dh < 0.0 ? dh : 0.0;
        const double e = dh - lam;
        const double du = dh / dc, eu = e / dc;
        R.d[j] = dh;
        q[0] += e * e;
        q[1] += du * du;
        q[2] += eu * eu;
        q[3] += (lam > 0.0 ? l * lam : 0.0) + (lam < 0.0 ? u * lam : 0.0);
        q[4] += c * R.xs[j];
      });
  __syncthreads();
  block_reduce<kFq>(q, is_max, red);
  if (threadIdx.x == 0)
    for (int k = 0; k < kFq; ++k) R.part_t[(size_t)bk * kFq + k] = q[k];
}

// One workgroup: the block partials in a fixed order -> R.out[FQ_N].
__global__ __launch_bounds__(kThreads) void k_refine_reduce(RefineArgs R) {
  __shared__ double red[(kThreads / 64) * FQ_N];
  double q[FQ_N];
  bool is_max[FQ_N];
#pragma unroll
  for (int k = 0; k < FQ_N; ++k) {
    q[k] = 0.0;
    is_max[k] = k == FQ_VMAXU;
  }
  for (int b = threadIdx.x; b < R.a_nblk; b += kThreads)
#pragma unroll
    for (int k = 0; k < kFq; ++k) {
      const double v = R.part_a[(size_t)b * kFq + k];
      q[k] = is_max[k] ? fmax(q[k], v) : q[k] + v;
    }
  for (int b = threadIdx.x; b < R.t_nblk; b += kThreads)
#pragma unroll
    for (int k = 0; k < kFq; ++k) q[kFq + k] += R.part_t[(size_t)b * kFq + k];
  block_reduce<FQ_N>(q, is_max, red);
  if (threadIdx.x == 0)
    for (int k = 0; k < FQ_N; ++k) R.out[k] = q[k];
}

// Correction data of the next round (FP64, and FP32 rounded so that every
// FP32-feasible correction maps back into the FP64 box and onto y >= 0).
__global__ void k_refine_form(RefineArgs R) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < R.n) {
    const double dc = R.dc[i];
    const double l = R.l_in[i] / dc, u = R.u_in[i] / dc;
    const double x = R.xs[i];
    const double ct = R.dd * R.d[i];
    const double lt = R.dp * (l - x), ut = R.dp * (u - x);
    R.c64[i] = ct;
    R.l64[i] = lt;
    R.u64[i] = ut;
    float lo = f32_up(lt), hi = f32_down(ut);
    if (lo > hi) lo = hi = (float)((lt + ut) / 2);
    R.c32[i] = (float)ct;
    R.l32[i] = lo;
    R.u32[i] = hi;
  } else if (i < (int64_t)R.n + R.m) {
    const int r = (int)(i - R.n);
    const double bt = R.dp * R.r[r];
    R.b64[r] = bt;
    R.b32[r] = (float)bt;
    R.ylo32[r] = r >= R.m_eq ? f32_up(-R.dd * R.ys[r]) : -INFINITY;
  }
}

// ---------------------------------------------------------------------------
// scenario batches: several right-hand sides / costs / bounds over one matrix
// ---------------------------------------------------------------------------
// Vectors are interleaved (element j of scenario s at j * nscen + s).  A
// workgroup stages the column indices and values of its row block in LDS
// once; lane s of each 16-lane group then walks one row for scenario s, so
// the 16 scenarios of a gathered element form one contiguous 64-byte (FP32)
// access, and one read of the matrix serves every scenario.
constexpr int kLanes = 16;                       // lanes per row (>= nscen)
constexpr int kRowsPerPass = kThreads / kLanes;  // rows per pass of the block
constexpr int kMsUnroll = 4;                     // rows per thread in flight

// One row's dot product for scenario sc from the staged entries [a, b): the
// first kMsDot entries are unrolled (predicated) so their gathers issue
// together, in entry order; longer rows continue in a loop.
constexpr int kMsDot = 4;

template <typename T>
__device__ inline T row_dot_ms(int a, int b, const int* lc, const T* lv, const UCLP_GLOBAL T* g, int ns, int sc) {
  T s = 0;
  if (b <= a) return s;
  T v[kMsDot], p[kMsDot];
#pragma unroll
  for (int t = 0; t < kMsDot; ++t) {
    const int k = min(a + t, b - 1);
    v[t] = lv[k];
    p[t] = g[(size_t)lc[k] * ns + sc];
  }
#pragma unroll
  for (int t = 0; t < kMsDot; ++t)
    if (a + t < b) s += v[t] * p[t];
  for (int k = a + kMsDot; k < b; ++k) s += lv[k] * g[(size_t)lc[k] * ns + sc];
  return s;
}

template <typename T>
__device__ inline T row_dot_ms_global(int a, int b, const int* __restrict__ col, const T* __restrict__ val,
                                      const UCLP_GLOBAL T* g, int ns, int sc) {
  T s = 0;
  for (int k = a; k < b; ++k) s += val[k] * g[(size_t)col[k] * ns + sc];
  return s;
}

template <typename T>
__device__ inline void stage_entries(const int* __restrict__ col, const T* __restrict__ val, int nz,
                                     int* lc, T* lv) {
  for (int k = threadIdx.x; k < nz; k += kThreads) {
    lc[k] = col[k];
    lv[k] = val[k];
  }
}

// W consecutive scenarios of one element as one access: W = 1, or the
// lanes of a 16-byte vector (4 FP32 / 2 FP64 values) when the batch width
// is a multiple of W, so that a thread moves 16 bytes per load and store.
template <typename T, int W>
__device__ __forceinline__ void ld_lanes(const UCLP_GLOBAL T* p, T (&o)[W]) {
  if constexpr (W == 1) {
    o[0] = p[0];
  } else {
    typedef T vt __attribute__((ext_vector_type(W)));
    const vt a = *reinterpret_cast<const UCLP_GLOBAL vt*>(p);
#pragma unroll
    for (int w = 0; w < W; ++w) o[w] = a[w];
  }
}

// Stores the lanes that are active (all of them with one vector store).
template <typename T, int W>
__device__ __forceinline__ void st_lanes(UCLP_GLOBAL T* p, const T (&v)[W], const bool (&act)[W], bool all) {
  if constexpr (W == 1) {
    if (act[0]) p[0] = v[0];
  } else if (all) {
    typedef T vt __attribute__((ext_vector_type(W)));
    vt a;
#pragma unroll
    for (int w = 0; w < W; ++w) a[w] = v[w];
    *reinterpret_cast<UCLP_GLOBAL vt*>(p) = a;
  } else {
#pragma unroll
    for (int w = 0; w < W; ++w)
      if (act[w]) p[w] = v[w];
  }
}

// row_dot_ms for the W lanes sc .. sc + W - 1: each lane's sum in entry order.
template <typename T, int W>
__device__ inline void row_dot_lanes(int a, int b, const int* lc, const T* lv, const UCLP_GLOBAL T* g, int ns,
                                     int sc, T (&s)[W]) {
#pragma unroll
  for (int w = 0; w < W; ++w) s[w] = 0;
  if (b <= a) return;
  T v[kMsDot], p[kMsDot][W];
#pragma unroll
  for (int t = 0; t < kMsDot; ++t) {
    const int k = min(a + t, b - 1);
    v[t] = lv[k];
    ld_lanes<T, W>(g + (size_t)lc[k] * ns + sc, p[t]);
  }
#pragma unroll
  for (int t = 0; t < kMsDot; ++t)
    if (a + t < b) {
#pragma unroll
      for (int w = 0; w < W; ++w) s[w] += v[t] * p[t][w];
    }
  for (int k = a + kMsDot; k < b; ++k) {
    T q[W];
    ld_lanes<T, W>(g + (size_t)lc[k] * ns + sc, q);
#pragma unroll
    for (int w = 0; w < W; ++w) s[w] += lv[k] * q[w];
  }
}

template <typename T, int W>
__device__ inline void row_dot_lanes_global(int a, int b, const int* __restrict__ col, const T* __restrict__ val,
                                            const UCLP_GLOBAL T* g, int ns, int sc, T (&s)[W]) {
#pragma unroll
  for (int w = 0; w < W; ++w) s[w] = 0;
  for (int k = a; k < b; ++k) {
    T q[W];
    ld_lanes<T, W>(g + (size_t)col[k] * ns + sc, q);
#pragma unroll
    for (int w = 0; w < W; ++w) s[w] += val[k] * q[w];
  }
}

// The lanes a thread serves (sc .. sc + W - 1) and which of them run;
// false when none does.
template <int W>
__device__ __forceinline__ bool lanes_of(const SlotDev& S, int sc, bool (&act)[W], bool& all) {
  bool any = false;
  all = true;
#pragma unroll
  for (int w = 0; w < W; ++w) {
    act[w] = S.active[sc + w] != 0;
    any = any || act[w];
    all = all && act[w];
  }
  return any;
}

// Batched primal half-step: the row block's entries are staged in LDS once;
// kLanes / W threads serve one row, thread sc / W its lanes sc .. sc + W - 1,
// each lane computing what k_primal computes for one instance.
template <typename T, bool CHECK, int W>
__global__ __launch_bounds__(kThreads) void k_primal_ms(const SlotDev* __restrict__ slots,
                                                        const Tile* __restrict__ tiles, int ntiles,
                                                        int jiter) {
  constexpr int G = kLanes / W;                    // threads per row
  constexpr int R = kThreads / G;                  // rows per pass
  constexpr int U = kMsUnroll / W > 0 ? kMsUnroll / W : 1;  // rows per thread in flight
  __shared__ int lc[kNnzTile];
  __shared__ T lv[kNnzTile];
  const int t = xcd_tile(ntiles);
  if (t < 0) return;
  const Tile tl = tiles[t];
  const SlotDev& S = slots[tl.slot];
  const Vecs<T>& V = vecs<T>(S);
  const int r0 = tl.r0, r1 = tl.r1;
  const int* __restrict__ ptr = S.t_ptr;
  const int k0 = tl.k0;
  const int nz = tl.k1 - k0;
  const bool staged = nz <= kNnzTile;
  if (staged) stage_entries<T>(S.t_col + k0, V.tv + k0, nz, lc, lv);
  __syncthreads();
  const int ns = S.nscen;
  const int sc = (threadIdx.x % G) * W;
  if (sc >= ns) return;
  bool act[W], all;
  if (!lanes_of<W>(S, sc, act, all)) return;
  const int fl = tl.flags;
  // full reflection: x is rebuilt from xbar and x0 as in k_primal
  const bool full = S.gamma == 1.0;
  const bool rebuild = full && jiter > 0;
  T tau[W], w[W], wa[W], wp[W], wap[W];
#pragma unroll
  for (int v = 0; v < W; ++v) {
    tau[v] = (T)S.tau[sc + v];
    const double kk = (double)(S.k0[sc + v] + jiter);
    w[v] = (T)((kk + 1.0) / (kk + 2.0));
    wa[v] = (T)(1.0 / (kk + 2.0));
    wp[v] = 0;
    wap[v] = 0;
    if (rebuild) {
      const double kp = (double)(S.k0[sc + v] + jiter - 1);
      wp[v] = (T)((kp + 1.0) / (kp + 2.0));
      wap[v] = (T)(1.0 / (kp + 2.0));
    }
  }
  const UCLP_GLOBAL T* y = gld(V.y);
  // U rows per thread at a time: their vector loads and gathers are all
  // issued before the first epilogue
  for (int jb = r0 + threadIdx.x / G; jb < r1; jb += U * R) {
    T acc[U][W], x[U][W], c[U][W], l[U][W], u[U][W], xa[U][W];
#pragma unroll
    for (int q = 0; q < U; ++q) {
      // straight-line loads: rows past the block's end load its last row
      const int j = min(jb + q * R, r1 - 1);
      const size_t e = (size_t)j * ns + sc;
#pragma unroll
      for (int v = 0; v < W; ++v) {
        c[q][v] = 0;
        u[q][v] = (T)INFINITY;
        l[q][v] = 0;
        xa[q][v] = 0;
      }
      if (!(fl & kColC0)) ld_lanes<T, W>(gld(V.c) + e, c[q]);
      if (!(fl & kColUInf)) ld_lanes<T, W>(gld(V.u) + e, u[q]);
      if (!(fl & (kColL0 | kColLInf | kColLNegU))) ld_lanes<T, W>(gld(V.l) + e, l[q]);
      if (rebuild) {
        ld_lanes<T, W>(gld(V.x0) + e, xa[q]);
        ld_lanes<T, W>(gld(V.xbar) + e, x[q]);
      } else {
        ld_lanes<T, W>(gld(V.x) + e, x[q]);
        if (!CHECK) ld_lanes<T, W>(gld(V.x0) + e, xa[q]);
      }
      if (staged) row_dot_lanes<T, W>(ptr[j] - k0, ptr[j + 1] - k0, lc, lv, y, ns, sc, acc[q]);
      else row_dot_lanes_global<T, W>(ptr[j], ptr[j + 1], S.t_col, V.tv, y, ns, sc, acc[q]);
    }
#pragma unroll
    for (int q = 0; q < U; ++q) {
      const int j = jb + q * R;
      if (j >= r1) break;
      const size_t e = (size_t)j * ns + sc;
      T xq[W], xb[W], xh[W], xn[W];
#pragma unroll
      for (int v = 0; v < W; ++v) {
        xq[v] = rebuild ? wp[v] * x[q][v] + wap[v] * xa[q][v] : x[q][v];
        const T lq = (fl & kColL0)     ? (T)0
                     : (fl & kColLInf)  ? -(T)INFINITY
                     : (fl & kColLNegU) ? -u[q][v]
                                        : l[q][v];
        xh[v] = clampv<T>(xq[v] - tau[v] * (c[q][v] - acc[q][v]), lq, u[q][v]);
        xb[v] = (T)2 * xh[v] - xq[v];
        xn[v] = w[v] * ((T)(1.0 + S.gamma) * xh[v] - (T)S.gamma * xq[v]) + wa[v] * xa[q][v];
      }
      st_lanes<T, W>(gst(V.xbar) + e, xb, act, all);
      if (CHECK) {
        st_lanes<T, W>(gst(V.xhat) + e, xh, act, all);
        if (rebuild) st_lanes<T, W>(gst(V.x) + e, xq, act, all);
      } else if (!full) {
        st_lanes<T, W>(gst(V.x) + e, xn, act, all);
      }
    }
  }
}

// Batched dual half-step, lanes as in k_primal_ms.
template <typename T, bool CHECK, int W>
__global__ __launch_bounds__(kThreads) void k_dual_ms(const SlotDev* __restrict__ slots,
                                                      const Tile* __restrict__ tiles, int ntiles,
                                                      int jiter) {
  constexpr int G = kLanes / W;
  constexpr int R = kThreads / G;
  constexpr int U = kMsUnroll / W > 0 ? kMsUnroll / W : 1;
  __shared__ int lc[kNnzTile];
  __shared__ T lv[kNnzTile];
  const int t = xcd_tile(ntiles);
  if (t < 0) return;
  const Tile tl = tiles[t];
  const SlotDev& S = slots[tl.slot];
  const Vecs<T>& V = vecs<T>(S);
  const int r0 = tl.r0, r1 = tl.r1;
  const int* __restrict__ ptr = S.a_ptr;
  const int k0 = tl.k0;
  const int nz = tl.k1 - k0;
  const bool staged = nz <= kNnzTile;
  if (staged) stage_entries<T>(S.a_col + k0, V.av + k0, nz, lc, lv);
  __syncthreads();
  const int ns = S.nscen;
  const int sc = (threadIdx.x % G) * W;
  if (sc >= ns) return;
  bool act[W], all;
  if (!lanes_of<W>(S, sc, act, all)) return;
  const bool b0 = (tl.flags & kRowB0) != 0;
  T sigma[W], w[W], wa[W];
#pragma unroll
  for (int v = 0; v < W; ++v) {
    sigma[v] = (T)S.sigma[sc + v];
    const double kk = (double)(S.k0[sc + v] + jiter);
    w[v] = (T)((kk + 1.0) / (kk + 2.0));
    wa[v] = (T)(1.0 / (kk + 2.0));
  }
  const T g1 = (T)(1.0 + S.gamma), g = (T)S.gamma;
  const UCLP_GLOBAL T* xbv = gld(V.xbar);
  for (int ib = r0 + threadIdx.x / G; ib < r1; ib += U * R) {
    T acc[U][W], y[U][W], bi[U][W], ya[U][W];
#pragma unroll
    for (int q = 0; q < U; ++q) {
      const int i = min(ib + q * R, r1 - 1);
      const size_t e = (size_t)i * ns + sc;
#pragma unroll
      for (int v = 0; v < W; ++v) {
        bi[q][v] = 0;
        ya[q][v] = 0;
      }
      if (!b0) ld_lanes<T, W>(gld(V.b) + e, bi[q]);
      ld_lanes<T, W>(gld(V.y) + e, y[q]);
      if (!CHECK) ld_lanes<T, W>(gld(V.y0) + e, ya[q]);
      if (staged) row_dot_lanes<T, W>(ptr[i] - k0, ptr[i + 1] - k0, lc, lv, xbv, ns, sc, acc[q]);
      else row_dot_lanes_global<T, W>(ptr[i], ptr[i + 1], S.a_col, V.av, xbv, ns, sc, acc[q]);
    }
#pragma unroll
    for (int q = 0; q < U; ++q) {
      const int i = ib + q * R;
      if (i >= r1) break;
      const size_t e = (size_t)i * ns + sc;
      T yh[W], yn[W];
#pragma unroll
      for (int v = 0; v < W; ++v) {
        yh[v] = y[q][v] + sigma[v] * (bi[q][v] - acc[q][v]);
        if (i >= S.m_eq) yh[v] = yh[v] > (T)0 ? yh[v] : (T)0;
        yn[v] = w[v] * (g1 * yh[v] - g * y[q][v]) + wa[v] * ya[q][v];
      }
      if (CHECK) st_lanes<T, W>(gst(V.yhat) + e, yh, act, all);
      else st_lanes<T, W>(gst(V.y) + e, yn, act, all);
    }
  }
}

// Per-scenario KKT partials of one row block, summed over the block's rows in
// a fixed order; part[((blk * NQ) + q) * kMaxScen + s].
template <int NQ>
__device__ inline void scen_block_partials(double (&q)[NQ], const bool (&is_max)[NQ], double* red,
                                           double* out_blk) {
  const int sc = threadIdx.x % kLanes;
  const int rl = threadIdx.x / kLanes;
#pragma unroll
  for (int k = 0; k < NQ; ++k) red[(rl * kLanes + sc) * NQ + k] = q[k];
  __syncthreads();
  for (int idx = threadIdx.x; idx < kLanes * NQ; idx += kThreads) {
    const int s2 = idx / NQ;
    const int k = idx % NQ;
    double acc = red[s2 * NQ + k];
    for (int r = 1; r < kRowsPerPass; ++r) {
      const double v = red[(r * kLanes + s2) * NQ + k];
      acc = is_max[k] ? fmax(acc, v) : acc + v;
    }
    out_blk[k * kMaxScen + s2] = acc;
  }
}

template <typename T>
__global__ __launch_bounds__(kThreads) void k_kkt_rows_ms(const SlotDev* __restrict__ slots,
                                                          const Tile* __restrict__ tiles, int ntiles) {
  __shared__ int lc[kNnzTile];
  __shared__ double lv[kNnzTile];
  __shared__ double red[kThreads * RQ_N];
  const int t = xcd_tile(ntiles);
  if (t < 0) return;
  const Tile tl = tiles[t];
  const SlotDev& S = slots[tl.slot];
  const Vecs<T>& V = vecs<T>(S);
  const int r0 = tl.r0, r1 = tl.r1;
  const int* __restrict__ ptr = S.a_ptr;
  const int k0 = tl.k0;
  const int nz = tl.k1 - k0;
  const bool staged = nz <= kNnzTile;
  if (staged) stage_entries<double>(S.a_col + k0, S.d.av + k0, nz, lc, lv);
  __syncthreads();
  const int ns = S.nscen;
  const int sc = threadIdx.x % kLanes;
  double q[RQ_N] = {0, 0, 0, 0, 0, 0, 0, 0};
  const bool is_max[RQ_N] = {false, false, false, false, false, false, true, false};
  if (sc < ns) {
    for (int i = r0 + threadIdx.x / kLanes; i < r1; i += kRowsPerPass) {
      double s1 = 0, s2 = 0;
      for (int k = ptr[i]; k < ptr[i + 1]; ++k) {
        const int c = staged ? lc[k - k0] : S.a_col[k];
        const double v = staged ? lv[k - k0] : S.d.av[k];
        const size_t e = (size_t)c * ns + sc;
        const double xh = (double)V.xhat[e];
        s1 += v * xh;
        s2 += v * (xh - (double)V.x[e]);
      }
      const size_t e = (size_t)i * ns + sc;
      double r = S.d.b[e] - s1;
      if (i >= S.m_eq) r = r > 0.0 ? r : 0.0;
      const double ru = r / S.dr[i];
      const double yh = (double)V.yhat[e];
      const double dy = yh - (double)V.y[e];
      const double d0 = yh - (double)V.y0[e];
      const double yneg = i >= S.m_eq && yh < 0.0 ? yh * S.dr[i] : 0.0;
      q[RQ_RES2] += ru * ru;
      q[RQ_BY] += S.d.b[e] * yh;
      q[RQ_DY2] += dy * dy;
      q[RQ_DYADX] += dy * s2;
      q[RQ_DY0] += d0 * d0;
      q[RQ_YNEG2] += yneg * yneg;
      q[RQ_RESMAX] = fmax(q[RQ_RESMAX], fabs(ru));
    }
  }
  scen_block_partials<RQ_N>(q, is_max, red, S.part_a + (size_t)tl.blk * RQ_N * kMaxScen);
}

template <typename T>
__global__ __launch_bounds__(kThreads) void k_kkt_cols_ms(const SlotDev* __restrict__ slots,
                                                          const Tile* __restrict__ tiles, int ntiles) {
  __shared__ int lc[kNnzTile];
  __shared__ double lv[kNnzTile];
  __shared__ double red[kThreads * CQ_N];
  const int t = xcd_tile(ntiles);
  if (t < 0) return;
  const Tile tl = tiles[t];
  const SlotDev& S = slots[tl.slot];
  const Vecs<T>& V = vecs<T>(S);
  const int r0 = tl.r0, r1 = tl.r1;
  const int* __restrict__ ptr = S.t_ptr;
  const int k0 = tl.k0;
  const int nz = tl.k1 - k0;
  const bool staged = nz <= kNnzTile;
  if (staged) stage_entries<double>(S.t_col + k0, S.d.tv + k0, nz, lc, lv);
  __syncthreads();
  const int ns = S.nscen;
  const int sc = threadIdx.x % kLanes;
  double q[CQ_N] = {0, 0, 0, 0, 0};
  const bool is_max[CQ_N] = {false, false, false, false, false};
  if (sc < ns) {
    for (int j = r0 + threadIdx.x / kLanes; j < r1; j += kRowsPerPass) {
      double acc = 0;
      for (int k = ptr[j]; k < ptr[j + 1]; ++k) {
        const int c = staged ? lc[k - k0] : S.t_col[k];
        const double v = staged ? lv[k - k0] : S.d.tv[k];
        acc += v * (double)V.yhat[(size_t)c * ns + sc];
      }
      const size_t e = (size_t)j * ns + sc;
      const double c = S.d.c[e], l = S.d.l[e], u = S.d.u[e];
      const double dh = c - acc;
      const bool fl = isfinite(l), fu = isfinite(u);
      double lam = 0.0;
      if (fl && fu) lam = dh;
      else if (fl) lam = dh > 0.0 ? dh : 0.0;
      else if (fu) lam = dh < 0.0 ? dh : 0.0;
      const double dres = (dh - lam) / S.dc[j];
      const double xhv = (double)V.xhat[e];
      const double dx = xhv - (double)V.x[e];
      const double d0 = xhv - (double)V.x0[e];
      q[CQ_DRES2] += dres * dres;
      q[CQ_LBUB] += (lam > 0.0 ? l * lam : 0.0) + (lam < 0.0 ? u * lam : 0.0);
      q[CQ_CX] += c * xhv;
      q[CQ_DX2] += dx * dx;
      q[CQ_DX0] += d0 * d0;
    }
  }
  scen_block_partials<CQ_N>(q, is_max, red, S.part_t + (size_t)tl.blk * CQ_N * kMaxScen);
}

// scal[s * kScal + q]: thread (q, s) sums its partial over all blocks in order
// Two-level reduction of the scenario partials: kRedChunksMs workgroups each
// reduce a fixed range of row blocks for every (quantity, scenario), then one
// workgroup reduces the chunks in order.  Deterministic.
constexpr int kRedChunksMs = 256;

__global__ __launch_bounds__(kThreads) void k_reduce_ms_part(const SlotDev* __restrict__ slots,
                                                             double* __restrict__ red2) {
  const SlotDev& S = slots[0];
  const int g = blockIdx.x;
  const int idx = threadIdx.x;
  if (idx >= (RQ_N + CQ_N) * kLanes) return;
  const int tq = idx / kLanes;
  const int sc = idx % kLanes;
  if (sc >= S.nscen) return;
  double acc = 0.0;
  if (tq < RQ_N) {
    const bool mx = tq == RQ_RESMAX;
    const int b0 = (int)((int64_t)S.a_nblk * g / kRedChunksMs), b1 = (int)((int64_t)S.a_nblk * (g + 1) / kRedChunksMs);
    for (int b = b0; b < b1; ++b) {
      const double v = S.part_a[((size_t)b * RQ_N + tq) * kMaxScen + sc];
      acc = mx ? fmax(acc, v) : acc + v;
    }
  } else {
    const int k = tq - RQ_N;
    const int b0 = (int)((int64_t)S.t_nblk * g / kRedChunksMs), b1 = (int)((int64_t)S.t_nblk * (g + 1) / kRedChunksMs);
    for (int b = b0; b < b1; ++b) acc += S.part_t[((size_t)b * CQ_N + k) * kMaxScen + sc];
  }
  red2[((size_t)g * (RQ_N + CQ_N) + tq) * kMaxScen + sc] = acc;
}

__global__ __launch_bounds__(kThreads) void k_reduce_ms(const SlotDev* __restrict__ slots,
                                                        const double* __restrict__ red2) {
  const SlotDev& S = slots[0];
  for (int idx = threadIdx.x; idx < (RQ_N + CQ_N) * kLanes; idx += kThreads) {
    const int tq = idx / kLanes;
    const int sc = idx % kLanes;
    if (sc >= S.nscen) continue;
    const bool mx = tq == RQ_RESMAX;
    double acc = 0.0;
    for (int g = 0; g < kRedChunksMs; ++g) {
      const double v = red2[((size_t)g * (RQ_N + CQ_N) + tq) * kMaxScen + sc];
      acc = mx ? fmax(acc, v) : acc + v;
    }
    S.scal[sc * kScal + tq] = acc;
  }
}

template <typename T>
__global__ __launch_bounds__(kThreads) void k_finish_ms(const SlotDev* __restrict__ slots, int64_t n_elems,
                                                        int which, int kk) {
  // which 0: x over n * nscen elements, 1: y over m * nscen
  const SlotDev& S = *slots;
  const Vecs<T>& V = vecs<T>(S);
  const int64_t e = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (e >= n_elems) return;
  const int sc = (int)(e % S.nscen);
  if (!S.active[sc]) return;
  const int flag = S.restart[sc];
  T* z = which ? V.y : V.x;
  T* z0 = which ? V.y0 : V.x0;
  const T zh = which ? V.yhat[e] : V.xhat[e];
  if (flag == 1) {
    z[e] = zh;
    z0[e] = zh;
    return;
  }
  const double k = (double)(S.k0[sc] + kk);
  const T w = (T)((k + 1.0) / (k + 2.0));
  const T wa = (T)(1.0 / (k + 2.0));
  const T refl = which ? (T)(1.0 + S.gamma) * zh - (T)S.gamma * z[e]
                       : (S.gamma == 1.0 ? V.xbar[e] : (T)(1.0 + S.gamma) * zh - (T)S.gamma * z[e]);
  const T zn = w * refl + wa * z0[e];
  z[e] = zn;
  if (flag == 2) z0[e] = zn;
}

__global__ __launch_bounds__(kThreads) void k_promote_ms(const SlotDev* __restrict__ slots, int64_t nx,
                                                         int64_t ny) {
  const SlotDev& S = *slots;
  const int64_t e = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (e < nx) {
    const double v = (double)S.f.xhat[e];
    S.d.x[e] = v;
    S.d.x0[e] = v;
    S.d.xhat[e] = v;
  } else if (e < nx + ny) {
    const int64_t i = e - nx;
    const double v = (double)S.f.yhat[i];
    S.d.y[i] = v;
    S.d.y0[i] = v;
    S.d.yhat[i] = v;
  }
}

// ---------------------------------------------------------------------------
// setup kernels
// ---------------------------------------------------------------------------

__global__ void k_expand_rows(const int* __restrict__ ptr, int m, int* __restrict__ row_of) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= m) return;
  for (int k = ptr[r]; k < ptr[r + 1]; ++k) row_of[k] = r;
}

__global__ void k_iota(int* v, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) v[i] = (int)i;
}

// One workgroup per segment: values and CSR positions in sorted order.
__global__ __launch_bounds__(kThreads) void k_gather_sorted(const int* __restrict__ perm,
                                                            const int* __restrict__ off, int nseg,
                                                            const double* __restrict__ v64,
                                                            const float* __restrict__ v32,
                                                            double* __restrict__ vs64,
                                                            float* __restrict__ vs32,
                                                            unsigned short* __restrict__ dst,
                                                            const int* __restrict__ cs,
                                                            const int* __restrict__ base,
                                                            unsigned* __restrict__ pk) {
  const int b = blockIdx.x;
  if (b >= nseg) return;
  const int s0 = off[b], s1 = off[b + 1];
  const bool fits = s1 - s0 <= kNnzTile;  // long-row blocks keep CSR order and never read dst
  const int bs = base[b];
  for (int k = s0 + threadIdx.x; k < s1; k += kThreads) {
    const int p = perm[k];
    vs64[k] = v64[p];
    vs32[k] = v32[p];
    dst[k] = fits ? (unsigned short)(p - s0) : (unsigned short)0;
    pk[k] = bs >= 0 ? ((unsigned)(p - s0) << kPackShift) | (unsigned)(cs[k] - bs) : 0u;
  }
}

__global__ void k_gather_transpose(const int* __restrict__ perm, const int* __restrict__ row_of,
                                   const double* __restrict__ val, int64_t nnz, int* __restrict__ t_col,
                                   double* __restrict__ t_val) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= nnz) return;
  const int k = perm[p];
  t_col[p] = row_of[k];
  t_val[p] = val[k];
}

// fac[r] = 1/sqrt(max_k |a_rk| drow_r dcol_c) (op 0) or of the sum (op 1); 1 for empty rows.
__global__ __launch_bounds__(kThreads) void k_scale_factor(int op, const int* __restrict__ ptr,
                                                           const int* __restrict__ col,
                                                           const double* __restrict__ val,
                                                           const double* __restrict__ drow,
                                                           const double* __restrict__ dcol,
                                                           const int* __restrict__ blk, int nblk,
                                                           double* __restrict__ fac) {
  __shared__ double red[kThreads / 64];
  const int b = blockIdx.x;
  if (b >= nblk) return;
  const int r0 = blk[b];
  const int r1 = blk[b + 1];
  const int k0 = ptr[r0];
  const int k1 = ptr[r1];
  const int nz = k1 - k0;
  auto term = [&](int k, int r) { return fabs(val[k]) * (drow[r] * dcol[col[k]]); };
  if (nz <= kNnzTile) {
    // each thread walks its own rows (rows are short after blocking)
    for (int r = r0 + threadIdx.x; r < r1; r += kThreads) {
      double acc = 0.0;
      for (int k = ptr[r]; k < ptr[r + 1]; ++k) {
        const double v = term(k, r);
        acc = op == 0 ? fmax(acc, v) : acc + v;
      }
      fac[r] = acc > 0.0 ? 1.0 / sqrt(acc) : 1.0;
    }
    return;
  }
  double acc = 0.0;
  for (int k = k0 + threadIdx.x; k < k1; k += kThreads) {
    const double v = term(k, r0);
    acc = op == 0 ? fmax(acc, v) : acc + v;
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    const double o = __shfl_down(acc, off, 64);
    acc = op == 0 ? fmax(acc, o) : acc + o;
  }
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = red[0];
    for (int w = 1; w < kThreads / 64; ++w) t = op == 0 ? fmax(t, red[w]) : t + red[w];
    fac[r0] = t > 0.0 ? 1.0 / sqrt(t) : 1.0;
  }
}

__global__ void k_mul_inplace(double* d, const double* f, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) d[i] *= f[i];
}

__global__ void k_scale_values(const int* __restrict__ ptr, const int* __restrict__ col,
                               const double* __restrict__ raw, const double* __restrict__ drow,
                               const double* __restrict__ dcol, int rows, double* __restrict__ v64,
                               float* __restrict__ v32) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= rows) return;
  const double dr = drow[r];
  for (int k = ptr[r]; k < ptr[r + 1]; ++k) {
    // raw * (d_row * d_col): the same rounding for A and for its transpose
    const double v = raw[k] * (dr * dcol[col[k]]);
    v64[k] = v;
    v32[k] = (float)v;
  }
}

__global__ void k_fill(double* d, double v, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) d[i] = v;
}

__global__ void k_scale_vectors(const double* __restrict__ c, const double* __restrict__ l,
                                const double* __restrict__ u, const double* __restrict__ b,
                                const double* __restrict__ dc, const double* __restrict__ dr, int n,
                                int m, int nscen, double* c64, double* l64, double* u64, double* b64,
                                float* c32, float* l32, float* u32, float* b32) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t nn = (int64_t)n * nscen;
  const int64_t mm = (int64_t)m * nscen;
  if (i < nn) {
    // scenario-major input (s * n + j) -> interleaved output (j * nscen + s)
    const int s = (int)(i / n);
    const int j = (int)(i % n);
    const int64_t o = (int64_t)j * nscen + s;
    const double d = dc[j];
    const double cv = c[i] * d;
    const double lv = l[i] / d;
    const double uv = u[i] / d;
    c64[o] = cv;
    l64[o] = lv;
    u64[o] = uv;
    c32[o] = (float)cv;
    l32[o] = (float)lv;
    u32[o] = (float)uv;
  } else if (i < nn + mm) {
    const int64_t k = i - nn;
    const int s = (int)(k / m);
    const int r = (int)(k % m);
    const int64_t o = (int64_t)r * nscen + s;
    const double bv = b[k] * dr[r];
    b64[o] = bv;
    b32[o] = (float)bv;
  }
}

template <typename V, typename ACC>
__global__ __launch_bounds__(kThreads) void k_spmv(const int* __restrict__ ptr, const int* __restrict__ col,
                                                   const V* __restrict__ val, const V* __restrict__ x,
                                                   V* __restrict__ y, const int* __restrict__ blk,
                                                   int nblk) {
  __shared__ ACC lds[kNnzTile];
  __shared__ ACC red[kThreads / 64];
  const int t = xcd_tile(nblk);
  if (t < 0) return;
  block_rows<ACC>(ptr, blk[t], blk[t + 1], lds, red, [&](int k) { return (ACC)val[k] * (ACC)x[col[k]]; },
                  [&](int r, ACC s) { y[r] = (V)s; });
}

// ---- merge-path SpMV (Merrill & Garland, SC'16) -----------------------------
// The merge of the row-end list (row_ptr[1..m]) with the entry indices
// 0..nnz-1 has m + nnz items; workgroup g starts near item g S with
// S = kMergeStep.  A small kernel finds every workgroup's start coordinate
// (rows consumed, entries consumed) by a binary search along its diagonal,
// then moves it back to the start of the row it falls in when that row
// began at most kMergeSlack items earlier: a tile then ends at a row
// boundary unless a long row crosses it, and holds at most
// S + kMergeSlack = kMergeTile items.  A row that spans workgroups gets the
// carries of the earlier workgroups added, in workgroup order, by a fix-up
// kernel (not launched when no tile ends inside a row).  Every sum is
// formed in an order fixed by the matrix alone.
__device__ inline void merge_search(int64_t diag, const int* __restrict__ row_end, int m, int64_t nnz,
                                    int& row, int& k) {
  int lo = (int)max(diag - nnz, (int64_t)0);
  int hi = (int)min(diag, (int64_t)m);
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    // consume a row end before entry (diag - mid - 1) when row_end[mid] <= that entry
    if ((int64_t)row_end[mid] <= diag - mid - 1) lo = mid + 1;
    else hi = mid;
  }
  row = lo;
  k = (int)(diag - lo);
}

__global__ void k_merge_coords(const int* __restrict__ ptr, int m, int64_t nnz, int nwg, int2* __restrict__ coord) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g > nwg) return;
  const int64_t d = min((int64_t)g * kMergeStep, (int64_t)m + nnz);
  int row, k;
  merge_search(d, ptr + 1, m, nnz, row, k);
  if (row < m) {
    const int start = ptr[row];
    if (k > start && k - start <= kMergeSlack) k = start;  // end the previous tile at a row boundary
  }
  coord[g] = make_int2(row, k);
}

// One merge-path tile per workgroup: the row ends and entries between two
// consecutive diagonals (at most kMergeTile items).  The products are staged
// in LDS and reduced by a segmented scan whose segments are the rows (a row
// starts where the previous row ends), balanced over the threads whatever
// the row lengths: thread t scans entries [kMergeItems t, kMergeItems (t+1))
// sequentially, the per-thread aggregates are combined by a wave-level then
// a block-level segmented scan, and each thread then finishes its own
// entries.  The rows that end in the tile are written by consecutive
// threads (coalesced stores), each reading the scan at its last entry.  A
// row still open at the end of the tile leaves its partial sum as the tile's
// carry (k_merge_fixup adds the carries, in tile order, to the row's value
// written by the tile where it ends).  LDS index e + e/8 keeps the
// per-thread runs of eight on distinct banks.
__device__ __forceinline__ int merge_lds(int e) { return e + (e >> 3); }

template <typename V>
__global__ __launch_bounds__(kThreads) void k_spmv_merge(const int* __restrict__ ptr, const int* __restrict__ col,
                                                         const V* __restrict__ val, const V* __restrict__ x,
                                                         V* __restrict__ y, const int2* __restrict__ coord,
                                                         int* __restrict__ carry_row, V* __restrict__ carry_val) {
  __shared__ V s_val[kMergeTile + kMergeTile / 8];  // products, then their segmented scan
  __shared__ int s_end[kMergeTile];                 // ends of the tile's rows, relative to k0
  __shared__ unsigned char s_head[kMergeTile];      // 1: a row starts at this entry
  __shared__ V s_wv[kThreads / 64];
  __shared__ int s_wf[kThreads / 64];
  const int g = blockIdx.x;
  const int t = threadIdx.x;
  const int lane = t & 63, wave = t >> 6;
  const int2 c0 = coord[g], c1 = coord[g + 1];
  const int row0 = c0.x, k0 = c0.y;
  const int nrows = c1.x - c0.x;  // row ends this workgroup consumes
  const int nk = c1.y - c0.y;     // entries it consumes
  // coalesced straight-line loads (items past the end re-read the last one)
  int e[kMergeItems];
  V pv[kMergeItems];
  if (nrows > 0) {
#pragma unroll
    for (int u = 0; u < kMergeItems; ++u) e[u] = ptr[row0 + 1 + min(t + u * kThreads, nrows - 1)] - k0;
  }
  if (nk > 0) {
    int cc[kMergeItems];
    V vv[kMergeItems];
#pragma unroll
    for (int u = 0; u < kMergeItems; ++u) {
      const int kk = k0 + min(t + u * kThreads, nk - 1);
      cc[u] = col[kk];
      vv[u] = val[kk];
    }
#pragma unroll
    for (int u = 0; u < kMergeItems; ++u) pv[u] = vv[u] * x[cc[u]];
  }
  const int first = max(ptr[row0] - k0, 0);  // first in-tile entry of row0
#pragma unroll
  for (int u = 0; u < kMergeItems; ++u) {
    const int i = t + u * kThreads;
    s_head[i] = 0;
    if (i < nk) s_val[merge_lds(i)] = pv[u];
  }
  __syncthreads();
  if (nrows > 0) {
#pragma unroll
    for (int u = 0; u < kMergeItems; ++u) {
      const int i = t + u * kThreads;
      if (i < nrows) {
        s_end[i] = e[u];
        if (e[u] < nk) s_head[e[u]] = 1;  // the next row starts here
      }
    }
  }
  __syncthreads();
  // this thread's entries: segmented prefix sums from its first entry
  const int b0 = t * kMergeItems;
  V acc = 0;
  int flag = 0;
#pragma unroll
  for (int u = 0; u < kMergeItems; ++u) {
    if (b0 + u < nk) {
      if (s_head[b0 + u]) {
        acc = 0;
        flag = 1;
      }
      acc += s_val[merge_lds(b0 + u)];
      pv[u] = acc;
    }
  }
  // inclusive segmented scan of (flag, aggregate) over the threads:
  // (f1, v1) then (f2, v2) gives (f1 | f2, f2 ? v2 : v1 + v2)
  V sv = acc;
  int sf = flag;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const V ov = __shfl_up(sv, off, 64);
    const int of = __shfl_up(sf, off, 64);
    if (lane >= off) {
      if (!sf) sv += ov;
      sf |= of;
    }
  }
  if (lane == 63) {
    s_wv[wave] = sv;
    s_wf[wave] = sf;
  }
  // the value of the lane before (inclusive), for this thread's carry-in
  const V pvv = __shfl_up(sv, 1, 64);
  const int pff = __shfl_up(sf, 1, 64);
  __syncthreads();
  // the segment arriving from earlier waves
  V wv = 0;
  for (int w = 0; w < wave; ++w) wv = s_wf[w] ? s_wv[w] : wv + s_wv[w];
  const V cin = lane == 0 ? wv : (pff ? pvv : wv + pvv);
  // finish this thread's entries: those before its first row start take the
  // carry-in
  int seen = 0;
#pragma unroll
  for (int u = 0; u < kMergeItems; ++u) {
    if (b0 + u < nk) {
      seen |= s_head[b0 + u];
      s_val[merge_lds(b0 + u)] = seen ? pv[u] : cin + pv[u];
    }
  }
  __syncthreads();
  // rows ending in this tile: the scan at their last entry (0 if none here)
  for (int i = t; i < nrows; i += kThreads) {
    const int end = s_end[i];
    const int beg = i == 0 ? first : s_end[i - 1];
    y[row0 + i] = end > beg ? s_val[merge_lds(end - 1)] : (V)0;
  }
  if (t == 0) {
    const int last = nrows > 0 ? s_end[nrows - 1] : first;
    carry_row[g] = row0 + nrows;
    carry_val[g] = nk > last ? s_val[merge_lds(nk - 1)] : (V)0;
  }
}

// Rows open at the end of a workgroup collect that workgroup's carry, and
// possibly those of the next ones, and are completed (written to y) by a
// later workgroup.  Carry g adds its whole run of equal rows, in workgroup
// order, if it is the first of that run.
template <typename V>
__global__ void k_merge_fixup(const int* __restrict__ carry_row, const V* __restrict__ carry_val, int nwg, int m,
                              V* __restrict__ y) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= nwg) return;
  const int r = carry_row[g];
  if (r >= m) return;
  if (g > 0 && carry_row[g - 1] == r) return;
  // the run's carries in order, eight independent loads at a time (a long
  // row spans many tiles)
  V s = 0;
  for (int u = g; u < nwg; u += 8) {
    int rr[8];
    V vv[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const int i = min(u + k, nwg - 1);
      rr[k] = carry_row[i];
      vv[k] = carry_val[i];
    }
    bool more = true;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      more = more && u + k < nwg && rr[k] == r;
      if (more) s += vv[k];
    }
    if (!more) break;
  }
  y[r] = s + y[r];
}

// ---- reductions / vectors --------------------------------------------------

__global__ __launch_bounds__(kThreads) void k_sumsq_part(const double* __restrict__ v, int64_t n,
                                                         double* __restrict__ part) {
  __shared__ double red[kThreads / 64];
  double acc = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kThreads)
    acc += v[i] * v[i];
  double q[1] = {acc};
  const bool mx[1] = {false};
  block_reduce<1>(q, mx, red);
  if (threadIdx.x == 0) part[blockIdx.x] = q[0];
}

__global__ __launch_bounds__(kThreads) void k_sum_part(const double* __restrict__ part, int np,
                                                       double* __restrict__ out) {
  __shared__ double red[kThreads / 64];
  double acc = 0.0;
  for (int i = threadIdx.x; i < np; i += kThreads) acc += part[i];
  double q[1] = {acc};
  const bool mx[1] = {false};
  block_reduce<1>(q, mx, red);
  if (threadIdx.x == 0) *out = q[0];
}

__global__ void k_normalize(const double* __restrict__ w, const double* __restrict__ nrm2,
                            double* __restrict__ v, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double s = *nrm2;
  v[i] = s > 0.0 ? w[i] / sqrt(s) : 0.0;
}

// deterministic pseudo-random start vector in [-1, 1): a 32-bit integer hash
// (Wang's mix) of (index, seed)
__global__ void k_hash_vector(double* v, int64_t n, uint32_t seed) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  uint32_t h = (uint32_t)i * 2654435761u ^ seed;
  h = (h ^ 61u) ^ (h >> 16);
  h *= 9u;
  h ^= h >> 4;
  h *= 0x27d4eb2du;
  h ^= h >> 15;
  v[i] = (double)h / 2147483648.0 - 1.0;
}

template <typename T>
__global__ void k_init_iterates(const SlotDev* __restrict__ slot, const double* __restrict__ x_in,
                                const double* __restrict__ y_in, int n, int m, int m_eq, int nscen) {
  const SlotDev& S = *slot;
  const Vecs<T>& V = vecs<T>(S);
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t nn = (int64_t)n * nscen;
  const int64_t mm = (int64_t)m * nscen;
  if (i < nn) {
    const int j = (int)(i / nscen);
    double v = x_in ? x_in[i] / S.dc[j] : 0.0;
    T tv = clampv<T>((T)v, V.l[i], V.u[i]);
    V.x[i] = tv;
    V.x0[i] = tv;
    V.xhat[i] = tv;
    V.xbar[i] = tv;
  } else if (i < nn + mm) {
    const int64_t k = i - nn;
    const int r = (int)(k / nscen);
    double v = y_in ? y_in[k] / S.dr[r] : 0.0;
    if (r >= m_eq && v < 0.0) v = 0.0;
    V.y[k] = (T)v;
    V.y0[k] = (T)v;
    V.yhat[k] = (T)v;
  }
}

template <typename T>
__global__ void k_unscale(const SlotDev* __restrict__ slot, double* __restrict__ x_out,
                          double* __restrict__ y_out, int n, int m, int nscen) {
  const SlotDev& S = *slot;
  const Vecs<T>& V = vecs<T>(S);
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t nn = (int64_t)n * nscen;
  const int64_t mm = (int64_t)m * nscen;
  if (i < nn) {
    x_out[i] = (double)V.xhat[i] * S.dc[i / nscen];
  } else if (i < nn + mm) {
    const int64_t k = i - nn;
    y_out[k] = (double)V.yhat[k] * S.dr[k / nscen];
  }
}

__global__ void k_to_f32(const double* a, float* b, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) b[i] = (float)a[i];
}

// Plain stream copy, 4 x 16 B per thread and iteration, grid-stride.
typedef float v4f __attribute__((ext_vector_type(4)));
constexpr int kCopyThreads = 256;

__global__ __launch_bounds__(kCopyThreads) void k_copy(const v4f* __restrict__ a, v4f* __restrict__ b,
                                                   int64_t n4) {
  const int64_t stride = (int64_t)gridDim.x * kCopyThreads * 4;
  for (int64_t i = (int64_t)blockIdx.x * kCopyThreads * 4 + threadIdx.x; i < n4; i += stride) {
    v4f v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u)
      if (i + u * kCopyThreads < n4) v[u] = __builtin_nontemporal_load(a + i + u * kCopyThreads);
#pragma unroll
    for (int u = 0; u < 4; ++u)
      if (i + u * kCopyThreads < n4) __builtin_nontemporal_store(v[u], b + i + u * kCopyThreads);
  }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------

static inline int nb(int64_t n, int t = kThreads) { return (int)((n + t - 1) / t); }

template <int NT, typename K>
static void launch_tiles(K kern, int ntiles, hipStream_t s, hipEvent_t e0, hipEvent_t e1,
                         const SlotDev* slots, const Tile* tiles, int jiter) {
  const dim3 g(xcd_grid(ntiles));
  if (e0 && e1) hipExtLaunchKernelGGL(kern, g, dim3(NT), 0, s, e0, e1, 0, slots, tiles, ntiles, jiter);
  else kern<<<g, NT, 0, s>>>(slots, tiles, ntiles, jiter);
}

// Workgroup size of the half-steps.  A launch of many tiles runs kThreads
// threads with several rows and kNnzTile / kThreads staged entries each:
// more loads in flight per thread, which is what a bandwidth-bound launch
// needs.  A launch that fits the chip in one pass even with one row per
// thread (kRowsPerBlock threads; four such workgroups per CU, 256 CUs) runs
// that shape instead, which shortens each thread's serial chain.
constexpr int kWideThreads = kRowsPerBlock;

template <typename T, bool CHECK>
static void launch_primal_t(int ntiles, hipStream_t s, hipEvent_t e0, hipEvent_t e1, const SlotDev* slots,
                            const Tile* tiles, int jiter, int threads) {
  if (threads == kWideThreads || (threads == 0 && ntiles < kFewTiles))
    launch_tiles<kWideThreads>(k_primal<T, CHECK, kWideThreads>, ntiles, s, e0, e1, slots, tiles, jiter);
  else
    launch_tiles<kThreads>(k_primal<T, CHECK, kThreads>, ntiles, s, e0, e1, slots, tiles, jiter);
}

template <typename T, bool CHECK>
static void launch_dual_t(int ntiles, hipStream_t s, hipEvent_t e0, hipEvent_t e1, const SlotDev* slots,
                          const Tile* tiles, int jiter, int threads) {
  if (threads == kWideThreads || (threads == 0 && ntiles < kFewTiles))
    launch_tiles<kWideThreads>(k_dual<T, CHECK, kWideThreads>, ntiles, s, e0, e1, slots, tiles, jiter);
  else
    launch_tiles<kThreads>(k_dual<T, CHECK, kThreads>, ntiles, s, e0, e1, slots, tiles, jiter);
}

void launch_primal(int prec, bool check, const SlotDev* slots, const Tile* tiles, int ntiles,
                   int jiter, int nscen, hipStream_t s, hipEvent_t e0, hipEvent_t e1, int threads) {
  if (ntiles <= 0) return;
  (void)nscen;
  if (prec == 1) {
    if (check) launch_primal_t<float, true>(ntiles, s, e0, e1, slots, tiles, jiter, threads);
    else launch_primal_t<float, false>(ntiles, s, e0, e1, slots, tiles, jiter, threads);
  } else {
    if (check) launch_primal_t<double, true>(ntiles, s, e0, e1, slots, tiles, jiter, threads);
    else launch_primal_t<double, false>(ntiles, s, e0, e1, slots, tiles, jiter, threads);
  }
}

void launch_dual(int prec, bool check, const SlotDev* slots, const Tile* tiles, int ntiles,
                 int jiter, int nscen, hipStream_t s, hipEvent_t e0, hipEvent_t e1, int threads) {
  if (ntiles <= 0) return;
  (void)nscen;
  if (prec == 1) {
    if (check) launch_dual_t<float, true>(ntiles, s, e0, e1, slots, tiles, jiter, threads);
    else launch_dual_t<float, false>(ntiles, s, e0, e1, slots, tiles, jiter, threads);
  } else {
    if (check) launch_dual_t<double, true>(ntiles, s, e0, e1, slots, tiles, jiter, threads);
    else launch_dual_t<double, false>(ntiles, s, e0, e1, slots, tiles, jiter, threads);
  }
}

void launch_kkt(int prec, const SlotDev* slots, const Tile* ttiles, int nttiles, const Tile* atiles,
                int natiles, int nscen, hipStream_t s) {
  (void)nscen;
  if (prec == 1) {
    if (natiles > 0) k_kkt_rows<float><<<xcd_grid(natiles), kThreads, 0, s>>>(slots, atiles, natiles);
    if (nttiles > 0) k_kkt_cols<float><<<xcd_grid(nttiles), kThreads, 0, s>>>(slots, ttiles, nttiles);
  } else {
    if (natiles > 0) k_kkt_rows<double><<<xcd_grid(natiles), kThreads, 0, s>>>(slots, atiles, natiles);
    if (nttiles > 0) k_kkt_cols<double><<<xcd_grid(nttiles), kThreads, 0, s>>>(slots, ttiles, nttiles);
  }
}

void launch_reduce(const SlotDev* slots, const int* slot_ids, int nslots, int nscen, double* red2,
                   hipStream_t s) {
  (void)nscen;
  if (nslots <= 0) return;
  k_reduce_part<<<dim3(kRedChunks, nslots), kThreads, 0, s>>>(slots, slot_ids, red2);
  k_reduce<<<nslots, kThreads, 0, s>>>(slots, slot_ids, red2);
}

void launch_finish(int prec, const SlotDev* slots, const Tile* ttiles, int nttiles, const Tile* atiles,
                   int natiles, int kk, int nscen, hipStream_t s) {
  (void)nscen;
  if (prec == 1) {
    if (nttiles > 0) k_finish_x<float><<<xcd_grid(nttiles), kThreads, 0, s>>>(slots, ttiles, nttiles, kk);
    if (natiles > 0) k_finish_y<float><<<xcd_grid(natiles), kThreads, 0, s>>>(slots, atiles, natiles, kk);
  } else {
    if (nttiles > 0) k_finish_x<double><<<xcd_grid(nttiles), kThreads, 0, s>>>(slots, ttiles, nttiles, kk);
    if (natiles > 0) k_finish_y<double><<<xcd_grid(natiles), kThreads, 0, s>>>(slots, atiles, natiles, kk);
  }
}

void launch_engine_check(SlotDev* slots, ChkState* chk, const ChkParams* prm, int nslots, hipStream_t s) {
  if (nslots > 0) k_engine_check<<<nb(nslots, 64), 64, 0, s>>>(slots, chk, prm, nslots);
}

void launch_stamp(unsigned long long* t, hipStream_t s) { k_stamp<<<1, 64, 0, s>>>(t); }

void launch_refine_measure(const RefineArgs& R, hipStream_t s) {
  const int64_t nm = (int64_t)R.n + R.m;
  k_refine_fold<<<nb(nm), kThreads, 0, s>>>(R);
  if (R.a_nblk > 0) k_refine_rows<<<R.a_nblk, kThreads, 0, s>>>(R);
  if (R.t_nblk > 0) k_refine_cols<<<R.t_nblk, kThreads, 0, s>>>(R);
  k_refine_reduce<<<1, kThreads, 0, s>>>(R);
}

void launch_refine_form(const RefineArgs& R, hipStream_t s) {
  const int64_t nm = (int64_t)R.n + R.m;
  k_refine_form<<<nb(nm), kThreads, 0, s>>>(R);
}

void launch_promote(const SlotDev* slots, const Tile* ttiles, int nttiles, const Tile* atiles,
                    int natiles, int nscen, hipStream_t s) {
  (void)nscen;
  if (nttiles > 0) k_promote_x<<<xcd_grid(nttiles), kThreads, 0, s>>>(slots, ttiles, nttiles);
  if (natiles > 0) k_promote_y<<<xcd_grid(natiles), kThreads, 0, s>>>(slots, atiles, natiles);
}

void launch_expand_rows(const int* ptr, int m, int* row_of, hipStream_t s) {
  if (m > 0) k_expand_rows<<<nb(m), kThreads, 0, s>>>(ptr, m, row_of);
}

void launch_iota(int* v, int64_t n, hipStream_t s) {
  if (n > 0) k_iota<<<nb(n), kThreads, 0, s>>>(v, n);
}

void launch_gather_transpose(const int* perm, const int* row_of, const double* val, int64_t nnz,
                             int* t_col, double* t_val, hipStream_t s) {
  if (nnz > 0) k_gather_transpose<<<nb(nnz), kThreads, 0, s>>>(perm, row_of, val, nnz, t_col, t_val);
}

static int key_bits(int n) {
  int b = 1;
  while (b < 31 && (1 << b) < n) ++b;
  return b;
}

size_t radix_sort_temp_bytes(int64_t nnz, int n) {
  size_t bytes = 0;
  (void)hipcub::DeviceRadixSort::SortPairs(nullptr, bytes, (const int*)nullptr, (int*)nullptr,
                                     (const int*)nullptr, (int*)nullptr, (int)nnz, 0, key_bits(n));
  // the size query may leave a non-sticky error behind; do not let a later
  // hipGetLastError() (the sort itself ends with one) report it
  (void)hipGetLastError();
  return bytes;
}

int radix_sort_pairs(void* temp, size_t temp_bytes, const int* keys_in, int* keys_out,
                     const int* vals_in, int* vals_out, int64_t nnz, int n, hipStream_t s) {
  if (nnz == 0) return 0;
  hipError_t e = hipcub::DeviceRadixSort::SortPairs(temp, temp_bytes, keys_in, keys_out, vals_in,
                                                    vals_out, (int)nnz, 0, key_bits(n), s);
  return (int)e;
}

size_t seg_sort_temp_bytes(int64_t nnz, int nseg, int ncols) {
  size_t bytes = 0;
  (void)hipcub::DeviceSegmentedRadixSort::SortPairs(nullptr, bytes, (const int*)nullptr, (int*)nullptr,
                                                    (const int*)nullptr, (int*)nullptr, (int)nnz, nseg,
                                                    (const int*)nullptr, (const int*)nullptr, 0,
                                                    key_bits(ncols));
  (void)hipGetLastError();
  return bytes;
}

int seg_sort_pairs(void* temp, size_t temp_bytes, const int* keys_in, int* keys_out, const int* vals_in,
                   int* vals_out, int64_t nnz, int nseg, const int* off, int ncols, hipStream_t s) {
  if (nnz == 0 || nseg == 0) return 0;
  hipError_t e = hipcub::DeviceSegmentedRadixSort::SortPairs(temp, temp_bytes, keys_in, keys_out, vals_in,
                                                             vals_out, (int)nnz, nseg, off, off + 1, 0,
                                                             key_bits(ncols), s);
  return (int)e;
}

void launch_gather_sorted(const int* perm, const int* off, int nseg, const double* v64, const float* v32,
                          double* vs64, float* vs32, unsigned short* dst, const int* cs,
                          const int* base, unsigned* pk, hipStream_t s) {
  if (nseg > 0)
    k_gather_sorted<<<nseg, kThreads, 0, s>>>(perm, off, nseg, v64, v32, vs64, vs32, dst, cs, base, pk);
}

void launch_scale_factor(int op, const int* ptr, const int* col, const double* val, const double* drow,
                         const double* dcol, const int* blk, int nblk, int rows, double* fac,
                         hipStream_t s) {
  (void)rows;
  if (nblk > 0) k_scale_factor<<<nblk, kThreads, 0, s>>>(op, ptr, col, val, drow, dcol, blk, nblk, fac);
}

void launch_mul_inplace(double* d, const double* f, int n, hipStream_t s) {
  if (n > 0) k_mul_inplace<<<nb(n), kThreads, 0, s>>>(d, f, n);
}

void launch_scale_values(const int* ptr, const int* col, const double* raw, const double* drow,
                         const double* dcol, int rows, double* v64, float* v32, hipStream_t s) {
  if (rows > 0) k_scale_values<<<nb(rows), kThreads, 0, s>>>(ptr, col, raw, drow, dcol, rows, v64, v32);
}

void launch_fill(double* d, double v, int64_t n, hipStream_t s) {
  if (n > 0) k_fill<<<nb(n), kThreads, 0, s>>>(d, v, n);
}

void launch_scale_vectors(const double* c, const double* l, const double* u, const double* b,
                          const double* dc, const double* dr, int n, int m, int nscen, double* c64,
                          double* l64, double* u64, double* b64, float* c32, float* l32, float* u32,
                          float* b32, hipStream_t s) {
  const int64_t tot = (int64_t)(n + m) * nscen;
  if (tot > 0)
    k_scale_vectors<<<nb(tot), kThreads, 0, s>>>(c, l, u, b, dc, dr, n, m, nscen, c64, l64, u64, b64,
                                                 c32, l32, u32, b32);
}

void launch_spmv64(const int* ptr, const int* col, const double* val, const double* x, double* y,
                   const int* blk, int nblk, hipStream_t s) {
  if (nblk > 0) k_spmv<double, double><<<xcd_grid(nblk), kThreads, 0, s>>>(ptr, col, val, x, y, blk, nblk);
}

void launch_spmv32(const int* ptr, const int* col, const float* val, const float* x, float* y,
                   const int* blk, int nblk, hipStream_t s) {
  if (nblk > 0) k_spmv<float, float><<<xcd_grid(nblk), kThreads, 0, s>>>(ptr, col, val, x, y, blk, nblk);
}

int merge_workgroups(int m, int64_t nnz) {
  return (int)(((int64_t)m + nnz + kMergeStep - 1) / kMergeStep);
}

template <typename V>
static void launch_spmv_merge_t(const int* ptr, const int* col, const V* val, const V* x, V* y, int m, int64_t nnz,
                                int2* coord, int* carry_row, V* carry_val, hipStream_t s, bool planned,
                                bool fixup) {
  const int nwg = merge_workgroups(m, nnz);
  if (nwg <= 0) return;
  if (!planned) k_merge_coords<<<nb(nwg + 1), kThreads, 0, s>>>(ptr, m, nnz, nwg, coord);
  k_spmv_merge<V><<<nwg, kThreads, 0, s>>>(ptr, col, val, x, y, coord, carry_row, carry_val);
  if (fixup || !planned) k_merge_fixup<V><<<nb(nwg), kThreads, 0, s>>>(carry_row, carry_val, nwg, m, y);
}

void launch_spmv_merge64(const int* ptr, const int* col, const double* val, const double* x, double* y, int m,
                         int64_t nnz, int2* coord, int* carry_row, double* carry_val, hipStream_t s, bool planned,
                         bool fixup) {
  launch_spmv_merge_t<double>(ptr, col, val, x, y, m, nnz, coord, carry_row, carry_val, s, planned, fixup);
}

void launch_spmv_merge32(const int* ptr, const int* col, const float* val, const float* x, float* y, int m,
                         int64_t nnz, int2* coord, int* carry_row, float* carry_val, hipStream_t s, bool planned,
                         bool fixup) {
  launch_spmv_merge_t<float>(ptr, col, val, x, y, m, nnz, coord, carry_row, carry_val, s, planned, fixup);
}

void launch_merge_coords(const int* ptr, int m, int64_t nnz, int2* coord, hipStream_t s) {
  const int nwg = merge_workgroups(m, nnz);
  if (nwg > 0) k_merge_coords<<<nb(nwg + 1), kThreads, 0, s>>>(ptr, m, nnz, nwg, coord);
}

void launch_norm2(const double* v, int64_t n, double* part, double* out, hipStream_t s) {
  int g = nb(n);
  if (g > 1024) g = 1024;
  if (g < 1) g = 1;
  k_sumsq_part<<<g, kThreads, 0, s>>>(v, n, part);
  k_sum_part<<<1, kThreads, 0, s>>>(part, g, out);
}

void launch_normalize(const double* w, const double* nrm2, double* v, int64_t n, hipStream_t s) {
  if (n > 0) k_normalize<<<nb(n), kThreads, 0, s>>>(w, nrm2, v, n);
}

void launch_hash_vector(double* v, int64_t n, uint32_t seed, hipStream_t s) {
  if (n > 0) k_hash_vector<<<nb(n), kThreads, 0, s>>>(v, n, seed);
}

void launch_init_iterates(const SlotDev* slot, int prec, const double* x_in, const double* y_in, int n,
                          int m, int m_eq, int nscen, hipStream_t s) {
  const int64_t tot = (int64_t)(n + m) * nscen;
  if (tot <= 0) return;
  if (prec == 1) k_init_iterates<float><<<nb(tot), kThreads, 0, s>>>(slot, x_in, y_in, n, m, m_eq, nscen);
  else k_init_iterates<double><<<nb(tot), kThreads, 0, s>>>(slot, x_in, y_in, n, m, m_eq, nscen);
}

void launch_unscale(const SlotDev* slot, int prec, double* x_out, double* y_out, int n, int m, int nscen,
                    hipStream_t s) {
  const int64_t tot = (int64_t)(n + m) * nscen;
  if (tot <= 0) return;
  if (prec == 1) k_unscale<float><<<nb(tot), kThreads, 0, s>>>(slot, x_out, y_out, n, m, nscen);
  else k_unscale<double><<<nb(tot), kThreads, 0, s>>>(slot, x_out, y_out, n, m, nscen);
}

void launch_to_f32(const double* a, float* b, int64_t n, hipStream_t s) {
  if (n > 0) k_to_f32<<<nb(n), kThreads, 0, s>>>(a, b, n);
}

void launch_copy_kernel(const float4* a, float4* b, int64_t n4, hipStream_t s) {
  int g = nb(n4, kCopyThreads * 4);
  if (g > 256 * 64) g = 256 * 64;
  if (g > 0) k_copy<<<g, kCopyThreads, 0, s>>>((const v4f*)a, (v4f*)b, n4);
}

// ---- scenario-batch launchers -------------------------------------------------

void launch_primal_ms(int prec, bool check, bool vec, const SlotDev* slots, const Tile* tiles, int ntiles,
                      int jiter, hipStream_t s) {
  if (ntiles <= 0) return;
  const dim3 g(xcd_grid(ntiles));
  if (prec == 1) {
    if (vec) {
      if (check) k_primal_ms<float, true, 4><<<g, kThreads, 0, s>>>(slots, tiles, ntiles, jiter);
      else k_primal_ms<float, false, 4><<<g, kThreads, 0, s>>>(slots, tiles, ntiles, jiter);
    } else {
      if (check) k_primal_ms<float, true, 1><<<g, kThreads, 0, s>>>(slots, tiles, ntiles, jiter);
      else k_primal_ms<float, false, 1><<<g, kThreads, 0, s>>>(slots, tiles, ntiles, jiter);
    }
  } else {
    if (vec) {
      if (check) k_primal_ms<double, true, 2><<<g, kThreads, 0, s>>>(slots, tiles, ntiles, jiter);
      else k_primal_ms<double, false, 2><<<g, kThreads, 0, s>>>(slots, tiles, ntiles, jiter);
    } else {
      if (check) k_primal_ms<double, true, 1><<<g, kThreads, 0, s>>>(slots, tiles, ntiles, jiter);
      else k_primal_ms<double, false, 1><<<g, kThreads, 0, s>>>(slots, tiles, ntiles, jiter);
    }
  }
}

void launch_dual_ms(int prec, bool check, bool vec, const SlotDev* slots, const Tile* tiles, int ntiles,
                    int jiter, hipStream_t s) {
  if (ntiles <= 0) return;
  const dim3 g(xcd_grid(ntiles));
  if (prec == 1) {
    if (vec) {
      if (check) k_dual_ms<float, true, 4><<<g, kThreads, 0, s>>>(slots, tiles, ntiles, jiter);
      else k_dual_ms<float, false, 4><<<g, kThreads, 0, s>>>(slots, tiles, ntiles, jiter);
    } else {
      if (check) k_dual_ms<float, true, 1><<<g, kThreads, 0, s>>>(slots, tiles, ntiles, jiter);
      else k_dual_ms<float, false, 1><<<g, kThreads, 0, s>>>(slots, tiles, ntiles, jiter);
    }
  } else {
    if (vec) {
      if (check) k_dual_ms<double, true, 2><<<g, kThreads, 0, s>>>(slots, tiles, ntiles, jiter);
      else k_dual_ms<double, false, 2><<<g, kThreads, 0, s>>>(slots, tiles, ntiles, jiter);
    } else {
      if (check) k_dual_ms<double, true, 1><<<g, kThreads, 0, s>>>(slots, tiles, ntiles, jiter);
      else k_dual_ms<double, false, 1><<<g, kThreads, 0, s>>>(slots, tiles, ntiles, jiter);
    }
  }
}

void launch_kkt_ms(int prec, const SlotDev* slots, const Tile* ttiles, int nttiles, const Tile* atiles,
                   int natiles, double* red2, hipStream_t s) {
  if (prec == 1) {
    if (natiles > 0) k_kkt_rows_ms<float><<<xcd_grid(natiles), kThreads, 0, s>>>(slots, atiles, natiles);
    if (nttiles > 0) k_kkt_cols_ms<float><<<xcd_grid(nttiles), kThreads, 0, s>>>(slots, ttiles, nttiles);
  } else {
    if (natiles > 0) k_kkt_rows_ms<double><<<xcd_grid(natiles), kThreads, 0, s>>>(slots, atiles, natiles);
    if (nttiles > 0) k_kkt_cols_ms<double><<<xcd_grid(nttiles), kThreads, 0, s>>>(slots, ttiles, nttiles);
  }
  k_reduce_ms_part<<<kRedChunksMs, kThreads, 0, s>>>(slots, red2);
  k_reduce_ms<<<1, kThreads, 0, s>>>(slots, red2);
}

size_t red2_ms_doubles() { return (size_t)kRedChunksMs * (RQ_N + CQ_N) * kMaxScen; }

void launch_finish_ms(int prec, const SlotDev* slots, int64_t nx, int64_t ny, int kk, hipStream_t s) {
  if (prec == 1) {
    if (nx > 0) k_finish_ms<float><<<nb(nx), kThreads, 0, s>>>(slots, nx, 0, kk);
    if (ny > 0) k_finish_ms<float><<<nb(ny), kThreads, 0, s>>>(slots, ny, 1, kk);
  } else {
    if (nx > 0) k_finish_ms<double><<<nb(nx), kThreads, 0, s>>>(slots, nx, 0, kk);
    if (ny > 0) k_finish_ms<double><<<nb(ny), kThreads, 0, s>>>(slots, ny, 1, kk);
  }
}

void launch_promote_ms(const SlotDev* slots, int64_t nx, int64_t ny, hipStream_t s) {
  if (nx + ny > 0) k_promote_ms<<<nb(nx + ny), kThreads, 0, s>>>(slots, nx, ny);
}

}  // namespace uclp
