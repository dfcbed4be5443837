// Structures shared by the device kernels (kernels.hip) and the host runtime
// (uclp.cpp) of libuclp.  Internal; not part of the C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace uclp {

// Row blocks: at most kRowsPerBlock rows and kNnzTile entries, except a
// block holding one row longer than kNnzTile (handled by a block-wide loop).
// Thread t of a workgroup owns rows r0 + t + q * kThreads, q < kRowsPerThread
// (the half-step kernels of launches with few tiles run kRowsPerBlock
// threads, one row each).
constexpr int kThreads = 256;
constexpr int kRowsPerThread = 2;
constexpr int kRowsPerBlock = kThreads * kRowsPerThread;
constexpr int kNnzTile = 2048;
constexpr int kMaxScen = 16;

// Per-block partial sums written by the KKT check kernels.
// RQ_YLOR: sum over inequality rows of ylo_i ((A x)_i - b_i), the term that
// a lower bound ylo != 0 on the inequality duals adds to the primal objective
// (zero outside the correction problems of iterative refinement).
enum RowQ { RQ_RES2 = 0, RQ_BY, RQ_DY2, RQ_DYADX, RQ_DY0, RQ_YNEG2, RQ_RESMAX, RQ_YLOR, RQ_N };
enum ColQ { CQ_DRES2 = 0, CQ_LBUB, CQ_CX, CQ_DX2, CQ_DX0, CQ_N };
// Per-slot scalars after the final reduction: row quantities then column ones.
constexpr int kScal = 16;

template <typename T>
struct Vecs {
  T* x;      // current iterate (n)
  T* x0;     // Halpern anchor (n)
  T* xbar;   // 2 x_hat - x, gathered by the dual half-step (n)
  T* xhat;   // x_hat, written on check iterations (n)
  T* y;      // (m)
  T* y0;
  T* yhat;
  const T* c;   // scaled problem data
  const T* l;
  const T* u;
  const T* b;
  const T* tv;  // scaled values of A^T (CSR order)
  const T* av;  // scaled values of A (CSR order)
  const T* tvs;  // scaled values of A^T, each row block sorted by column index
  const T* avs;  // scaled values of A, each row block sorted by column index
};

// Everything a kernel needs to know about one resident instance (a "slot").
// nscen > 1: vectors hold nscen interleaved scenarios (element i of scenario
// s at i * nscen + s) and c, l, u, b are per scenario; tau/sigma per scenario.
struct SlotDev {
  const int* a_ptr;
  const int* a_col;
  const int* t_ptr;
  const int* t_col;
  const int* a_blk;  // row-block boundaries of A   (a_nblk + 1)
  const int* t_blk;  // row-block boundaries of A^T (t_nblk + 1)
  // Entries of each row block re-ordered by column index (so the gathers of
  // neighbouring lanes hit neighbouring cache lines) and, per entry, its
  // position inside the block in CSR order (where its product goes in LDS).
  const int* a_cs;
  const int* t_cs;
  const unsigned short* a_dst;
  const unsigned short* t_dst;
  const unsigned* a_pk;  // packed entries (Tile::base >= 0)
  const unsigned* t_pk;
  // end of each row's entries relative to its row block's first entry
  // (0 in long-row blocks); a row starts where the previous row of the
  // block ends
  const unsigned short* a_end;
  const unsigned short* t_end;
  int m, n, m_eq, nscen;
  int a_nblk, t_nblk;
  const double* dr;  // D_r (m)
  const double* dc;  // D_c (n)
  Vecs<float> f;
  Vecs<double> d;
  // lower bound of the inequality duals (m, FP32), read by the dual
  // half-step and the KKT kernels only in tiles flagged kRowYlo (the
  // correction problems of iterative refinement); elsewhere the bound is 0
  const float* ylo;
  double* part_a;    // [a_nblk * RQ_N] (scenario batches: [a_nblk * RQ_N * kMaxScen])
  double* part_t;    // [t_nblk * CQ_N] (scenario batches: [t_nblk * CQ_N * kMaxScen])
  double* scal;      // [kScal] (scenario batches: [nscen * kScal])
  long long k0[kMaxScen];       // inner iteration index at the epoch start
  double tau[kMaxScen];
  double sigma[kMaxScen];
  int restart[kMaxScen];        // set by the host before the finish kernel
  int active[kMaxScen];         // 0: scenario frozen (converged)
  double gamma;                 // Halpern reflection: w((1+g) T(z) - g z) + (1-w) z0
  long long kfin;               // single-scenario slots: iteration index of the
                                // check step the finish kernel completes
};

// One unit of work of the batched kernels: a row block of one slot, with its
// row range [r0, r1) and entry range [k0, k1) precomputed on the host so a
// workgroup needs a single 32-byte load before it can issue its data loads.
struct Tile {
  int slot;
  int blk;
  int r0, r1;
  int k0, k1;
  int flags;  // TileFlag bits: data that are uniform over the block's rows
  int base;   // smallest gathered index of the block, or -1: the block's
              // entries are read from the packed words (see kPackShift)
};

// Packed entry of a row block in column order: (LDS slot << kPackShift) |
// (gathered index - block base).  Blocks whose gathered indices span
// 2^kPackShift or more, and long-row blocks, keep the separate index and
// slot arrays (Tile::base = -1).
constexpr int kPackShift = 21;
constexpr unsigned kPackMask = (1u << kPackShift) - 1;
static_assert(kNnzTile <= (1 << (32 - kPackShift)), "LDS slot must fit the packed word");

// A row block of A^T (columns of A) whose c, l or u take one known value on
// every column, or a row block of A whose b is zero on every row, does not
// read that vector: the half-step kernels substitute the value.  The flags
// are exact (bit patterns) and are recomputed whenever the data change.
enum TileFlag {
  kColC0 = 1,     // c_j == +0
  kColL0 = 2,     // l_j == +0
  kColLInf = 4,   // l_j == -inf
  kColLNegU = 8,  // l_j == -u_j
  kColUInf = 16,  // u_j == +inf
  kRowB0 = 1,     // b_i == +0
  kRowYlo = 2     // inequality duals bounded below by SlotDev::ylo instead of 0
};

// ---- launchers (kernels.hip) --------------------------------------------
// prec: 0 = FP64, 1 = FP32.  All launches go to `s`.
// e0/e1 (optional): events that record the start and end of the kernel itself
// threads: workgroup size of the half-steps, 0 = by launch size (kRowsPerBlock
// threads, one row each, below kFewTiles tiles; kThreads otherwise)
constexpr int kFewTiles = 1024;
void launch_primal(int prec, bool check, const SlotDev* slots, const Tile* tiles, int ntiles,
                   int jiter, int nscen, hipStream_t s, hipEvent_t e0 = nullptr,
                   hipEvent_t e1 = nullptr, int threads = 0);
void launch_dual(int prec, bool check, const SlotDev* slots, const Tile* tiles, int ntiles,
                 int jiter, int nscen, hipStream_t s, hipEvent_t e0 = nullptr,
                 hipEvent_t e1 = nullptr, int threads = 0);
void launch_kkt(int prec, const SlotDev* slots, const Tile* ttiles, int nttiles,
                const Tile* atiles, int natiles, int nscen, hipStream_t s);
// Two-level deterministic reduction of the KKT partials of each listed slot
// into its scal: kRedChunks workgroups per slot each reduce a fixed range of
// row blocks into red2 (nslots * kRedChunks * (RQ_N + CQ_N) doubles), then one
// workgroup per slot reduces those in a fixed order.
constexpr int kRedChunks = 64;
void launch_reduce(const SlotDev* slots, const int* slot_ids, int nslots, int nscen, double* red2,
                   hipStream_t s);
void launch_finish(int prec, const SlotDev* slots, const Tile* ttiles, int nttiles,
                   const Tile* atiles, int natiles, int kk, int nscen, hipStream_t s);
void launch_promote(const SlotDev* slots, const Tile* ttiles, int nttiles, const Tile* atiles,
                    int natiles, int nscen, hipStream_t s);
// the engine's check of every active slot (check.h), and a device clock stamp
struct ChkState;
struct ChkParams;
void launch_engine_check(SlotDev* slots, ChkState* chk, const ChkParams* prm, int nslots, hipStream_t s);
void launch_stamp(unsigned long long* t, hipStream_t s);

// scenario batches (nscen <= kMaxScen interleaved scenarios in slot 0)
// vec: the batch width is a multiple of the lanes of a 16-byte vector (4 FP32
// or 2 FP64 values) and every vector is 16-byte aligned; a thread then serves
// that many consecutive scenarios with one access per element
void launch_primal_ms(int prec, bool check, bool vec, const SlotDev* slots, const Tile* tiles, int ntiles,
                      int jiter, hipStream_t s);
void launch_dual_ms(int prec, bool check, bool vec, const SlotDev* slots, const Tile* tiles, int ntiles,
                    int jiter, hipStream_t s);
// KKT partials and their reduction into slots[0].scal[s * kScal + q]
void launch_kkt_ms(int prec, const SlotDev* slots, const Tile* ttiles, int nttiles, const Tile* atiles,
                   int natiles, double* red2, hipStream_t s);
// doubles of the red2 buffer that launch_kkt_ms needs
size_t red2_ms_doubles();
void launch_finish_ms(int prec, const SlotDev* slots, int64_t nx, int64_t ny, int kk, hipStream_t s);
void launch_promote_ms(const SlotDev* slots, int64_t nx, int64_t ny, hipStream_t s);

// iterative refinement: one round boundary of one instance (scaled space).
// Original scaled data are formed on the fly from the unscaled internal data
// and D_r, D_c, with the operations of the setup.
enum RefQ {
  FQ_VIOL2 = 0,  // ||v||^2, v = (b_hat - A_hat x*) with G rows max(., 0)
  FQ_R2U,        // sum ((b_hat - A_hat x*)_i / D_r,i)^2  (||b~|| / D_P, unscaled)
  FQ_VIOL2U,     // sum (v_i / D_r,i)^2
  FQ_BY,         // b_hat' y*
  FQ_VMAXU,      // max |v_i / D_r,i|
  FQ_DRES2,      // ||e||^2, e = d - lambda(d), d = c_hat - A_hat' y*
  FQ_D2U,        // sum (d_j / D_c,j)^2  (||c~|| / D_D, unscaled)
  FQ_DRES2U,     // sum (e_j / D_c,j)^2
  FQ_LBUB,       // sum l_hat lambda+ + u_hat lambda-
  FQ_CX,         // c_hat' x*
  FQ_N
};
struct RefineArgs {
  const int *a_ptr, *a_col, *t_ptr, *t_col, *a_blk, *t_blk;
  const double *a_v, *t_v;                     // scaled FP64 values, CSR order
  const double *c_in, *b_in, *l_in, *u_in;     // unscaled internal data
  const double *dr, *dc;
  int m, n, m_eq, a_nblk, t_nblk, first;
  double inv_dp, inv_dd;                       // 1/D_P, 1/D_D of the correction folded in
  double dp, dd;                               // D_P, D_D of the next correction problem
  double* xs;  // refined point x* (n), y* (m), FP64
  double* ys;
  const float* xc;  // correction solve output (n), (m)
  const float* yc;
  double* r;       // b_hat - A_hat x* (m)
  double* d;       // c_hat - A_hat' y* (n)
  double* part_a;  // FQ partials per row block of A  (a_nblk * 5)
  double* part_t;  // FQ partials per row block of A^T (t_nblk * 5)
  double* out;     // FQ_N reduced scalars
  double *c64, *l64, *u64, *b64;              // correction data, FP64
  float *c32, *l32, *u32, *b32, *ylo32;       // and as the FP32 solve reads them
};
// fold the correction into (x*, y*), then residuals and their FQ scalars
void launch_refine_measure(const RefineArgs& R, hipStream_t s);
// correction data of the next round from r, d, x*, y* and R.dp, R.dd
void launch_refine_form(const RefineArgs& R, hipStream_t s);

// setup
void launch_expand_rows(const int* ptr, int m, int* row_of, hipStream_t s);
void launch_gather_transpose(const int* perm, const int* row_of, const double* val, int64_t nnz,
                             int* t_col, double* t_val, hipStream_t s);
size_t radix_sort_temp_bytes(int64_t nnz, int n);
// returns the hipError_t of the sort (0 = hipSuccess)
int radix_sort_pairs(void* temp, size_t temp_bytes, const int* keys_in, int* keys_out,
                     const int* vals_in, int* vals_out, int64_t nnz, int n, hipStream_t s);
void launch_iota(int* v, int64_t n, hipStream_t s);
// stable sort of (key, value) pairs inside each segment [off[b], off[b+1])
size_t seg_sort_temp_bytes(int64_t nnz, int nseg, int ncols);
int seg_sort_pairs(void* temp, size_t temp_bytes, const int* keys_in, int* keys_out, const int* vals_in,
                   int* vals_out, int64_t nnz, int nseg, const int* off, int ncols, hipStream_t s);
// vs*[k] = v*[perm[k]], dst[k] = perm[k] - off[b] for the segment b holding k
void launch_gather_sorted(const int* perm, const int* off, int nseg, const double* v64, const float* v32,
                          double* vs64, float* vs32, unsigned short* dst, const int* cs,
                          const int* base, unsigned* pk, hipStream_t s);
// op 0: row max |a| D_r D_c ; op 1: row sum of |a| D_r D_c.  Result -> fac[r] = 1/sqrt(v) or 1.
void launch_scale_factor(int op, const int* ptr, const int* col, const double* val, const double* drow,
                         const double* dcol, const int* blk, int nblk, int rows, double* fac,
                         hipStream_t s);
void launch_mul_inplace(double* d, const double* f, int n, hipStream_t s);
void launch_scale_values(const int* ptr, const int* col, const double* raw, const double* drow,
                         const double* dcol, int rows, double* v64, float* v32, hipStream_t s);
void launch_fill(double* d, double v, int64_t n, hipStream_t s);
// c_hat = c*dc, l_hat = l/dc, u_hat = u/dc (n); b_hat = b*dr (m); FP32 copies; per scenario.
void launch_scale_vectors(const double* c, const double* l, const double* u, const double* b,
                          const double* dc, const double* dr, int n, int m, int nscen,
                          double* c64, double* l64, double* u64, double* b64, float* c32,
                          float* l32, float* u32, float* b32, hipStream_t s);
// plain SpMV y = A x on one matrix (FP64 values and accumulation)
void launch_spmv64(const int* ptr, const int* col, const double* val, const double* x, double* y,
                   const int* blk, int nblk, hipStream_t s);
void launch_spmv32(const int* ptr, const int* col, const float* val, const float* x, float* y,
                   const int* blk, int nblk, hipStream_t s);
// merge-path SpMV: at most kMergeTile merge items (row ends + entries) per
// workgroup, kMergeItems per thread; tiles start every kMergeStep items,
// moved back by at most kMergeSlack to a row start.  nwg =
// merge_workgroups(m, nnz) workgroups and scratch of coord[nwg + 1],
// carry_row[nwg], carry_val[nwg]
constexpr int kMergeItems = 8;
constexpr int kMergeTile = kThreads * kMergeItems;
constexpr int kMergeSlack = kThreads;
constexpr int kMergeStep = kMergeTile - kMergeSlack;
int merge_workgroups(int m, int64_t nnz);
// planned: coord[] already holds the workgroups' merge coordinates (they
// depend on the row pointers only; launch_merge_coords computes them), and
// fixup = false skips the carry fix-up (correct when no tile ends inside a
// row); unplanned launches compute the coordinates and always fix up
void launch_spmv_merge64(const int* ptr, const int* col, const double* val, const double* x,
                         double* y, int m, int64_t nnz, int2* coord, int* carry_row, double* carry_val,
                         hipStream_t s, bool planned = false, bool fixup = true);
void launch_spmv_merge32(const int* ptr, const int* col, const float* val, const float* x, float* y,
                         int m, int64_t nnz, int2* coord, int* carry_row, float* carry_val, hipStream_t s,
                         bool planned = false, bool fixup = true);
void launch_merge_coords(const int* ptr, int m, int64_t nnz, int2* coord, hipStream_t s);
// sum of squares of v (n) into *out (deterministic two-pass); part sized >= 1024
void launch_norm2(const double* v, int64_t n, double* part, double* out, hipStream_t s);
// v = w / sqrt(*nrm2)
void launch_normalize(const double* w, const double* nrm2, double* v, int64_t n, hipStream_t s);
void launch_hash_vector(double* v, int64_t n, uint32_t seed, hipStream_t s);
// initial iterates: x = clamp(x_in/dc or 0), y = y_in/dr or 0 (projected), anchors = start
void launch_init_iterates(const SlotDev* slot, int prec, const double* x_in, const double* y_in,
                          int n, int m, int m_eq, int nscen, hipStream_t s);
// x_out = dc * x_hat ; y_out = dr * y_hat (FP64 outputs, per scenario interleaved)
void launch_unscale(const SlotDev* slot, int prec, double* x_out, double* y_out, int n, int m,
                    int nscen, hipStream_t s);
void launch_to_f32(const double* a, float* b, int64_t n, hipStream_t s);
void launch_copy_kernel(const float4* a, float4* b, int64_t n4, hipStream_t s);

}  // namespace uclp
