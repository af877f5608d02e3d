// Host-side launchers of the liblogdet device kernels.  Every launcher checks
// the shapes its kernel and grid assume and returns hipErrorInvalidValue
// instead of launching when they do not hold.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "ld_device.h"

namespace ld {

enum ValueType : int { VT_F64 = 0, VT_F32 = 1, VT_BF16 = 2 };

constexpr int kMaxBlocks = 2048;  // 256 CUs x 8 resident 256-thread blocks
constexpr int kMaxC = 4;          // 16-byte chunks per lane
constexpr int kMaxLd = 256;       // probe-block row length (columns) of the Krylov kernels
constexpr int kMaxRowStride = 32767;  // Geom::ts
constexpr int kSoSlqMaxSketch = 48;  // So-SLQ sketch width (Jacobi eigen-solve in LDS)

// Row partition of an [n][ld] probe block.  The streaming kernels sweep
// chunks of 4 floor(64/L) consecutive rows (256/L for a power-of-two L),
// block b taking chunks b, b+nblk, ...; the sketch kernels give block b the
// rows [b*rpb, min(n, (b+1)*rpb)).  A row is handled by L lanes, each
// touching C chunks of `vec` consecutive columns (16 bytes).
// The partition fixes the order of every reduction, so results are bitwise
// reproducible for a given (n, ld, element size).  Per-block partial sums are
// stored transposed: part[i * nblk + block].
struct Geom {
  int64_t n = 0;
  int ld = 0;      // leading dimension (multiple of 4)
  int xbytes = 8;  // element size: 8 (FP64) or 4 (FP32)
  int vec = 2;
  int ncolv = 0;   // ld / vec
  int L = 1;       // lanes per row (<= 64; a power of two with an entry split)
  int lgL = 0;     // log2(L)
  int C = 1;       // 16-byte chunks per lane (<= 4), L * C >= ncolv
  int nblk = 0;
  int rpb = 0;     // rows per block
  int lges = 0;    // product only: log2 of the entry split (L / 2^lges column lanes)
  int xil = 0;     // product only: 1 = consecutive row chunks on consecutive blocks
                   // (XCDs interleaved), 0 = a contiguous band of chunks per XCD
  int ts = 0;      // product only, L a power of two: 0, or S = a multiple of the rows
                   // per wave (64 / L): the block's 4 waves take rows S apart (one
                   // tile of 4 rows of S rows), so a stencil's +-S neighbours of
                   // one wave's rows are the rows its sibling waves gather
  int rg = 0;      // product only: 1 = the matrix's row groups (RowGroups below)
                   // instead of its CSR rows; FP32 values on FP32 vectors or
                   // FP64 values on FP64 or FP32 vectors, C <= 2, no entry
                   // split, no row tiles
};
Geom make_geom(int64_t n, int ld, int xbytes);
// The same with an explicit lanes-per-row L and chunks per lane C (an
// autotuned choice); geom_usable tells whether it covers ld.
Geom make_geom_lc(int64_t n, int ld, int xbytes, int L, int C);
bool geom_usable(const Geom& g);

// Row groups of a CSR matrix: rows kRowGroup g .. kRowGroup g + kRowGroup - 1
// form group g; its entries are the sorted union of the rows' columns,
// col[gp[g] .. gp[g+1]), and for each union column u the kRowGroup values
// val[kRowGroup u + r] of row r (zero where the row has no entry there).
// One gather of a neighbour's probe row then serves every row of the group
// that references it; the rows' sums see their nonzero terms in CSR order.
constexpr int kRowGroup = 4;
struct RowGroups {
  const int* gp = nullptr;
  const int* col = nullptr;
  const float* val = nullptr;    // FP32 values (FP32 probe blocks)
  const double* val64 = nullptr;  // FP64 values (FP64 probe blocks)
};

// Row groups of an n-row CSR matrix (rows sorted) on the device: cnt[g] =
// group g's union columns; then, with gp the exclusive prefix sums of cnt
// (gp[g] = first union column of group g), the union columns col and their
// values, kRowGroup per column: val (v64 rounded to FP32) and val64 (v64
// itself), each when not null.
hipError_t launch_rowgroup_count(hipStream_t st, int64_t n, const int* rp, const int* ci, int* cnt);
hipError_t launch_rowgroup_fill(hipStream_t st, int64_t n, const int* rp, const int* ci,
                                const double* v64, const int* gp, int* col, float* val,
                                double* val64);

// ---------------------------------------------------------------------------
// Batched per-step launches: one launch advances the same kernel for up to
// kMaxBatch requests (the scheduler's continuous batching); a single request
// is a batch of one.  Device-side descriptors travel by value in the kernel
// arguments; entry r owns grid blocks (or outputs) off[r] .. off[r+1]-1.
// ---------------------------------------------------------------------------
constexpr int kMaxBatch = 16;

template <typename D>
struct BatchArgs {
  int count;
  int off[kMaxBatch + 1];
  D d[kMaxBatch];
};

struct SpmmDesc {
  int64_t n;
  const int* rp;
  const int* ci;
  const void* va;
  const void* X;
  void* W;
  const double* xmult;
  double opscale;
  const void* fx[2];
  const double* fmult[2];
  double* part;
  int L, lgES, ld, ncolv, voff;  // L lanes per row (see Geom)
  int il;                        // Geom::xil
  int ts;                        // Geom::ts
  // optional early subtraction W -= sd[col] * smult[col] * sx[row][col]
  // (a window vector whose coefficient is known before the product)
  const void* sx;
  const double* smult;
  const double* sd;
};

struct UpdDesc {
  int64_t n;
  void* W;
  const void* vx[kMaxNv];
  const double* vmult[kMaxNv];
  const double* d;
  const void* v1;
  const double* v1mult;
  double* part;
  int L, ld, ncolv, nv, voff, want_norm;
  int dhole;  // 0, or 1 + a coefficient row the vectors skip
};

struct RedDesc {
  const double* part;
  double* out;
  int nblk, width;
};

struct FinDesc {
  double* d;
  const double* part;
  double* H;
  int* meff;
  int* active;
  double* mult_next;
  double* g;
  int* flags;
  const double* gin_mult;  // non-null: also g[t] from part[3]
  double tol;
  double inv_s;  // 1 / the power-of-two scale the product output is stored at
  int B, ld, t, m, j0, nv, nblk, sym_row;
};

// Columns col0 .. col0+ncols-1 of X: probe columns pbase .. pbase+nvalid-1,
// then zeros up to ncols (padding).
// With seed_dev, the kernels read the seed from that device word instead (a
// launch sequence that does not depend on the seed, e.g. a replayed graph).
hipError_t launch_rademacher(hipStream_t st, uint64_t seed, int64_t n, int pbase, int ncols,
                             int nvalid, void* X, int xbytes, int ld, int col0,
                             const uint64_t* seed_dev = nullptr);
// Same for either distribution (PROBE_RADEMACHER or PROBE_GAUSSIAN).
constexpr int PROBE_RADEMACHER = 0;
constexpr int PROBE_GAUSSIAN = 1;
hipError_t launch_probes(hipStream_t st, int dist, uint64_t seed, int64_t n, int pbase, int ncols,
                         int nvalid, void* X, int xbytes, int ld, int col0,
                         const uint64_t* seed_dev = nullptr);
// Rademacher probe columns pbase .. pbase+ncols-1 as sign bits: bit j of
// masks[row][w] is 1 where column pbase + 64 w + j holds -1 (the same Philox
// bits as launch_rademacher); nw = ceil(ncols / 64) words per row.
hipError_t launch_rademacher_mask(hipStream_t st, uint64_t seed, int64_t n, int pbase, int ncols,
                                  uint64_t* masks, int nw, const uint64_t* seed_dev = nullptr);

// A block of FP64 probe columns read by the sketch kernels: dense values
// (dense[row * ld + j]) or Rademacher signs packed 64 per word
// (mask[row * nw + j / 64], bit j % 64 set for -1).
struct GSrc {
  const double* dense;
  int ld;
  const uint64_t* mask;
  int nw;
};
__device__ inline double gsrc_at(const GSrc& g, int64_t row, int j) {
  if (g.dense) return g.dense[(size_t)row * g.ld + j];
  const uint64_t w = g.mask[(size_t)row * g.nw + (j >> 6)];
  return ((w >> (j & 63)) & 1ull) ? -1.0 : 1.0;
}

// W = opscale * (Q X) * diag(xmult); X, W share ld/type.  With nf (<= 2)
// fused vectors: part[voff+v][col][block] = mult_v[col] * sum x_v w, where
// fused->x[nf-1] must be X itself.  The streaming launchers pick their own
// grid (at most one resident wave of blocks) and report it in *nblk_out, the
// block count of the partial sums they wrote (at most kMaxBlocks).
// With sx: before the epilogue's inner products and the store, W[row][col]
// -= sd[col] * smult[col] * sx[row][col] in the update's arithmetic (sx is a
// window vector, sd its coefficient row, smult its multipliers).
// With g.rg the product reads the row groups `rg` instead of rp / ci / va
// (their FP32 values with vt = VT_F32 on FP32 blocks, their FP64 values with
// vt = VT_F64 on FP64 or FP32 blocks).
hipError_t launch_spmm(hipStream_t st, const Geom& g, const int* rp, const int* ci,
                       const void* va, int vt, const void* X, void* W,
                       const double* xmult, double opscale, const VecSet* fused, int nf,
                       int voff, double* part, int* nblk_out, const void* sx = nullptr,
                       const double* smult = nullptr, const double* sd = nullptr,
                       const RowGroups* rg = nullptr);

// part[voff+v][col][block] = mult_v[col] * sum_{rows of block} x_v[row][col] w[row][col],
// v < nv <= kDotsPerLaunch, or nv <= kDotsWide with one chunk per lane (FP32
// or FP64 vectors)
constexpr int kDotsPerLaunch = 4;
constexpr int kDotsWide = 8;
hipError_t launch_dots(hipStream_t st, const Geom& g, const void* W, const VecSet& vs, int nv,
                       int voff, double* part, int* nblk_out);

// w[row][col] -= sum_v d[voff+r(v)][col] * mult_v[col] * x_v[row][col] (nv <= kMaxNv,
// at most 4 with FP16 vectors; r(v) = v, or v + 1 from v = dhole - 1 on when
// dhole > 0: the vectors skip that coefficient row); when
// want_norm: part[0][col][block] = sum w^2, part[1][col][block] = v1mult[col] *
// sum v1[row][col] w[row][col] and part[3][col][block] = v1mult[col] * sum
// v1[row][col] x_{nv-1}[row][col] (the newest input vector; both zero when v1
// is null) and, with sym, part[2][col][block] = sum w_in[row][col]
// w[row][col] (w_in: W before the update).
hipError_t launch_update(hipStream_t st, const Geom& g, void* W, const VecSet& vs, int nv,
                         const double* d, int voff, int want_norm, const void* v1,
                         const double* v1mult, bool sym, double* part, int* nblk_out,
                         int dhole = 0);

// Host-side items of the batched launchers (same meaning as the arguments of
// launch_spmm / launch_update / launch_reduce / launch_step_finish); nblk is
// an output (the partial-sum blocks the item's product or update used).
struct SpmmItem {
  Geom g;
  const int* rp;
  const int* ci;
  const void* va;
  int vt;
  const void* X;
  void* W;
  const double* xmult;
  double opscale;
  VecSet fused;
  int nf;
  int voff;
  double* part;
  int nblk;
  const void* sx;  // optional early subtraction (see launch_spmm)
  const double* smult;
  const double* sd;
  RowGroups rg;  // with g.rg
};
struct UpdateItem {
  Geom g;
  void* W;
  VecSet vs;
  int nv;
  const double* d;
  int voff;
  int want_norm;
  const void* v1;
  const double* v1mult;
  bool sym;
  double* part;
  int nblk;
  int dhole;  // see launch_update
};
struct ReduceItem {
  const double* part;
  int nblk;
  int width;
  double* out;
};
struct FinishItem {
  int B, ld, t, m;
  double* d;
  int j0, nv;
  const double* part;
  int nblk;
  double tol;
  double* H;
  int* meff;
  int* active;
  double* mult_next;
  double* g;
  int* flags;
  int sym_row;
  double inv_s;
  // with g: g[t] = (reduced part[3]) * gin_mult[p] as well (the v1 dot of the
  // step's input vector), also on a breakdown step
  const double* gin_mult = nullptr;
};
hipError_t launch_spmm_batch(hipStream_t st, SpmmItem* items, int count);
// The row-group items of a batch (g.rg, checked by launch_spmm_batch), at
// most kMaxBatch of them with the same C and nf: one launch.
hipError_t launch_spmm_rg_group(hipStream_t st, SpmmItem* items, const int* idx, int cnt);
// Grid of a streaming kernel `fn` over g's rows (row groups with g.rg): at
// most one resident wave of blocks, a multiple of 8 from 8 blocks up.
int stream_grid(const Geom& g, const void* fn);
hipError_t launch_update_batch(hipStream_t st, UpdateItem* items, int count);
hipError_t launch_reduce_batch(hipStream_t st, const ReduceItem* items, int count);
hipError_t launch_step_finish_batch(hipStream_t st, const FinishItem* items, int count);

// out[i] = sum_{b < nblk} part[i*nblk + b], fixed order.
hipError_t launch_reduce(hipStream_t st, const double* part, int nblk, int width, double* out);

// Per-probe bookkeeping (B real probes, ld columns), each fused with the
// reduction of the partial sums it consumes (part in the transposed layout).
// The start block is stored at the scale 1 / inv_oscale (its squared norms
// are those of the unscaled vectors); the product output at 1 / inv_s.
hipError_t launch_start_finish(hipStream_t st, int B, int ld, const double* part, int nblk,
                               double* norm2, double* mult0, int* active, int* meff, double* g,
                               int gstride, double inv_oscale);
// With sym_row >= 0 it also reduces part[2] and stores, per probe, the inner
// product of the new vector with the product it came from (sum / ||w||) in
// d[sym_row][p], where the next step's window inner products are read.
// With g it stores g[p][t+1] = v1^T v_{t+1} from part[1] and, when gin_mult
// is given, g[p][t] = v1^T v_t from part[3] times gin_mult (mult_t).
hipError_t launch_step_finish(hipStream_t st, int B, int ld, int t, int m, double* d, int j0,
                              int nv, const double* part, int nblk, double tol, double* H,
                              int* meff, int* active, double* mult_next, double* g, int* flags,
                              int sym_row, double inv_s, const double* gin_mult = nullptr);

// Gauss quadrature of log on each probe's T (diag h_tt, subdiag h_t+1,t).
// (need: when non-null, only runs with need[p] != 0 are evaluated.)
hipError_t launch_gauss_log(hipStream_t st, int B, int m, const double* H, const int* meff,
                            double* K, int* flags, const int* need);
// The same value K = e1^T log(T) e1 from the trapezoidal rule on the Stieltjes
// integral of log, valid when T's spectrum lies in [a, b]; runs whose T has
// an eigenvalue outside [a/1000, 1000 b] get need[p] = 1 (left to the
// Golub-Welsch kernel), the others need[p] = 0.
hipError_t launch_quad_log(hipStream_t st, int B, int m, const double* H, const int* meff, double a,
                           double b, double* K, int* need, int* flags);
// Adaptive Krylov dimension: for the active runs at dimension dim, K from the
// same rule is compared with kprev (then replaced); a run whose K moved by at
// most rtol |K| stops (active = 0, mult_next = 0, flag bit 4); nactive is
// incremented once per run still active.
hipError_t launch_quad_check(hipStream_t st, int B, int m, const double* H, const int* meff,
                             double a, double b, int dim, int* active, double* kprev, double rtol,
                             double* mult_next, int* flags, int* nactive);

// OSA-IOP: Gauss-Legendre rule of the Pade step of log(H) e1 (nodes on [0, 1]).
struct LogRule {
  double x[10];
  double w[10];
};
// mode 0: ell[p][t] = (log H_p e1)_t; mode 1: K[p] = sum_t g[p][t] (log H_p e1)_t + shift.
// work: wstride >= hess_log_wstride(m) doubles per run; need: B ints of scratch.
// Runs whose H is symmetric tridiagonal to within symtol * max|h| take the
// trapezoidal Stieltjes rule (spectrum inside [a, b], the operator's
// interval) or else the O(m^2) eigen-path; the others inverse scaling and
// squaring.
int hess_log_wstride(int m);
hipError_t launch_hess_log(hipStream_t st, int B, int m, const double* H, const int* meff,
                           double a, double b, double* work, int wstride, int mode, double* ell,
                           const double* g, double shift, double* K, int* flags, double symtol,
                           int* need);
hipError_t launch_osa_coef(hipStream_t st, int B, int ld, int m, const double* ell,
                           const double* mult, const double* norm2, const int* meff, double shift,
                           double* coef);
// Y[row][col] = sum_{t < nt} coef[t][col] X_t[row][col], X_t = slots + t * slot_elems;
// with accumulate the sum continues from Y (the same FMA chain as one pass).
hipError_t launch_combine(hipStream_t st, int64_t n, int ld, int nt, const void* slots, int xbytes,
                          size_t slot_elems, const double* coef, double* Y, int ldy,
                          bool accumulate = false);

// Dense pieces of the Hutch++ sketch (FP64).
// part[i][j][b] = sum_{rows of b} Xa[row][i] * Xb[row][j], i < ca, j < cb
hipError_t launch_gemm_tn(hipStream_t st, const Geom& g, const double* Xa, int lda, int ca,
                          const double* Xb, int ldb, int cb, double* part);
// Y = opscale (Q S) in FP64 for Rademacher S given as sign words
// (masks[row][w], bit j of word w set where column 64 w + j holds -1; columns
// s .. ldy-1 of Y are zero): each entry gathers one word instead of a row of
// S.  Entries accumulate in CSR order with one FMA each, as in launch_spmm on
// the FP64 +-1 block.  ldy even, s <= ldy <= 128, nw = ceil(s / 64).
hipError_t launch_spmm_signs(hipStream_t st, int64_t n, const int* rp, const int* ci,
                             const void* va, int vt, const uint64_t* masks, int nw, int s,
                             double* Y, int ldy, double opscale);
// Same with the right operand given as dense columns or packed signs.
hipError_t launch_gemm_tn_g(hipStream_t st, const Geom& g, const double* Xa, int lda, int ca,
                            const GSrc& Xb, int cb, double* part);
hipError_t launch_chol_inv(hipStream_t st, int s, const double* G, double* work, double* Rinv,
                           int* flag);
hipError_t launch_trsm_rows(hipStream_t st, int64_t n, double* Y, int ld, int s, const double* Rinv);
// Y[row][j] <- sum_{i < s} Y[row][i] M[i][j], j < sout <= s (M is s x sout), in place.
hipError_t launch_rows_mat(hipStream_t st, int64_t n, double* Y, int ld, int s, const double* M,
                           int sout);
// U (q x k, row-major): v_j / sqrt(lambda_j) for the eigenpairs of the Gram
// matrix G (q x q, q <= 48) with the k largest eigenvalues; flag = 1 when
// Jacobi did not converge or lambda_k <= 1e-13 lambda_1.
hipError_t launch_subspace_eig(hipStream_t st, int q, int k, const double* G, double* U, int* flag);
// X0[row][i] = A[row][i] (i < s); X0[row][s+j] = G[row][j] - sum_i A[row][i] P[i][j];
// part[col][b] = sum over rows of b of X0[row][col]^2 (FP64 values).
// X0 is stored at the scale oscale (a power of two); the norm partials are
// those of the unscaled FP64 vectors.
hipError_t launch_project(hipStream_t st, const Geom& g, const double* A, int lda, int s,
                          const GSrc& Gm, int r, const double* P, void* X0, double* part,
                          double oscale);

// Fill up to kMaxFill ranges of 32-bit words with a value each, in one launch
// (kernels, not memset nodes: the estimate's launches can be captured in a
// HIP graph and replayed).
constexpr int kMaxFill = 4;
struct FillItem {
  void* p;
  size_t n32;    // 32-bit words
  uint32_t val;
};
hipError_t launch_fill(hipStream_t st, const FillItem* items, int count);

// dst[0 .. n32) = src[0 .. n32), 32-bit words (a kernel rather than a copy
// node when the sequence is captured in a graph).
hipError_t launch_copy_words(hipStream_t st, void* dst, const void* src, size_t n32);

// The per-run results an estimate hands back, packed for one copy:
// [K: ld doubles | norm2: ld doubles | meff: ld ints | flags: ld ints |
//  dflag: 4 ints | meff0: ld ints] (meff0 may be null: zeros).
inline size_t pack_results_bytes(int ld) { return (size_t)ld * 28 + 16; }
constexpr size_t kHostPackBytes = 8192;  // >= pack_results_bytes(kMaxLd)
static_assert((size_t)kMaxLd * 28 + 16 <= kHostPackBytes, "host pack buffer too small");
hipError_t launch_pack_results(hipStream_t st, int ld, const double* K, const double* norm2,
                               const int* meff, const int* flags, const int* dflag,
                               const int* meff0, void* out);

// Plain device copy of `bytes` (multiple of 16 used), calibration only.
hipError_t launch_copy16(hipStream_t st, const void* src, void* dst, size_t bytes);
// Bandwidth probe: reads `reads` (1..3) streams src[0..reads-1] of `bytes`
// each and writes their sum to dst (writes = 1); with writes = 0 the sums
// stay in registers and reach sink (kMaxBlocks * kThreads floats) only if
// one is not a number.
hipError_t launch_stream_rw(hipStream_t st, int reads, int writes, const void* const* src, void* dst,
                            float* sink, size_t bytes);

// Matrix set-up.
hipError_t launch_gershgorin(hipStream_t st, int64_t n, const int* rp, const int* ci,
                             const double* va, double* part, int* nparts);

}  // namespace ld
