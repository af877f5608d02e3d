// Streaming kernels of the Krylov hot loop: probe generation, the CSR
// product over a probe block, the window inner products, the update/norm
// pass, fixed-order reductions and the per-probe step bookkeeping.
//
// Layout: a probe block is row-major [n][ld] (ld a multiple of 4, padding
// columns held at zero), so one sparse entry gathers one contiguous run of
// probe values.  Every reduction goes through per-block partial sums in a
// fixed order (no floating-point atomics): results are bitwise reproducible.
#include "ld_kernels.h"
#include <type_traits>
#include "gw_ql.h"

#include <algorithm>
#include <map>
#include <vector>
#include <mutex>

namespace ld {

// ---------------------------------------------------------------------------
// Philox4x64-10 (Salmon et al., SC'11) and Rademacher probes.
// Probe column p, row i: block at counter (i / 256, p, 0, 0), key (seed, 0);
// bit i % 64 of word (i / 64) % 4; set -> -1, clear -> +1.
// ---------------------------------------------------------------------------
__device__ inline void philox4x64_10(uint64_t& c0, uint64_t& c1, uint64_t& c2, uint64_t& c3,
                                     uint64_t k0, uint64_t k1) {
  constexpr uint64_t kM0 = 0xD2E7470EE14C6C93ull, kM1 = 0xCA5A826395121157ull;
  constexpr uint64_t kW0 = 0x9E3779B97F4A7C15ull, kW1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
  for (int rnd = 0; rnd < 10; ++rnd) {
    if (rnd) { k0 += kW0; k1 += kW1; }
    const uint64_t lo0 = kM0 * c0, hi0 = __umul64hi(kM0, c0);
    const uint64_t lo1 = kM1 * c2, hi1 = __umul64hi(kM1, c2);
    const uint64_t n0 = hi1 ^ c1 ^ k0;
    const uint64_t n2 = hi0 ^ c3 ^ k1;
    c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
  }
}

template <typename T>
__global__ __launch_bounds__(kThreads) void k_rademacher(uint64_t seed, const uint64_t* seed_dev,
                                                        int64_t n, int pbase, int ncols, int nvalid,
                                                        T* __restrict__ X, int ld, int col0) {
  if (seed_dev) seed = *seed_dev;
  __shared__ uint64_t words[64][4];
  const int64_t r0 = (int64_t)blockIdx.x * 256;
  const int cbase = blockIdx.y * 64;
  const int nc = min(64, ncols - cbase);
  if ((int)threadIdx.x < nc) {
    uint64_t c0 = (uint64_t)blockIdx.x, c1 = (uint64_t)(pbase + cbase + (int)threadIdx.x), c2 = 0,
             c3 = 0;
    philox4x64_10(c0, c1, c2, c3, seed, 0ull);
    words[threadIdx.x][0] = c0;
    words[threadIdx.x][1] = c1;
    words[threadIdx.x][2] = c2;
    words[threadIdx.x][3] = c3;
  }
  __syncthreads();
  for (int e = threadIdx.x; e < 256 * nc; e += kThreads) {
    const int rr = e / nc, j = e - (e / nc) * nc;
    const int64_t row = r0 + rr;
    if (row >= n) break;
    const uint64_t w = words[j][(rr >> 6) & 3];
    const T val = ((w >> (rr & 63)) & 1ull) ? T(-1) : T(1);
    X[(size_t)row * ld + col0 + cbase + j] = (cbase + j < nvalid) ? val : T(0);
  }
}

// Gaussian probe columns: Box-Muller on Philox4x64-10 words.  Thread (b, j)
// takes the block at counter (b, pbase + cbase + j, 1, 0) and writes rows
// 4b..4b+3 of column j: words (w0, w1) give rows 4b, 4b+1 and (w2, w3) rows
// 4b+2, 4b+3, each pair as u1 = ((wa >> 11) + 1) 2^-53 in (0, 1],
// u2 = (wb >> 11) 2^-53, rho = sqrt(-2 log u1), rows rho cos(2 pi u2) and
// rho sin(2 pi u2).  Columns are the fastest thread index so that a wave
// writes contiguous row segments.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_gaussian(uint64_t seed, const uint64_t* seed_dev,
                                                      int64_t n, int pbase, int ncols, int nvalid,
                                                      T* __restrict__ X, int ld, int col0) {
  if (seed_dev) seed = *seed_dev;
  const int j = (int)(threadIdx.x % 64) + 64 * (int)blockIdx.y;
  const int64_t b = (int64_t)blockIdx.x * (kThreads / 64) + threadIdx.x / 64;
  if (j >= ncols || 4 * b >= n) return;
  uint64_t c0 = (uint64_t)b, c1 = (uint64_t)(pbase + j), c2 = 1, c3 = 0;
  philox4x64_10(c0, c1, c2, c3, seed, 0ull);
  const uint64_t w[4] = {c0, c1, c2, c3};
  constexpr double kTwoPi = 6.283185307179586;
  constexpr double kInv53 = 1.0 / 9007199254740992.0;  // 2^-53
#pragma unroll
  for (int pair = 0; pair < 2; ++pair) {
    const double u1 = (double)((w[2 * pair] >> 11) + 1) * kInv53;
    const double u2 = (double)(w[2 * pair + 1] >> 11) * kInv53;
    const double rho = sqrt(-2.0 * log(u1));
    double sn, cs;
    sincos(kTwoPi * u2, &sn, &cs);
    const int64_t r0 = 4 * b + 2 * pair;
    const bool valid = j < nvalid;
    if (r0 < n) X[(size_t)r0 * ld + col0 + j] = valid ? T(rho * cs) : T(0);
    if (r0 + 1 < n) X[(size_t)(r0 + 1) * ld + col0 + j] = valid ? T(rho * sn) : T(0);
  }
}

// ---------------------------------------------------------------------------
// CSR x probe block, with up to two window inner products fused into the
// epilogue (NF of them).  The newest window vector is the product's own
// input: its value on the row comes from the gathered diagonal entry (every
// row stores its diagonal), so only an older one (NF = 2) is read again.
// W = opscale * (Q X) * diag(xmult); column index and value of an entry are
// read once by the row's lanes; each lane gathers C contiguous 16-byte
// segments of the neighbour's probe vector.  For v < NF:
// part[voff+v][col][block] = mult_v[col] * sum_rows x_v[row][col] w[row][col].
// With sx, a window vector whose coefficient sd is already known (the
// second newest, by the operator's symmetry) is subtracted from W first, in
// the update's arithmetic, so the update does not read it again; the inner
// products above then see the reduced W, as modified Gram-Schmidt would.
// ---------------------------------------------------------------------------
template <typename VT, typename XT, int C, int NF, bool SPLIT>
__device__ inline void spmm_body(int64_t n, int Lr, int lgES_arg, const int* __restrict__ rp,
                                 const int* __restrict__ ci, const VT* __restrict__ va,
                                 const XT* __restrict__ X, XT* __restrict__ W, int ld, int ncolv,
                                 const double* __restrict__ xmult, double opscale, const void* const* fx,
                                 const double* const* fmult, int voff, double* __restrict__ part,
                                 int bk, int nbk, int il, int ts, const XT* __restrict__ sx,
                                 const double* __restrict__ smult, const double* __restrict__ sd) {
  // FP32 sums for FP32 (or BF16) values on FP32 vectors; FP64 sums whenever
  // the values or the vectors are FP64
  using A = typename std::conditional<std::is_same<VT, double>::value, double,
                                      typename Acc<XT>::type>::type;
  constexpr int VEC = V16<XT>::N;
  constexpr bool FUSED = NF > 0;
  // the early subtraction's arithmetic: the update's (FP64, FP32 for FP16 vectors)
  using U = typename std::conditional<std::is_same<XT, _Float16>::value, float, double>::type;
  // one fused product: its per-thread FP64 sums live in the thread's own LDS
  // slots (fewer registers, more waves in flight for the gather); two: in
  // registers, with the LDS array used for the final column sums
  constexpr bool LDSACC = NF == 1;
  constexpr int ND = (FUSED && !LDSACC) ? NF : 1;
  // sparse entries whose (column, value) a lane loads per round
  constexpr int KE = C >= 3 ? 2 : 4;
  __shared__ double red[FUSED ? kThreads * VEC * C : 1];
  __shared__ A scs[kMaxLd];  // opscale * xmult[col], in the accumulation type
  __shared__ U scf[kMaxLd];  // sd[col] * smult[col] (early subtraction)
  // entry split only in the SPLIT instantiations (the plain path keeps its
  // registers and code)
  const int lgES = SPLIT ? lgES_arg : 0;
  const RowMap rm = RowMap::lanes(Lr, lgES);
  const int ES = 1 << lgES;
  for (int i = threadIdx.x; i < ld; i += kThreads) {
    scs[i] = A(opscale * (xmult ? xmult[i] : 1.0));
    if (sx) scf[i] = U(sd[i] * (smult ? smult[i] : 1.0));
  }
  bool okc[C];
  int colc[C];
#pragma unroll
  for (int c = 0; c < C; ++c) {
    const int cv = rm.cl + rm.Lc * c;
    okc[c] = cv < ncolv;
    colc[c] = cv * VEC;
    if constexpr (LDSACC) {
      if (rm.on)
#pragma unroll
        for (int e = 0; e < VEC; ++e) red[red_slot<C, VEC>(rm, c, e)] = 0.0;
    }
  }
  __syncthreads();
  double dacc[ND][C][VEC];
#pragma unroll
  for (int v = 0; v < ND; ++v)
#pragma unroll
    for (int c = 0; c < C; ++c)
#pragma unroll
      for (int e = 0; e < VEC; ++e) dacc[v][c][e] = 0.0;
  const int nn = (int)n;  // n < 2^31
  const int nchunk = (nn + rm.rpi - 1) / rm.rpi;
  // row tiles (ts > 0): tile t is the 4 ts consecutive rows from 4 t ts;
  // for chunk t segs + q the block's wave w takes its rpw rows from
  // 4 t ts + w ts + q rpw, so the four waves work ts rows apart; chunks past
  // the last whole tile keep consecutive rows
  const int rpw = rm.rpi >> 2;  // rows per wave (L a power of two)
  const int segs = ts > 0 ? ts / rpw : 1;
  const int tchunks = ts > 0 ? (nn / (4 * ts)) * segs : 0;
  const int wv = (int)threadIdx.x >> 6, rw = rm.rg - wv * rpw;
  for (int j = 0; j * nbk < nchunk; ++j) {
    // per-XCD bands keep a row's neighbours in one L2; interleaving streams
    // better on wide rows (a tuning choice)
    const int ch = il ? j * nbk + bk : chunk_of(j, bk, nbk);
    int row = ch * rm.rpi + rm.rg;
    if (ch < tchunks) {
      const int t = ch / segs, q = ch - t * segs;
      row = (t * 4 + wv) * ts + q * rpw + rw;
    }
    if (!rm.on || ch >= nchunk || row >= nn) continue;
    A acc[C][VEC];
    V16<XT> xd[FUSED ? C : 1];
#pragma unroll
    for (int c = 0; c < C; ++c)
#pragma unroll
      for (int e = 0; e < VEC; ++e) acc[c][e] = A(0);
    // accumulate a_k x_k in entry order; two entries' gathers in flight
    auto step2 = [&](int c0, A a0, int c1, A a1) {
      V16<XT> x0[C], x1[C];
#pragma unroll
      for (int c = 0; c < C; ++c)
        if (okc[c]) {
          x0[c].load(X + (size_t)c0 * ld + colc[c]);
          x1[c].load(X + (size_t)c1 * ld + colc[c]);
        }
#pragma unroll
      for (int c = 0; c < C; ++c)
        if (okc[c]) {
#pragma unroll
          for (int e = 0; e < VEC; ++e) {
            acc[c][e] = fma(a0, A(x0[c].v[e]), acc[c][e]);
            acc[c][e] = fma(a1, A(x1[c].v[e]), acc[c][e]);
          }
          if (FUSED) {
            if (c0 == row) xd[c] = x0[c];
            if (c1 == row) xd[c] = x1[c];
          }
        }
    };
    auto step1 = [&](int c0, A a0) {
#pragma unroll
      for (int c = 0; c < C; ++c)
        if (okc[c]) {
          V16<XT> x;
          x.load(X + (size_t)c0 * ld + colc[c]);
#pragma unroll
          for (int e = 0; e < VEC; ++e) acc[c][e] = fma(a0, A(x.v[e]), acc[c][e]);
          if (FUSED && c0 == row) xd[c] = x;
        }
    };
    const int kbeg = rp[row];
    const int kend = rp[row + 1];
    // the row's L lanes load KE * L consecutive entries (column, value) per
    // round, lane l holding entries l, l + L, ..., and pass them around the
    // group by lane shuffles; entries are accumulated in order
    for (int base = kbeg; base < kend; base += rm.L * KE) {
      int myc[KE];
      A mya[KE];
#pragma unroll
      for (int u = 0; u < KE; ++u) {
        const int kk = base + rm.gl + rm.L * u;
        myc[u] = row;
        mya[u] = A(0);
        if (kk < kend) {
          myc[u] = ci[kk];
          mya[u] = value_as<VT, A>(va[kk]);
        }
      }
#pragma unroll
      for (int u = 0; u < KE; ++u) {
        const int cnt = min(rm.L, kend - base - rm.L * u);
        if (cnt <= 0) break;
        if (ES == 1) {
          int j = 0;
          for (; j + 2 <= cnt; j += 2)
            step2(__shfl(myc[u], rm.lb + j), __shfl(mya[u], rm.lb + j),
                  __shfl(myc[u], rm.lb + j + 1), __shfl(mya[u], rm.lb + j + 1));
          if (j < cnt) step1(__shfl(myc[u], rm.lb + j), __shfl(mya[u], rm.lb + j));
        } else {
          // entry group eg: entries eg, eg + ES, ... of the round (absent
          // ones gather the row itself with a zero coefficient)
          const int ni = (cnt + ES - 1) >> lgES;
          for (int i = 0; i < ni; i += 2) {
            const int e0 = rm.eg + (i << lgES), e1 = e0 + ES;
            int c0 = __shfl(myc[u], rm.lb + e0), c1 = __shfl(myc[u], rm.lb + e1);
            A a0 = __shfl(mya[u], rm.lb + e0), a1 = __shfl(mya[u], rm.lb + e1);
            if (e0 >= cnt) {
              c0 = row;
              a0 = A(0);
            }
            if (i + 1 >= ni || e1 >= cnt) {
              c1 = row;
              a1 = A(0);
            }
            step2(c0, a0, c1, a1);
          }
        }
      }
    }
    if (ES > 1) {
      // add the entry groups' sums (a fixed butterfly: every lane of the row
      // ends with the same total); the diagonal block row is read again
#pragma unroll
      for (int c = 0; c < C; ++c)
#pragma unroll
        for (int e = 0; e < VEC; ++e)
          for (int d = rm.Lc; d < rm.L; d <<= 1) acc[c][e] += __shfl_xor(acc[c][e], d, 64);
      if (FUSED) {
#pragma unroll
        for (int c = 0; c < C; ++c)
          if (okc[c]) xd[c].load(X + (size_t)row * ld + colc[c]);
      }
    }
#pragma unroll
    for (int c = 0; c < C; ++c)
      if (okc[c] && rm.eg == 0) {
        V16<XT> out;
        const A* sce = scs + colc[c];
        if (sx) {
          V16<XT> xs;
          xs.load_nt(sx + (size_t)row * ld + colc[c]);  // read once per step
          const U* cfe = scf + colc[c];
#pragma unroll
          for (int e = 0; e < VEC; ++e)
            out.v[e] = XT(fma(-cfe[e], U(xs.v[e]), U(acc[c][e] * sce[e])));
        } else {
#pragma unroll
          for (int e = 0; e < VEC; ++e) out.v[e] = XT(acc[c][e] * sce[e]);
        }
        out.store_nt(W + (size_t)row * ld + colc[c]);
        if constexpr (LDSACC) {
          // the newest window vector is X itself
#pragma unroll
          for (int e = 0; e < VEC; ++e) {
            double& slot = red[red_slot<C, VEC>(rm, c, e)];
            slot = fma(double(xd[c].v[e]), double(out.v[e]), slot);
          }
        } else if constexpr (FUSED) {
#pragma unroll
          for (int v = 0; v < NF; ++v) {
              V16<XT> x;
              if (v == NF - 1)
                x = xd[c];  // the newest window vector is X itself
              else
                x.load(static_cast<const XT*>(fx[v]) + (size_t)row * ld + colc[c]);
#pragma unroll
              for (int e = 0; e < VEC; ++e)
                dacc[v][c][e] = fma(double(x.v[e]), double(out.v[e]), dacc[v][c][e]);
            }
        }
      }
  }
  if constexpr (LDSACC) {
    __syncthreads();
    red_partials<C, VEC>(red, rm, ld, fmult[0], part, (size_t)voff * ld, bk, nbk);
  } else if constexpr (FUSED) {
#pragma unroll
    for (int v = 0; v < NF; ++v)
      block_partials<C, VEC>(dacc[v], red, rm, ld, fmult[v], part, (size_t)(voff + v) * ld, bk, nbk);
  }
}

// One CSR x block product per batch entry: blocks off[r] .. off[r+1]-1 of
// the grid belong to request r (a single product is a batch of one).  Three
// or more chunks per lane take 5 blocks per CU instead of 6 (their gathers
// then fit the registers without spills to scratch).
template <typename VT, typename XT, int C, int NF, bool SPLIT>
__global__ __launch_bounds__(kThreads, (NF == 2 || (sizeof(VT) == 8 && sizeof(XT) < 8))
                                           ? 4
                                           : (C >= 3 ? 5 : 6)) void k_spmm(
    BatchArgs<SpmmDesc> bt) {
  int r = 0;
  while (r + 1 < bt.count && (int)blockIdx.x >= bt.off[r + 1]) ++r;
  const SpmmDesc& q = bt.d[r];
  spmm_body<VT, XT, C, NF, SPLIT>(q.n, q.L, q.lgES, q.rp, q.ci, static_cast<const VT*>(q.va),
                           static_cast<const XT*>(q.X), static_cast<XT*>(q.W), q.ld, q.ncolv, q.xmult,
                           q.opscale, q.fx, q.fmult, q.voff, q.part, (int)blockIdx.x - bt.off[r],
                           bt.off[r + 1] - bt.off[r], q.il, q.ts, static_cast<const XT*>(q.sx), q.smult,
                           q.sd);
}

// ---------------------------------------------------------------------------
// Window inner products not fused into the product: up to NV vectors per
// launch, 4 in any geometry, 8 with one 16-byte chunk per lane (the FP64
// sums of 8 vectors then fit the registers).
// ---------------------------------------------------------------------------
template <typename XT, int C, int NV>
__global__ __launch_bounds__(kThreads) void k_dots(int64_t n, int Lr, const XT* __restrict__ W,
                                                  int ld, int ncolv, VecSet vs, int nv, int voff,
                                                  double* __restrict__ part) {
  constexpr int VEC = V16<XT>::N;
  __shared__ double red[kThreads * VEC * C];
  const RowMap rm = RowMap::lanes(Lr, 0);
  bool okc[C];
  int colc[C];
#pragma unroll
  for (int c = 0; c < C; ++c) {
    const int cv = rm.gl + rm.L * c;
    okc[c] = cv < ncolv;
    colc[c] = cv * VEC;
  }
  double acc[NV][C][VEC];
#pragma unroll
  for (int v = 0; v < NV; ++v)
#pragma unroll
    for (int c = 0; c < C; ++c)
#pragma unroll
      for (int e = 0; e < VEC; ++e) acc[v][c][e] = 0.0;
  const int nn = (int)n;  // n < 2^31
  const int nchunk = (nn + rm.rpi - 1) / rm.rpi;
  for (int j = 0; j * (int)gridDim.x < nchunk; ++j) {
    // a pure stream: consecutive chunks on consecutive blocks (see the update)
    const int ch = j * (int)gridDim.x + (int)blockIdx.x;
    const int row = ch * rm.rpi + rm.rg;
    if (!rm.on || ch >= nchunk || row >= nn) continue;
#pragma unroll
    for (int c = 0; c < C; ++c)
      if (okc[c]) {
        V16<XT> w;
        w.load_nt(W + (size_t)row * ld + colc[c]);
#pragma unroll
        for (int v = 0; v < NV; ++v)
          if (v < nv) {
            V16<XT> x;
            x.load_nt(static_cast<const XT*>(vs.x[v]) + (size_t)row * ld + colc[c]);
#pragma unroll
            for (int e = 0; e < VEC; ++e)
              acc[v][c][e] = fma(double(x.v[e]), double(w.v[e]), acc[v][c][e]);
          }
      }
  }
#pragma unroll
  for (int v = 0; v < NV; ++v)
    if (v < nv)
      block_partials<C, VEC>(acc[v], red, rm, ld, vs.mult[v], part, (size_t)(voff + v) * ld,
                             (int)blockIdx.x, (int)gridDim.x);
}

// ---------------------------------------------------------------------------
// Orthogonalisation update and the new norm: w -= sum_v h_v v_v (nv <= NV
// vectors per launch).  With want_norm the block partials of ||w||^2 go to
// part[0][col][block]; when v1 is given, those of v1^T w to
// part[1][col][block]; with SYM, those of w_in^T w (w_in = W as it was read,
// before the update) to part[2][col][block].  For a symmetric operator J and
// W = J v_t, w_in^T w / ||w|| = (J v_t)^T v_t+1 = v_t^T (J v_t+1): the window
// inner product of v_t with the next product, which the next step then does
// not have to read v_t for.  The coefficients h_v * mult_v live in LDS; with
// dhole > 0 the vectors skip coefficient row voff + dhole - 1 (a vector the
// product already subtracted).
// ---------------------------------------------------------------------------
template <typename XT, int C, int NV, bool V1, bool SYM>
__device__ inline void update_body(int64_t n, int Lr, XT* __restrict__ W, int ld, int ncolv,
                                   const void* const* vx, const double* const* vmult, int nv,
                                   const double* __restrict__ d, int voff, int dhole,
                                   int want_norm, const XT* __restrict__ v1,
                                   const double* __restrict__ v1mult, double* __restrict__ part,
                                   int bk, int nbk) {
  constexpr int VEC = V16<XT>::N;
  // the vector arithmetic: FP64 for FP64 and FP32 storage; FP32 for FP16
  // storage (its 11-bit results leave FP32 rounding far below their own)
  using U = typename std::conditional<std::is_same<XT, _Float16>::value, float, double>::type;
  __shared__ double red[kThreads * VEC * C];
  __shared__ U cf[NV * kMaxLd];
  const RowMap rm = RowMap::lanes(Lr, 0);
  for (int i = threadIdx.x; i < NV * ld; i += kThreads) {
    const int v = i / ld, col = i - v * ld;
    const int dr = voff + v + ((dhole > 0 && v >= dhole - 1) ? 1 : 0);
    cf[i] = U(v < nv ? d[(size_t)dr * ld + col] * (vmult[v] ? vmult[v][col] : 1.0) : 0.0);
  }
  __syncthreads();
  bool okc[C];
  int colc[C];
#pragma unroll
  for (int c = 0; c < C; ++c) {
    const int cv = rm.gl + rm.L * c;
    okc[c] = cv < ncolv;
    colc[c] = cv * VEC;
  }
  // V1: v1^T w (the new vector) and v1^T x_{nv-1} (the newest input vector)
  double nacc[C][VEC], gacc[V1 ? C : 1][VEC], hacc[V1 ? C : 1][VEC], sacc[SYM ? C : 1][VEC];
#pragma unroll
  for (int c = 0; c < C; ++c)
#pragma unroll
    for (int e = 0; e < VEC; ++e) {
      nacc[c][e] = 0.0;
      if constexpr (V1) {
        gacc[c][e] = 0.0;
        hacc[c][e] = 0.0;
      }
      if constexpr (SYM) sacc[c][e] = 0.0;
    }
  const int nn = (int)n;  // n < 2^31
  const int nchunk = (nn + rm.rpi - 1) / rm.rpi;
  for (int j = 0; j * nbk < nchunk; ++j) {
    // a pure stream: consecutive chunks go to consecutive blocks (so the
    // XCDs interleave), which streams faster than the XCD bands the product
    // uses for its neighbour gathers
    const int ch = j * nbk + bk;
    const int row = ch * rm.rpi + rm.rg;
    if (!rm.on || ch >= nchunk || row >= nn) continue;
#pragma unroll
    for (int c = 0; c < C; ++c)
      if (okc[c]) {
        V16<XT> w;
        w.load_nt(W + (size_t)row * ld + colc[c]);  // the product is read once
        U wd[VEC];
#pragma unroll
        for (int e = 0; e < VEC; ++e) wd[e] = U(w.v[e]);
        V16<XT> x1;
        if constexpr (V1) x1.load_nt(v1 + (size_t)row * ld + colc[c]);
#pragma unroll
        for (int v = 0; v < NV; ++v)
          if (v < nv) {
            V16<XT> x;
            // every block is read once per launch and a block is far larger
            // than the caches: streaming loads throughout
            x.load_nt(static_cast<const XT*>(vx[v]) + (size_t)row * ld + colc[c]);
            const U* cfv = cf + v * ld + colc[c];
#pragma unroll
            for (int e = 0; e < VEC; ++e) wd[e] = fma(-cfv[e], U(x.v[e]), wd[e]);
            if constexpr (V1) {
              if (v == nv - 1 && want_norm) {
#pragma unroll
                for (int e = 0; e < VEC; ++e)
                  hacc[c][e] = fma(double(U(x1.v[e])), double(U(x.v[e])), hacc[c][e]);
              }
            }
          }
        V16<XT> o;
#pragma unroll
        for (int e = 0; e < VEC; ++e) o.v[e] = XT(wd[e]);
        o.store_nt(W + (size_t)row * ld + colc[c]);
        if (want_norm) {
          double od[VEC];
#pragma unroll
          for (int e = 0; e < VEC; ++e) od[e] = double(U(o.v[e]));
#pragma unroll
          for (int e = 0; e < VEC; ++e) nacc[c][e] = fma(od[e], od[e], nacc[c][e]);
          if constexpr (SYM) {
#pragma unroll
            for (int e = 0; e < VEC; ++e)
              sacc[c][e] = fma(double(U(w.v[e])), od[e], sacc[c][e]);
          }
          if constexpr (V1) {
#pragma unroll
            for (int e = 0; e < VEC; ++e)
              gacc[c][e] = fma(double(U(x1.v[e])), od[e], gacc[c][e]);
          }
        }
      }
  }
  if (want_norm) {
    block_partials<C, VEC>(nacc, red, rm, ld, nullptr, part, 0, bk, nbk);
    if constexpr (V1) {
      block_partials<C, VEC>(gacc, red, rm, ld, v1mult, part, (size_t)ld, bk, nbk);
      block_partials<C, VEC>(hacc, red, rm, ld, v1mult, part, (size_t)3 * ld, bk, nbk);
    } else {
      for (int i = threadIdx.x; i < ld; i += kThreads) {
        part[((size_t)ld + i) * nbk + bk] = 0.0;
        part[((size_t)3 * ld + i) * nbk + bk] = 0.0;
      }
    }
    if constexpr (SYM) block_partials<C, VEC>(sacc, red, rm, ld, nullptr, part, (size_t)2 * ld, bk, nbk);
  }
}

// One update per batch entry (see k_spmm for the block ranges).  With V1 and
// more than 8 elements per lane its four sets of FP64 column sums do not fit
// 128 registers: 3 waves per SIMD instead of 4, 2 beyond 12 elements and 1
// beyond 24 (no spills to scratch).
template <typename XT, int C, int V1E = C * V16<XT>::N>
constexpr int update_min_blocks(bool v1) {
  return !v1 ? 4 : (V1E > 24 ? 1 : (V1E > 12 ? 2 : (V1E > 8 ? 3 : 4)));
}
template <typename XT, int C, int NV, bool V1, bool SYM>
__global__ __launch_bounds__(kThreads, (update_min_blocks<XT, C>(V1))) void k_update(
    BatchArgs<UpdDesc> bt) {
  int r = 0;
  while (r + 1 < bt.count && (int)blockIdx.x >= bt.off[r + 1]) ++r;
  const UpdDesc& q = bt.d[r];
  update_body<XT, C, NV, V1, SYM>(q.n, q.L, static_cast<XT*>(q.W), q.ld, q.ncolv, q.vx, q.vmult,
                                  q.nv, q.d, q.voff, q.dhole, q.want_norm, static_cast<const XT*>(q.v1),
                                  q.v1mult, q.part, (int)blockIdx.x - bt.off[r],
                                  bt.off[r + 1] - bt.off[r]);
}

// ---------------------------------------------------------------------------
// out[i] = sum_b part[i][b]: one wave per output, lanes take every 64th
// block in order, then a fixed xor-shuffle tree.
// ---------------------------------------------------------------------------
__device__ inline double wave_sum_fixed(double s) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
  return s;
}

__device__ inline double row_sum(const double* __restrict__ p, int nblk, int lane) {
  double s = 0.0;
  // unrolled so that the loads are in flight together; the sum keeps its order
#pragma unroll 8
  for (int b = lane; b < nblk; b += 64) s += p[b];
  return wave_sum_fixed(s);
}

// One wave per output; outputs off[r] .. off[r+1]-1 belong to batch entry r.
__global__ __launch_bounds__(kThreads) void k_reduce(BatchArgs<RedDesc> bt) {
  const int lane = threadIdx.x & 63;
  const int o = blockIdx.x * (kThreads / 64) + (threadIdx.x >> 6);
  if (o >= bt.off[bt.count]) return;
  int r = 0;
  while (r + 1 < bt.count && o >= bt.off[r + 1]) ++r;
  const RedDesc& q = bt.d[r];
  const int i = o - bt.off[r];
  const double s = row_sum(q.part + (size_t)i * q.nblk, q.nblk, lane);
  if (lane == 0) q.out[i] = s;
}

// ---------------------------------------------------------------------------
// Per-probe bookkeeping fused with the reduction of the norm partials.
// flags: bit 0 numeric (NaN/Inf), bit 1 non-positive Ritz value / log,
//        bit 2 breakdown (h < tol), bit 3 eigen-iteration did not converge.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kThreads) void k_start_finish(int B, int ld, const double* __restrict__ part,
                                                          int nblk, double* __restrict__ norm2,
                                                          double* __restrict__ mult0,
                                                          int* __restrict__ active,
                                                          int* __restrict__ meff,
                                                          double* __restrict__ g, int gstride,
                                                          double inv_oscale) {
  const int lane = threadIdx.x & 63;
  const int p = blockIdx.x * (kThreads / 64) + (threadIdx.x >> 6);
  if (p >= ld) return;
  const double s = row_sum(part + (size_t)p * nblk, nblk, lane);
  if (lane != 0) return;
  const double v = (p < B) ? s : 0.0;
  norm2[p] = v;
  meff[p] = 0;
  if (p < B && v > 0.0 && isfinite(v)) {
    mult0[p] = inv_oscale / sqrt(v);  // the block is stored at scale 1 / inv_oscale
    active[p] = 1;
  } else {
    mult0[p] = 0.0;
    active[p] = 0;
  }
  if (g && p < B) g[(size_t)p * gstride] = 1.0;
}

// One wave per probe column; columns off[r] .. off[r+1]-1 belong to batch
// entry r.
__global__ __launch_bounds__(kThreads) void k_step_finish(BatchArgs<FinDesc> bt) {
  const int lane = threadIdx.x & 63;
  const int o = blockIdx.x * (kThreads / 64) + (threadIdx.x >> 6);
  if (o >= bt.off[bt.count]) return;
  int r = 0;
  while (r + 1 < bt.count && o >= bt.off[r + 1]) ++r;
  const FinDesc& q = bt.d[r];
  const int p = o - bt.off[r];
  const int B = q.B, ld = q.ld, t = q.t, m = q.m, j0 = q.j0, nv = q.nv, nblk = q.nblk;
  const int sym_row = q.sym_row;
  const double tol = q.tol;
  double* __restrict__ d = q.d;
  const double* __restrict__ part = q.part;
  double* __restrict__ H = q.H;
  int* __restrict__ meff = q.meff;
  int* __restrict__ active = q.active;
  double* __restrict__ mult_next = q.mult_next;
  double* __restrict__ g = q.g;
  int* __restrict__ flags = q.flags;
  const double nrm2 = row_sum(part + (size_t)p * nblk, nblk, lane);
  const double gdot = g ? row_sum(part + (size_t)(ld + p) * nblk, nblk, lane) : 0.0;
  const double gin = (g && q.gin_mult) ? row_sum(part + (size_t)(3 * ld + p) * nblk, nblk, lane) : 0.0;
  const double sdot = sym_row >= 0 ? row_sum(part + (size_t)(2 * ld + p) * nblk, nblk, lane) : 0.0;
  if (lane != 0) return;
  // the window inner products of this step are read below before d[sym_row]
  // (a row of the same array, for the next step) is written
  double* dsym = sym_row >= 0 ? d + (size_t)sym_row * ld + p : nullptr;
  if (p >= B || !active[p]) {
    mult_next[p] = 0.0;
    if (dsym) *dsym = 0.0;
    return;
  }
  // v1^T v_t of this step's input vector (needed even if the step breaks down)
  if (g && q.gin_mult) g[(size_t)p * (m + 1) + t] = gin * q.gin_mult[p];
  double* Hp = H + (size_t)p * (m + 1) * m;
  bool finite = true;
  // the product output, and with it every window inner product and the new
  // vector, is stored at the scale 1 / inv_s (a power of two)
  for (int v = 0; v < nv; ++v) {
    const double h = d[(size_t)v * ld + p] * q.inv_s;
    finite = finite && isfinite(h);
    Hp[(size_t)(j0 + v) * m + t] = h;
  }
  const double nrm = sqrt(nrm2);  // norm of the stored new vector
  const double beta = nrm * q.inv_s;
  Hp[(size_t)(t + 1) * m + t] = beta;
  meff[p] = t + 1;
  if (!finite || !isfinite(beta)) {
    flags[p] |= 1;
    active[p] = 0;
    mult_next[p] = 0.0;
    if (dsym) *dsym = 0.0;
    return;
  }
  if (!(beta >= tol)) {
    flags[p] |= 4;
    active[p] = 0;
    mult_next[p] = 0.0;
    if (dsym) *dsym = 0.0;
    return;
  }
  if (g) g[(size_t)p * (m + 1) + t + 1] = gdot / nrm;
  if (dsym) *dsym = sdot / nrm;
  mult_next[p] = 1.0 / nrm;
}

// ---------------------------------------------------------------------------
// Gauss quadrature of log per probe (Golub-Welsch on T = tridiag(h)).
// One thread per probe; the d/e/z work arrays are [m][B] so that consecutive
// threads touch consecutive addresses.
// ---------------------------------------------------------------------------
__global__ void k_gauss_log(int B, int m, int pb, const double* __restrict__ H,
                            const int* __restrict__ meff, double* __restrict__ K,
                            int* __restrict__ flags, const int* __restrict__ need) {
  extern __shared__ double sm[];
  const int pl = threadIdx.x;
  const int p = blockIdx.x * pb + pl;
  if (pl >= pb || p >= B) return;
  if (need && !need[p]) return;
  const int nn = meff[p];
  if (nn <= 0) {
    K[p] = 0.0;
    return;
  }
  // per-thread arrays in LDS, element i of thread pl at [i * pb + pl]
  double* dd = sm + pl;
  double* ee = sm + (size_t)m * pb + pl;
  double* zz = sm + (size_t)2 * m * pb + pl;
  const double* Hp = H + (size_t)p * (m + 1) * m;
  for (int i = 0; i < nn; ++i) dd[(size_t)i * pb] = Hp[(size_t)i * m + i];
  for (int i = 0; i + 1 < nn; ++i) ee[(size_t)i * pb] = Hp[(size_t)(i + 1) * m + i];
  const int rc = tridiag_ql_first_row(nn, dd, ee, zz, pb);
  int bad = 0;
  const double s = gauss_log_sum(nn, dd, zz, pb, &bad);
  if (rc) flags[p] |= 8;
  if (bad) flags[p] |= 2;
  if (!isfinite(s)) flags[p] |= 1;
  K[p] = s;
}

// ---------------------------------------------------------------------------
// Gauss quadrature value K = e1^T log(T) e1 = sum_k tau_k^2 log(theta_k) of
// each run's tridiagonal T (diagonal h_tt, subdiagonal h_t+1,t, its first
// meff rows), from the Stieltjes form of the logarithm,
//   log x = integral over s > 0 of 1/(1+s) - 1/(x+s) ds,
// which for the matrix reads K = integral of 1/(1+s) - e1^T (T + sI)^{-1} e1.
// With s = e^u the integrand is analytic in the strip |Im u| < pi and decays
// exponentially at both ends, so the trapezoidal rule with step 1/2 on
// [log(a) - 40, log(max(b, 1)) + 40] is accurate to rounding when the
// spectrum of T lies in [a, b] (the exponentially convergent trapezoidal
// rule, Trefethen & Weideman, SIAM Review 2014).  e1^T (T + sI)^{-1} e1 is
// 1/d_1 for the pivots of T + sI eliminated from the bottom
// (d_t = alpha_t + s, d_i = alpha_i + s - beta_i^2 / d_{i+1}); the integrand
// is formed as s n / ((1+s) d_1) with n = d_1 - (1+s) computed directly, so
// nothing cancels.  One wave per run, the nodes spread over the lanes, a
// fixed-order reduction.
//
// A run whose T has an eigenvalue outside [a/1000, 1000 b] (Sturm counts) is
// left to the Golub-Welsch kernel (need[p] = 1).  In check mode (the adaptive
// Krylov dimension) only runs that are active and advanced to dimension dim
// are evaluated: K is compared with the previous check's value kprev[p] and
// the run stops (active = 0, mult_next = 0, flag bit 4) once
// |K - kprev| <= rtol |K|; nactive counts the runs still active.
// ---------------------------------------------------------------------------
constexpr int kQuadWaves = 4;      // runs per 256-thread block
constexpr double kQuadStep = 0.5;  // trapezoidal step in u = log s
constexpr double kQuadTail = 40.0; // e^-40: both tails below rounding

__device__ inline int sturm_below(int nn, const double* al, const double* b2, double x) {
  int cnt = 0;
  double q = 1.0;
  for (int i = 0; i < nn; ++i) {
    q = al[i] - x - (i > 0 ? b2[i - 1] / q : 0.0);
    if (q == 0.0) q = -1e-300;
    if (q < 0.0) ++cnt;
  }
  return cnt;
}

__global__ __launch_bounds__(kThreads) void k_quad_log(int B, int m, const double* __restrict__ H,
                                                      const int* __restrict__ meff, double a, double b,
                                                      double* __restrict__ K, int* __restrict__ need,
                                                      int check_dim, int* __restrict__ active,
                                                      double* __restrict__ kprev, double rtol,
                                                      double* __restrict__ mult_next,
                                                      int* __restrict__ flags,
                                                      int* __restrict__ nactive) {
  extern __shared__ double qsm[];
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int p = blockIdx.x * kQuadWaves + w;
  double* al = qsm + (size_t)w * 2 * m;
  double* b2 = al + m;
  if (p >= B) return;
  const bool check = check_dim > 0;
  const int nn = meff[p];
  if (check && (!active[p] || nn != check_dim)) return;
  if (nn <= 0) {
    if (!check && lane == 0) {
      K[p] = 0.0;
      need[p] = 0;
    }
    return;
  }
  const double* Hp = H + (size_t)p * (m + 1) * m;
  for (int i = lane; i < nn; i += 64) {
    al[i] = Hp[(size_t)i * m + i];
    const double be = (i + 1 < nn) ? Hp[(size_t)(i + 1) * m + i] : 0.0;
    b2[i] = be * be;
  }
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  // spectrum inside the trusted interval?
  int outside = 0;
  if (lane == 0) outside = sturm_below(nn, al, b2, a * 1e-3) > 0;
  if (lane == 1) outside = sturm_below(nn, al, b2, b * 1e3) < nn;
  outside = __shfl(outside, 0, 64) | __shfl(outside, 1, 64);
  if (outside) {
    if (!check && lane == 0) need[p] = 1;
    return;  // check mode: this run keeps going
  }
  const double umin = log(a) - kQuadTail;
  const double umax = log(b > 1.0 ? b : 1.0) + kQuadTail;
  const int nodes = (int)ceil((umax - umin) / kQuadStep) + 1;
  double acc = 0.0;
  for (int j = lane; j < nodes; j += 64) {
    const double sv = exp(umin + j * kQuadStep);
    double d = al[nn - 1] + sv;
    for (int i = nn - 2; i >= 1; --i) d = al[i] + sv - b2[i] / d;
    const double num = (al[0] - 1.0) - (nn >= 2 ? b2[0] / d : 0.0);
    const double d1 = (1.0 + sv) + num;
    acc += sv * num / ((1.0 + sv) * d1);
  }
  const double kval = wave_sum_fixed(acc) * kQuadStep;
  if (lane != 0) return;
  if (!check) {
    K[p] = kval;
    need[p] = 0;
    if (!isfinite(kval)) flags[p] |= 1;
    return;
  }
  const double prev = kprev[p];
  kprev[p] = kval;
  if (fabs(kval - prev) <= rtol * fabs(kval)) {  // false for the first check (prev NaN)
    active[p] = 0;
    mult_next[p] = 0.0;
    flags[p] |= 16;
  } else {
    atomicAdd(nactive, 1);
  }
}

// ---------------------------------------------------------------------------
// Host launchers.
// ---------------------------------------------------------------------------
static int pow2_at_least(int x) {
  int p = 1;
  while (p < x) p <<= 1;
  return p;
}

// Rows a 256-thread block holds with L lanes per row (rows never straddle a
// 64-lane wave).
static int rows_per_block(int L) {
  if (L < 1 || L > 64) return 1;
  return (kThreads / 64) * (64 / L);
}

Geom make_geom(int64_t n, int ld, int xbytes) {
  Geom g;
  g.vec = 16 / xbytes;
  g.ncolv = ld / g.vec;
  // FP16 blocks: one chunk per lane (the per-thread column sums of the
  // fused inner products, 8 per chunk, then fit the registers and the
  // block's LDS at full occupancy)
  if (xbytes == 2 && pow2_at_least(g.ncolv) <= 64)
    return make_geom_lc(n, ld, xbytes, pow2_at_least(g.ncolv), 1);
  // lanes per row L (power of two <= 64) and 16-byte chunks per lane C <= 4:
  // least idle lanes, then the fewest chunks per lane (more rows of lanes in
  // flight, fewer registers)
  int bestL = 64, bestC = 1, bestWaste = 1 << 30, bestPref = 1 << 30;
  for (int C = 1; C <= kMaxC; ++C) {
    const int L = pow2_at_least((g.ncolv + C - 1) / C);
    if (L > 64) continue;
    const int waste = L * C - g.ncolv;
    const int pref = C;
    if (waste < bestWaste || (waste == bestWaste && pref < bestPref)) {
      bestL = L;
      bestC = C;
      bestWaste = waste;
      bestPref = pref;
    }
  }
  return make_geom_lc(n, ld, xbytes, bestL, bestC);
}

Geom make_geom_lc(int64_t n, int ld, int xbytes, int L, int C) {
  Geom g;
  g.n = n;
  g.ld = ld;
  g.xbytes = xbytes;
  g.vec = 16 / xbytes;
  g.ncolv = ld / g.vec;
  g.L = L;
  g.C = C;
  g.lgL = 0;
  while (g.lgL < 7 && (1 << g.lgL) < g.L) ++g.lgL;
  const int rpi = rows_per_block(L);
  const int64_t nchunk = (n + rpi - 1) / rpi;
  int64_t nb = nchunk;
  if (nb > kMaxBlocks) nb = kMaxBlocks;
  if (nb < 1) nb = 1;
  g.nblk = (int)nb;
  g.rpb = (int)((n + nb - 1) / nb);  // contiguous partition for the sketch kernels
  return g;
}

static bool geom_ok(const Geom& g);
bool geom_usable(const Geom& g) { return geom_ok(g); }

// Any L <= 64 without an entry split; a power of two with one.
static bool geom_ok(const Geom& g) {
  const bool lanes = (1 << g.lgL) == g.L || g.lges == 0;
  return g.n > 0 && g.ld > 0 && g.ld % 4 == 0 && (g.xbytes == 8 || g.xbytes == 4 || g.xbytes == 2) &&
         g.vec * g.ncolv == g.ld && g.L >= 1 && g.L <= 64 && lanes && g.C >= 1 &&
         g.C <= kMaxC && g.lges >= 0 && g.lges <= g.lgL && g.lges <= 3 &&
         (g.lges == 0 || g.C <= 2) &&
         (g.L >> g.lges) * g.C >= g.ncolv && g.nblk >= 1 && (int64_t)g.nblk * g.rpb >= g.n &&
         g.ts >= 0 && g.ts <= kMaxRowStride &&
         (g.ts == 0 || ((1 << g.lgL) == g.L && g.ts % (64 / g.L) == 0)) &&
         (g.rg == 0 || (g.rg == 1 && g.lges == 0 && g.ts == 0 && g.C <= 2 && g.xbytes >= 4));
}

// Resident 256-thread blocks of a kernel on the whole device (cached).
static int resident_blocks(const void* fn) {
  static std::mutex mu;
  static std::map<const void*, int> cache;
  std::lock_guard<std::mutex> lk(mu);
  auto it = cache.find(fn);
  if (it != cache.end()) return it->second;
  int dev = 0, cus = 0, per_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    cus = 256;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, kThreads, 0) != hipSuccess ||
      per_cu < 1)
    per_cu = 1;
  const int r = std::min(kMaxBlocks, std::max(1, per_cu * cus));
  cache[fn] = r;
  return r;
}

// Grid of a chunk-sweeping kernel: at most one resident wave of blocks, a
// multiple of 8 from 8 blocks up (see chunk_of).
int stream_grid(const Geom& g, const void* fn) {
  const int rpi = rows_per_block(g.L);
  // a row-group product sweeps groups of kRowGroup rows the way the others
  // sweep rows
  const int64_t units = g.rg ? (g.n + kRowGroup - 1) / kRowGroup : g.n;
  const int64_t nchunk = (units + rpi - 1) / rpi;
  int64_t nb = std::min<int64_t>(nchunk, resident_blocks(fn));
  if (nb >= 8) nb &= ~int64_t(7);
  return (int)std::max<int64_t>(1, nb);
}

#define LD_DISPATCH_C(C, ...)                             \
  switch (C) {                                            \
    case 1: { constexpr int CC = 1; __VA_ARGS__; } break; \
    case 2: { constexpr int CC = 2; __VA_ARGS__; } break; \
    case 3: { constexpr int CC = 3; __VA_ARGS__; } break; \
    default: { constexpr int CC = 4; __VA_ARGS__; } break; \
  }

// Block (b, w): Philox blocks (b, pbase + 64 w + j) for j < 64 into LDS, then
// thread rr packs row 256 b + rr's 64 sign bits.
__global__ __launch_bounds__(kThreads) void k_rademacher_mask(uint64_t seed,
                                                             const uint64_t* seed_dev, int64_t n,
                                                             int pbase, int ncols,
                                                             uint64_t* __restrict__ masks, int nw) {
  if (seed_dev) seed = *seed_dev;
  __shared__ uint64_t words[64][4];
  const int64_t r0 = (int64_t)blockIdx.x * 256;
  const int w = blockIdx.y;
  const int nc = min(64, ncols - 64 * w);
  if ((int)threadIdx.x < nc) {
    uint64_t c0 = (uint64_t)blockIdx.x, c1 = (uint64_t)(pbase + 64 * w + (int)threadIdx.x), c2 = 0,
             c3 = 0;
    philox4x64_10(c0, c1, c2, c3, seed, 0ull);
    words[threadIdx.x][0] = c0;
    words[threadIdx.x][1] = c1;
    words[threadIdx.x][2] = c2;
    words[threadIdx.x][3] = c3;
  }
  __syncthreads();
  const int rr = threadIdx.x;
  const int64_t row = r0 + rr;
  if (row >= n) return;
  uint64_t m = 0;
  for (int j = 0; j < nc; ++j) m |= ((words[j][(rr >> 6) & 3] >> (rr & 63)) & 1ull) << j;
  masks[(size_t)row * nw + w] = m;
}

hipError_t launch_rademacher_mask(hipStream_t st, uint64_t seed, int64_t n, int pbase, int ncols,
                                  uint64_t* masks, int nw, const uint64_t* seed_dev) {
  if (n <= 0 || ncols <= 0) return hipSuccess;
  if (!masks || pbase < 0 || nw != (ncols + 63) / 64) return hipErrorInvalidValue;
  static_assert(kThreads == 256, "one thread per row of a 256-row Philox block");
  dim3 grid((unsigned)((n + 255) / 256), (unsigned)nw);
  hipLaunchKernelGGL(k_rademacher_mask, grid, dim3(kThreads), 0, st, seed, seed_dev, n, pbase, ncols,
                     masks, nw);
  return hipGetLastError();
}

// L lanes per row (a power of two), lane l holding columns 2 l and 2 l + 1.
// The row's lanes load L entries at a time (lane q: entry q of the round: its
// column, value and the sign words of that column) and pass them around the
// row by lane shuffles; every lane accumulates the entries in CSR order.
template <typename VT>
__global__ __launch_bounds__(kThreads) void k_spmm_signs(int64_t n, int lgL,
                                                        const int* __restrict__ rp,
                                                        const int* __restrict__ ci,
                                                        const VT* __restrict__ va,
                                                        const uint64_t* __restrict__ masks, int nw,
                                                        int s, double* __restrict__ Y, int ldy,
                                                        double opscale) {
  const int L = 1 << lgL, rpb = kThreads >> lgL;
  const int l = (int)threadIdx.x & (L - 1);
  const int c0 = 2 * l;
  const bool outl = c0 < ldy;  // lanes past the row's columns only load and pass entries
  const int wsel = min(c0 >> 6, nw - 1), sh = c0 & 63;  // padding columns: any valid word
  const bool v0 = c0 < s, v1 = c0 + 1 < s;
  const int64_t nn = n;
  // every lane of the block runs the same number of row rounds (shuffles)
  const int64_t rounds = (nn + (int64_t)gridDim.x * rpb - 1) / ((int64_t)gridDim.x * rpb);
  for (int64_t rr = 0; rr < rounds; ++rr) {
    const int64_t row = (rr * gridDim.x + blockIdx.x) * rpb + ((int)threadIdx.x >> lgL);
    const bool live = row < nn;
    const int kb = live ? rp[row] : 0, ke = live ? rp[row + 1] : 0;
    // the row's longest-lived count decides its rounds; rows of one wave run
    // the wave's maximum (absent entries carry a zero coefficient)
    int cnt = ke - kb;
    for (int d = L; d < 64; d <<= 1) cnt = max(cnt, __shfl_xor(cnt, d, 64));
    double acc0 = 0.0, acc1 = 0.0;
    for (int base = 0; base < cnt; base += L) {
      const int k = kb + base + l;
      const bool have = k < ke;
      const int col = have ? ci[k] : 0;
      const double a = have ? value_as<VT, double>(va[k]) : 0.0;
      uint64_t w0 = 0, w1 = 0;
      if (have) {
        w0 = masks[(size_t)col * nw];
        if (nw > 1) w1 = masks[(size_t)col * nw + 1];
      }
      const int m = min(L, cnt - base);
      for (int q = 0; q < m; ++q) {
        const double aq = __shfl(a, q, L);
        // entry q's sign word for this lane's columns (the owner holds both)
        uint64_t wq = (uint64_t)(uint32_t)__shfl((int)(uint32_t)w0, q, L) |
                      ((uint64_t)(uint32_t)__shfl((int)(uint32_t)(w0 >> 32), q, L) << 32);
        if (nw > 1) {
          const uint64_t wq1 = (uint64_t)(uint32_t)__shfl((int)(uint32_t)w1, q, L) |
                               ((uint64_t)(uint32_t)__shfl((int)(uint32_t)(w1 >> 32), q, L) << 32);
          if (wsel) wq = wq1;
        }
        const bool hq = __shfl((int)have, q, L) != 0;
        if (hq) {
          const double x0 = v0 ? (((wq >> sh) & 1ull) ? -1.0 : 1.0) : 0.0;
          const double x1 = v1 ? (((wq >> (sh + 1)) & 1ull) ? -1.0 : 1.0) : 0.0;
          acc0 = fma(aq, x0, acc0);
          acc1 = fma(aq, x1, acc1);
        }
      }
    }
    if (live && outl) {
      double2 o;
      o.x = acc0 * opscale;
      o.y = acc1 * opscale;
      *reinterpret_cast<double2*>(Y + (size_t)row * ldy + c0) = o;
    }
  }
}

hipError_t launch_spmm_signs(hipStream_t st, int64_t n, const int* rp, const int* ci,
                             const void* va, int vt, const uint64_t* masks, int nw, int s,
                             double* Y, int ldy, double opscale) {
  if (n < 1 || !rp || !ci || !va || !masks || !Y || s < 1 || ldy < s || ldy > 128 || ldy % 2 ||
      nw != (s + 63) / 64 || reinterpret_cast<uintptr_t>(Y) % 16)
    return hipErrorInvalidValue;
  int lgL = 0;
  while ((1 << lgL) < ldy / 2) ++lgL;
  const int rpb = kThreads >> lgL;
  const int64_t nb = std::min<int64_t>((n + rpb - 1) / rpb, 8 * (int64_t)kMaxBlocks);
  if (vt == VT_F64)
    hipLaunchKernelGGL(k_spmm_signs<double>, dim3((unsigned)nb), dim3(kThreads), 0, st, n, lgL, rp,
                       ci, static_cast<const double*>(va), masks, nw, s, Y, ldy, opscale);
  else if (vt == VT_F32)
    hipLaunchKernelGGL(k_spmm_signs<float>, dim3((unsigned)nb), dim3(kThreads), 0, st, n, lgL, rp,
                       ci, static_cast<const float*>(va), masks, nw, s, Y, ldy, opscale);
  else if (vt == VT_BF16)
    hipLaunchKernelGGL(k_spmm_signs<uint16_t>, dim3((unsigned)nb), dim3(kThreads), 0, st, n, lgL,
                       rp, ci, static_cast<const uint16_t*>(va), masks, nw, s, Y, ldy, opscale);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_rademacher(hipStream_t st, uint64_t seed, int64_t n, int pbase, int ncols,
                             int nvalid, void* X, int xbytes, int ld, int col0,
                             const uint64_t* seed_dev) {
  if (n <= 0 || ncols <= 0) return hipSuccess;
  if (!X || col0 < 0 || col0 + ncols > ld || pbase < 0 || nvalid < 0 || nvalid > ncols)
    return hipErrorInvalidValue;
  dim3 grid((unsigned)((n + 255) / 256), (unsigned)((ncols + 63) / 64));
  if (xbytes == 8)
    hipLaunchKernelGGL(k_rademacher<double>, grid, dim3(kThreads), 0, st, seed, seed_dev, n, pbase,
                       ncols, nvalid, static_cast<double*>(X), ld, col0);
  else if (xbytes == 4)
    hipLaunchKernelGGL(k_rademacher<float>, grid, dim3(kThreads), 0, st, seed, seed_dev, n, pbase,
                       ncols, nvalid, static_cast<float*>(X), ld, col0);
  else if (xbytes == 2)
    hipLaunchKernelGGL(k_rademacher<_Float16>, grid, dim3(kThreads), 0, st, seed, seed_dev, n, pbase,
                       ncols, nvalid, static_cast<_Float16*>(X), ld, col0);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_probes(hipStream_t st, int dist, uint64_t seed, int64_t n, int pbase, int ncols,
                         int nvalid, void* X, int xbytes, int ld, int col0,
                         const uint64_t* seed_dev) {
  if (dist == PROBE_RADEMACHER)
    return launch_rademacher(st, seed, n, pbase, ncols, nvalid, X, xbytes, ld, col0, seed_dev);
  if (dist != PROBE_GAUSSIAN) return hipErrorInvalidValue;
  if (n <= 0 || ncols <= 0) return hipSuccess;
  if (!X || col0 < 0 || col0 + ncols > ld || pbase < 0 || nvalid < 0 || nvalid > ncols)
    return hipErrorInvalidValue;
  const int64_t nb4 = (n + 3) / 4;
  dim3 grid((unsigned)((nb4 + kThreads / 64 - 1) / (kThreads / 64)), (unsigned)((ncols + 63) / 64));
  if (xbytes == 8)
    hipLaunchKernelGGL(k_gaussian<double>, grid, dim3(kThreads), 0, st, seed, seed_dev, n, pbase,
                       ncols, nvalid, static_cast<double*>(X), ld, col0);
  else if (xbytes == 4)
    hipLaunchKernelGGL(k_gaussian<float>, grid, dim3(kThreads), 0, st, seed, seed_dev, n, pbase,
                       ncols, nvalid, static_cast<float*>(X), ld, col0);
  else if (xbytes == 2)
    hipLaunchKernelGGL(k_gaussian<_Float16>, grid, dim3(kThreads), 0, st, seed, seed_dev, n, pbase,
                       ncols, nvalid, static_cast<_Float16*>(X), ld, col0);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Batched launches.  Every per-step launcher takes a list of items (a single
// request is a list of one); items that need the same kernel instantiation
// share one launch of at most kMaxBatch entries, each entry keeping the grid
// it would get alone (so a request's partial sums, and therefore its result,
// do not depend on what it is batched with).
// ---------------------------------------------------------------------------
template <typename Item, typename KeyFn, typename LaunchFn>
static hipError_t launch_grouped(Item* items, int count, KeyFn key, LaunchFn launch) {
  std::vector<char> used((size_t)count, 0);
  for (int a = 0; a < count; ++a) {
    if (used[a]) continue;
    const uint64_t k = key(items[a]);
    int idx[kMaxBatch];
    int cnt = 0;
    for (int b = a; b < count && cnt < kMaxBatch; ++b)
      if (!used[b] && key(items[b]) == k) {
        idx[cnt++] = b;
        used[b] = 1;
      }
    const hipError_t e = launch(idx, cnt);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

static bool spmm_item_ok(const SpmmItem& it) {
  const Geom& g = it.g;
  if (!geom_ok(g) || g.ld > kMaxLd || !it.rp || !it.ci || !it.va || !it.X || !it.W ||
      it.X == it.W || it.nf < 0 || it.nf > 2 || (it.nf > 0 && (!it.part || it.voff < 0)))
    return false;
  if (!(it.vt == VT_F64 || it.vt == VT_F32 || it.vt == VT_BF16)) return false;
  if (g.xbytes == 8 && it.vt != VT_F64 && it.vt != VT_F32 && it.vt != VT_BF16) return false;
  for (int v = 0; v < it.nf; ++v)
    if (!it.fused.x[v] || it.fused.x[v] == it.W) return false;
  if (it.nf > 0 && it.fused.x[it.nf - 1] != it.X) return false;  // newest vector = the input
  if (it.sx && (!it.sd || it.sx == it.W || it.sx == it.X)) return false;
  if (g.rg && (!it.rg.gp || !it.rg.col ||
               !(it.vt == VT_F32 ? (it.rg.val && g.xbytes == 4)
                                 : (it.vt == VT_F64 && it.rg.val64))))
    return false;
  return true;
}

template <typename VT, typename XT, int C, int NF, bool SPLIT>
static hipError_t spmm_launch(hipStream_t st, SpmmItem* items, const int* idx, int cnt) {
  auto fn = k_spmm<VT, XT, C, NF, SPLIT>;
  BatchArgs<SpmmDesc> bt{};
  bt.count = cnt;
  int off = 0;
  for (int q = 0; q < cnt; ++q) {
    SpmmItem& it = items[idx[q]];
    const int nb = stream_grid(it.g, (const void*)fn);
    it.nblk = nb;
    SpmmDesc& d = bt.d[q];
    d.n = it.g.n;
    d.rp = it.rp;
    d.ci = it.ci;
    d.va = it.va;
    d.X = it.X;
    d.W = it.W;
    d.xmult = it.xmult;
    d.opscale = it.opscale;
    for (int v = 0; v < 2; ++v) {
      d.fx[v] = v < it.nf ? it.fused.x[v] : nullptr;
      d.fmult[v] = v < it.nf ? it.fused.mult[v] : nullptr;
    }
    d.part = it.part;
    d.L = it.g.L;
    d.lgES = it.g.lges;
    d.ld = it.g.ld;
    d.ncolv = it.g.ncolv;
    d.voff = it.voff;
    d.il = it.g.xil;
    d.ts = it.g.ts;
    d.sx = it.sx;
    d.smult = it.smult;
    d.sd = it.sd;
    bt.off[q] = off;
    off += nb;
  }
  bt.off[cnt] = off;
  hipLaunchKernelGGL(fn, dim3(off), dim3(kThreads), 0, st, bt);
  return hipGetLastError();
}

template <typename VT, typename XT, int NF>
static hipError_t spmm_launch_c(hipStream_t st, int C, SpmmItem* items, const int* idx, int cnt) {
  hipError_t e = hipErrorInvalidValue;
  if (items[idx[0]].g.lges > 0) {
    // entry-split instantiations: one or two chunks per lane
    if (C == 1) return spmm_launch<VT, XT, 1, NF, true>(st, items, idx, cnt);
    if (C == 2) return spmm_launch<VT, XT, 2, NF, true>(st, items, idx, cnt);
    return hipErrorInvalidValue;
  }
  LD_DISPATCH_C(C, { e = spmm_launch<VT, XT, CC, NF, false>(st, items, idx, cnt); });
  return e;
}

template <typename VT, typename XT>
static hipError_t spmm_launch_typed(hipStream_t st, int C, int nf, SpmmItem* items, const int* idx,
                                    int cnt) {
  if (nf == 2) return spmm_launch_c<VT, XT, 2>(st, C, items, idx, cnt);
  if (nf == 1) return spmm_launch_c<VT, XT, 1>(st, C, items, idx, cnt);
  return spmm_launch_c<VT, XT, 0>(st, C, items, idx, cnt);
}

hipError_t launch_spmm_batch(hipStream_t st, SpmmItem* items, int count) {
  if (count < 0 || (count > 0 && !items)) return hipErrorInvalidValue;
  for (int a = 0; a < count; ++a)
    if (!spmm_item_ok(items[a])) return hipErrorInvalidValue;
  auto key = [](const SpmmItem& it) -> uint64_t {
    return (uint64_t)it.g.xbytes | ((uint64_t)it.vt << 8) | ((uint64_t)it.g.C << 16) |
           ((uint64_t)it.nf << 24) | ((uint64_t)(it.g.lges > 0) << 32) |
           ((uint64_t)it.g.rg << 33);
  };
  return launch_grouped(items, count, key, [&](const int* idx, int cnt) -> hipError_t {
    const SpmmItem& it = items[idx[0]];
    if (it.g.rg) return launch_spmm_rg_group(st, items, idx, cnt);
    if (it.g.xbytes == 8) {
      if (it.vt == VT_F64) return spmm_launch_typed<double, double>(st, it.g.C, it.nf, items, idx, cnt);
      if (it.vt == VT_F32) return spmm_launch_typed<float, double>(st, it.g.C, it.nf, items, idx, cnt);
      return spmm_launch_typed<uint16_t, double>(st, it.g.C, it.nf, items, idx, cnt);
    }
    if (it.g.xbytes == 2) {
      if (it.vt == VT_F64)
        return spmm_launch_typed<double, _Float16>(st, it.g.C, it.nf, items, idx, cnt);
      if (it.vt == VT_F32)
        return spmm_launch_typed<float, _Float16>(st, it.g.C, it.nf, items, idx, cnt);
      return spmm_launch_typed<uint16_t, _Float16>(st, it.g.C, it.nf, items, idx, cnt);
    }
    if (it.vt == VT_F64) return spmm_launch_typed<double, float>(st, it.g.C, it.nf, items, idx, cnt);
    if (it.vt == VT_F32) return spmm_launch_typed<float, float>(st, it.g.C, it.nf, items, idx, cnt);
    return spmm_launch_typed<uint16_t, float>(st, it.g.C, it.nf, items, idx, cnt);
  });
}

hipError_t launch_spmm(hipStream_t st, const Geom& g, const int* rp, const int* ci, const void* va,
                       int vt, const void* X, void* W, const double* xmult, double opscale,
                       const VecSet* fused, int nf, int voff, double* part, int* nblk_out,
                       const void* sx, const double* smult, const double* sd,
                       const RowGroups* rg) {
  SpmmItem it{};
  if (rg) it.rg = *rg;
  it.g = g;
  it.rp = rp;
  it.ci = ci;
  it.va = va;
  it.vt = vt;
  it.X = X;
  it.W = W;
  it.xmult = xmult;
  it.opscale = opscale;
  if (nf > 0) {
    if (!fused) return hipErrorInvalidValue;
    it.fused = *fused;
  }
  it.nf = nf;
  it.voff = voff;
  it.part = part;
  it.sx = sx;
  it.smult = smult;
  it.sd = sd;
  const hipError_t e = launch_spmm_batch(st, &it, 1);
  if (nblk_out) *nblk_out = it.nblk;
  return e;
}

hipError_t launch_dots(hipStream_t st, const Geom& g, const void* W, const VecSet& vs, int nv,
                       int voff, double* part, int* nblk_out) {
  int dummy = 0;
  if (!nblk_out) nblk_out = &dummy;
  if (!geom_ok(g) || g.lges != 0 || g.ts != 0 || g.rg != 0 || !W || !part || nv < 1 || nv > kDotsWide ||
      voff < 0)
    return hipErrorInvalidValue;
  for (int v = 0; v < nv; ++v)
    if (!vs.x[v]) return hipErrorInvalidValue;
  if (nv > kDotsPerLaunch) {
    // the wide launch: one chunk per lane (FP32 or FP64 vectors)
    if (g.xbytes == 4 && g.C == 1) {
      auto fn = k_dots<float, 1, kDotsWide>;
      const int nb = stream_grid(g, (const void*)fn);
      *nblk_out = nb;
      hipLaunchKernelGGL(fn, dim3(nb), dim3(kThreads), 0, st, g.n, g.L,
                         static_cast<const float*>(W), g.ld, g.ncolv, vs, nv, voff, part);
    } else if (g.xbytes == 8 && g.C == 1) {
      auto fn = k_dots<double, 1, kDotsWide>;
      const int nb = stream_grid(g, (const void*)fn);
      *nblk_out = nb;
      hipLaunchKernelGGL(fn, dim3(nb), dim3(kThreads), 0, st, g.n, g.L,
                         static_cast<const double*>(W), g.ld, g.ncolv, vs, nv, voff, part);
    } else {
      return hipErrorInvalidValue;
    }
    return hipGetLastError();
  }
  if (g.xbytes == 8) {
    LD_DISPATCH_C(g.C, {
      auto fn = k_dots<double, CC, kDotsPerLaunch>;
      const int nb = stream_grid(g, (const void*)fn);
      *nblk_out = nb;
      hipLaunchKernelGGL(fn, dim3(nb), dim3(kThreads), 0, st, g.n, g.L,
                         static_cast<const double*>(W), g.ld, g.ncolv, vs, nv, voff, part);
    });
  } else if (g.xbytes == 4) {
    LD_DISPATCH_C(g.C, {
      auto fn = k_dots<float, CC, kDotsPerLaunch>;
      const int nb = stream_grid(g, (const void*)fn);
      *nblk_out = nb;
      hipLaunchKernelGGL(fn, dim3(nb), dim3(kThreads), 0, st, g.n, g.L,
                         static_cast<const float*>(W), g.ld, g.ncolv, vs, nv, voff, part);
    });
  } else {
    LD_DISPATCH_C(g.C, {
      auto fn = k_dots<_Float16, CC, kDotsPerLaunch>;
      const int nb = stream_grid(g, (const void*)fn);
      *nblk_out = nb;
      hipLaunchKernelGGL(fn, dim3(nb), dim3(kThreads), 0, st, g.n, g.L,
                         static_cast<const _Float16*>(W), g.ld, g.ncolv, vs, nv, voff, part);
    });
  }
  return hipGetLastError();
}

static bool update_item_ok(const UpdateItem& it) {
  const Geom& g = it.g;
  if (!geom_ok(g) || g.lges != 0 || g.ts != 0 || g.rg != 0 || g.ld > kMaxLd || !it.W || !it.d || it.nv < 0 ||
      it.nv > kMaxNv || (it.nv > 4 && g.xbytes == 2) ||
      (it.want_norm && !it.part) || (it.v1 && !it.v1mult) || (it.sym && !it.want_norm) ||
      it.dhole < 0 || it.dhole > it.nv)
    return false;
  for (int v = 0; v < it.nv; ++v)
    if (!it.vs.x[v] || it.vs.x[v] == it.W) return false;
  return true;
}

// update instantiations by window vectors per launch: 1, 2, up to 4, up to
// 8 (FP32 and FP64 vectors; FP16 vectors take windows up to 4)
static int update_nv_class(int nv) { return nv <= 1 ? 1 : (nv == 2 ? 2 : (nv <= 4 ? 4 : 8)); }

template <typename XT, int C, int NV, bool V1, bool SYM>
static hipError_t update_launch(hipStream_t st, UpdateItem* items, const int* idx, int cnt) {
  auto fn = k_update<XT, C, NV, V1, SYM>;
  BatchArgs<UpdDesc> bt{};
  bt.count = cnt;
  int off = 0;
  for (int q = 0; q < cnt; ++q) {
    UpdateItem& it = items[idx[q]];
    const int nb = stream_grid(it.g, (const void*)fn);
    it.nblk = nb;
    UpdDesc& d = bt.d[q];
    d.n = it.g.n;
    d.W = it.W;
    for (int v = 0; v < kMaxNv; ++v) {
      d.vx[v] = v < it.nv ? it.vs.x[v] : nullptr;
      d.vmult[v] = v < it.nv ? it.vs.mult[v] : nullptr;
    }
    d.d = it.d;
    d.v1 = it.v1;
    d.v1mult = it.v1mult;
    d.part = it.part;
    d.L = it.g.L;
    d.ld = it.g.ld;
    d.ncolv = it.g.ncolv;
    d.nv = it.nv;
    d.voff = it.voff;
    d.dhole = it.dhole;
    d.want_norm = it.want_norm;
    bt.off[q] = off;
    off += nb;
  }
  bt.off[cnt] = off;
  hipLaunchKernelGGL(fn, dim3(off), dim3(kThreads), 0, st, bt);
  return hipGetLastError();
}

template <typename XT, int NV, bool V1, bool SYM>
static hipError_t update_launch_c(hipStream_t st, int C, UpdateItem* items, const int* idx,
                                  int cnt) {
  hipError_t e = hipErrorInvalidValue;
  LD_DISPATCH_C(C, { e = update_launch<XT, CC, NV, V1, SYM>(st, items, idx, cnt); });
  return e;
}

template <typename XT, int NV>
static hipError_t update_launch_flags(hipStream_t st, int C, bool v1, bool sym, UpdateItem* items,
                                      const int* idx, int cnt) {
  if (v1)
    return sym ? update_launch_c<XT, NV, true, true>(st, C, items, idx, cnt)
               : update_launch_c<XT, NV, true, false>(st, C, items, idx, cnt);
  return sym ? update_launch_c<XT, NV, false, true>(st, C, items, idx, cnt)
             : update_launch_c<XT, NV, false, false>(st, C, items, idx, cnt);
}

template <typename XT>
static hipError_t update_launch_typed(hipStream_t st, const UpdateItem& it, UpdateItem* items,
                                      const int* idx, int cnt) {
  const bool v1 = it.v1 != nullptr;
  switch (update_nv_class(it.nv)) {
    case 1: return update_launch_flags<XT, 1>(st, it.g.C, v1, it.sym, items, idx, cnt);
    case 2: return update_launch_flags<XT, 2>(st, it.g.C, v1, it.sym, items, idx, cnt);
    case 4: return update_launch_flags<XT, 4>(st, it.g.C, v1, it.sym, items, idx, cnt);
    default:
      if constexpr (sizeof(XT) == 2) return hipErrorInvalidValue;
      else return update_launch_flags<XT, 8>(st, it.g.C, v1, it.sym, items, idx, cnt);
  }
}

hipError_t launch_update_batch(hipStream_t st, UpdateItem* items, int count) {
  if (count < 0 || (count > 0 && !items)) return hipErrorInvalidValue;
  for (int a = 0; a < count; ++a)
    if (!update_item_ok(items[a])) return hipErrorInvalidValue;
  auto key = [](const UpdateItem& it) -> uint64_t {
    return (uint64_t)it.g.xbytes | ((uint64_t)it.g.C << 8) |
           ((uint64_t)update_nv_class(it.nv) << 16) | ((uint64_t)(it.v1 != nullptr) << 24) |
           ((uint64_t)it.sym << 25);
  };
  return launch_grouped(items, count, key, [&](const int* idx, int cnt) -> hipError_t {
    const UpdateItem& it = items[idx[0]];
    if (it.g.xbytes == 8) return update_launch_typed<double>(st, it, items, idx, cnt);
    if (it.g.xbytes == 4) return update_launch_typed<float>(st, it, items, idx, cnt);
    return update_launch_typed<_Float16>(st, it, items, idx, cnt);
  });
}

hipError_t launch_update(hipStream_t st, const Geom& g, void* W, const VecSet& vs, int nv,
                         const double* d, int voff, int want_norm, const void* v1,
                         const double* v1mult, bool sym, double* part, int* nblk_out,
                         int dhole) {
  UpdateItem it{};
  it.g = g;
  it.W = W;
  it.vs = vs;
  it.nv = nv;
  it.d = d;
  it.voff = voff;
  it.want_norm = want_norm;
  it.v1 = v1;
  it.v1mult = v1mult;
  it.sym = sym;
  it.part = part;
  it.dhole = dhole;
  const hipError_t e = launch_update_batch(st, &it, 1);
  if (nblk_out) *nblk_out = it.nblk;
  return e;
}

hipError_t launch_reduce_batch(hipStream_t st, const ReduceItem* items, int count) {
  if (count < 0 || (count > 0 && !items)) return hipErrorInvalidValue;
  for (int a = 0; a < count; ++a)
    if (!items[a].part || !items[a].out || items[a].nblk < 1 || items[a].width < 1)
      return hipErrorInvalidValue;
  for (int a0 = 0; a0 < count; a0 += kMaxBatch) {
    const int cnt = std::min(kMaxBatch, count - a0);
    BatchArgs<RedDesc> bt{};
    bt.count = cnt;
    int off = 0;
    for (int q = 0; q < cnt; ++q) {
      const ReduceItem& it = items[a0 + q];
      bt.d[q] = RedDesc{it.part, it.out, it.nblk, it.width};
      bt.off[q] = off;
      off += it.width;
    }
    bt.off[cnt] = off;
    hipLaunchKernelGGL(k_reduce, dim3((off + 3) / 4), dim3(kThreads), 0, st, bt);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_reduce(hipStream_t st, const double* part, int nblk, int width, double* out) {
  const ReduceItem it{part, nblk, width, out};
  return launch_reduce_batch(st, &it, 1);
}

hipError_t launch_start_finish(hipStream_t st, int B, int ld, const double* part, int nblk,
                               double* norm2, double* mult0, int* active, int* meff, double* g,
                               int gstride, double inv_oscale) {
  if (B < 1 || ld < B || !part || nblk < 1 || !(inv_oscale > 0.0)) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_start_finish, dim3((ld + 3) / 4), dim3(kThreads), 0, st, B, ld, part, nblk,
                     norm2, mult0, active, meff, g, gstride, inv_oscale);
  return hipGetLastError();
}

hipError_t launch_step_finish_batch(hipStream_t st, const FinishItem* items, int count) {
  if (count < 0 || (count > 0 && !items)) return hipErrorInvalidValue;
  for (int a = 0; a < count; ++a) {
    const FinishItem& it = items[a];
    // the next step has at most nv + 1 window vectors: its second newest sits
    // at row <= nv - 1 of d
    if (it.B < 1 || it.ld < it.B || it.t < 0 || it.t >= it.m || it.j0 < 0 ||
        it.j0 + it.nv != it.t + 1 || !it.part || it.nblk < 1 || it.sym_row >= it.nv ||
        (it.sym_row >= 0 && it.t + 1 >= it.m))
      return hipErrorInvalidValue;
  }
  for (int a0 = 0; a0 < count; a0 += kMaxBatch) {
    const int cnt = std::min(kMaxBatch, count - a0);
    BatchArgs<FinDesc> bt{};
    bt.count = cnt;
    int off = 0;
    for (int q = 0; q < cnt; ++q) {
      const FinishItem& it = items[a0 + q];
      FinDesc& d = bt.d[q];
      d.d = it.d;
      d.part = it.part;
      d.H = it.H;
      d.meff = it.meff;
      d.active = it.active;
      d.mult_next = it.mult_next;
      d.g = it.g;
      d.flags = it.flags;
      d.gin_mult = it.gin_mult;
      d.tol = it.tol;
      d.B = it.B;
      d.ld = it.ld;
      d.t = it.t;
      d.m = it.m;
      d.j0 = it.j0;
      d.nv = it.nv;
      d.nblk = it.nblk;
      d.sym_row = it.sym_row < 0 ? -1 : it.sym_row;
      d.inv_s = it.inv_s;
      bt.off[q] = off;
      off += it.ld;
    }
    bt.off[cnt] = off;
    hipLaunchKernelGGL(k_step_finish, dim3((off + 3) / 4), dim3(kThreads), 0, st, bt);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_step_finish(hipStream_t st, int B, int ld, int t, int m, double* d, int j0,
                              int nv, const double* part, int nblk, double tol, double* H,
                              int* meff, int* active, double* mult_next, double* g, int* flags,
                              int sym_row, double inv_s, const double* gin_mult) {
  const FinishItem it{B,     ld,   t,    m,      d,         j0, nv,    part,    nblk,
                      tol,   H,    meff, active, mult_next, g,  flags, sym_row, inv_s, gin_mult};
  return launch_step_finish_batch(st, &it, 1);
}

hipError_t launch_gauss_log(hipStream_t st, int B, int m, const double* H, const int* meff,
                            double* K, int* flags, const int* need) {
  if (B < 1 || m < 1 || m > 1024) return hipErrorInvalidValue;
  // one probe per wave: the implicit QL sweeps of different probes converge
  // differently, and lanes of one wave would serialise on each other's paths
  int pb = 1;
  const size_t lds = (size_t)3 * m * pb * sizeof(double);
  hipLaunchKernelGGL(k_gauss_log, dim3((B + pb - 1) / pb), dim3(64), lds, st, B, m, pb, H, meff, K,
                     flags, need);
  return hipGetLastError();
}

hipError_t launch_quad_log(hipStream_t st, int B, int m, const double* H, const int* meff, double a,
                           double b, double* K, int* need, int* flags) {
  if (B < 1 || m < 1 || m > 1024 || !(a > 0.0) || !(b >= a) || !H || !meff || !K || !need ||
      !flags)
    return hipErrorInvalidValue;
  const size_t lds = (size_t)kQuadWaves * 2 * m * sizeof(double);
  hipLaunchKernelGGL(k_quad_log, dim3((B + kQuadWaves - 1) / kQuadWaves), dim3(kThreads), lds, st, B,
                     m, H, meff, a, b, K, need, 0, nullptr, nullptr, 0.0, nullptr, flags, nullptr);
  return hipGetLastError();
}

hipError_t launch_quad_check(hipStream_t st, int B, int m, const double* H, const int* meff,
                             double a, double b, int dim, int* active, double* kprev, double rtol,
                             double* mult_next, int* flags, int* nactive) {
  if (B < 1 || m < 1 || m > 1024 || dim < 1 || dim > m || !(a > 0.0) || !(b >= a) || !H ||
      !meff || !active || !kprev || !mult_next || !flags || !nactive)
    return hipErrorInvalidValue;
  const size_t lds = (size_t)kQuadWaves * 2 * m * sizeof(double);
  hipLaunchKernelGGL(k_quad_log, dim3((B + kQuadWaves - 1) / kQuadWaves), dim3(kThreads), lds, st, B,
                     m, H, meff, a, b, nullptr, nullptr, dim, active, kprev, rtol, mult_next, flags,
                     nactive);
  return hipGetLastError();
}

}  // namespace ld
