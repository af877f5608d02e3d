// Row-group sparse product W = opscale * (Q X) * diag(xmult), FP32 values on
// FP32 probe blocks or FP64 values on FP64 or FP32 blocks (Alg 1's operator
// application, as in the CSR product of k_stream.hip, over the matrix's row
// groups).
//
// A group is kRowGroup consecutive rows with the sorted union of their
// columns and, per union column, one value per row (zero where the row has
// no entry).  The group's L lanes gather each union column's probe row once
// and multiply it into every row of the group: on covariance-like matrices,
// whose neighbouring rows share most of their columns, the gathers (and the
// bytes the L1 returns to the lanes, which bound that product) drop by the
// ratio of entries to union columns.  A row's sum sees its own nonzero terms
// in CSR order (a zero value adds an exact zero), so W is the CSR product's
// W; the epilogue (scaling, early subtraction, store, fused inner products)
// is the CSR product's, per row.
#include <climits>
#include <type_traits>

#include "ld_kernels.h"

namespace ld {

struct RgDesc {
  int64_t n;
  const int* gp;
  const int* col;
  const void* val;  // kRowGroup values per union column, in the element type
  const void* X;
  void* W;
  const double* xmult;
  double opscale;
  const void* fx[2];
  const double* fmult[2];
  double* part;
  int L, ld, ncolv, voff, il;
  const void* sx;
  const double* smult;
  const double* sd;
};

// The kRowGroup values of one union column.
template <typename T>
struct Vals4 {
  T v[4];
  __device__ inline void load(const T* p, int u) {
    if constexpr (sizeof(T) == 4) {
      const float4 t = reinterpret_cast<const float4*>(p)[u];
      v[0] = t.x; v[1] = t.y; v[2] = t.z; v[3] = t.w;
    } else {
      const double2 a = reinterpret_cast<const double2*>(p)[2 * u];
      const double2 b = reinterpret_cast<const double2*>(p)[2 * u + 1];
      v[0] = a.x; v[1] = a.y; v[2] = b.x; v[3] = b.y;
    }
  }
  // lane src's values (wave lane index)
  __device__ inline Vals4 from(int src) const {
    Vals4 o;
#pragma unroll
    for (int r = 0; r < 4; ++r) o.v[r] = __shfl(v[r], src);
    return o;
  }
};

// VT: the values' type, T: the probe blocks' (FP32 values on FP32 blocks,
// FP64 on FP64, FP64 on FP32); the sums are in FP64 when either is, else in
// FP32, as in the CSR product of the same types.
template <typename VT, typename T, int C, int NF>
__device__ inline void rg_body(const RgDesc& q, int bk, int nbk) {
  using A = typename std::conditional<sizeof(VT) == 8 || sizeof(T) == 8, double, float>::type;
  constexpr int VEC = V16<T>::N;
  constexpr int G = kRowGroup;
  static_assert(G == 4, "four values per union column");
  constexpr bool FUSED = NF > 0;
  // one fused product: per-thread FP64 sums in the thread's LDS slots; two:
  // in registers (as in the CSR product)
  constexpr bool LDSACC = NF == 1;
  constexpr int ND = (FUSED && !LDSACC) ? NF : 1;
  // union entries whose (column, values) a lane loads per round (four with
  // FP32 values and one chunk per lane: fewer rounds of dependent entry
  // loads per group)
  constexpr int KE = (sizeof(VT) == 4 && C == 1) ? 4 : 2;
  __shared__ double red[FUSED ? kThreads * VEC * C : 1];
  __shared__ A scs[kMaxLd];       // opscale * xmult[col]
  __shared__ double scf[kMaxLd];  // sd[col] * smult[col] (early subtraction)
  const RowMap rm = RowMap::lanes(q.L, 0);
  const int ld = q.ld;
  for (int i = threadIdx.x; i < ld; i += kThreads) {
    scs[i] = A(q.opscale * (q.xmult ? q.xmult[i] : 1.0));
    if (q.sx) scf[i] = q.sd[i] * (q.smult ? q.smult[i] : 1.0);
  }
  bool okc[C];
  int colc[C];
#pragma unroll
  for (int c = 0; c < C; ++c) {
    const int cv = rm.cl + rm.Lc * c;
    okc[c] = cv < q.ncolv;
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
  const int nn = (int)q.n;  // n < 2^31
  const int ng = (nn + G - 1) / G;
  const int nchunk = (ng + rm.rpi - 1) / rm.rpi;
  const VT* vals = static_cast<const VT*>(q.val);
  const T* X = static_cast<const T*>(q.X);
  T* W = static_cast<T*>(q.W);
  const T* sx = static_cast<const T*>(q.sx);
  for (int j = 0; j * nbk < nchunk; ++j) {
    const int ch = q.il ? j * nbk + bk : chunk_of(j, bk, nbk);
    const int grp = ch * rm.rpi + rm.rg;
    if (!rm.on || ch >= nchunk || grp >= ng) continue;
    const int r0 = grp * G;
    A acc[G][C][VEC];
#pragma unroll
    for (int r = 0; r < G; ++r)
#pragma unroll
      for (int c = 0; c < C; ++c)
#pragma unroll
        for (int e = 0; e < VEC; ++e) acc[r][c][e] = A(0);
    // one union column into the group's rows
    auto add = [&](const V16<T> (&x)[C], const Vals4<VT>& a) {
#pragma unroll
      for (int c = 0; c < C; ++c)
        if (okc[c]) {
#pragma unroll
          for (int e = 0; e < VEC; ++e)
#pragma unroll
            for (int r = 0; r < G; ++r)
              acc[r][c][e] = fma(A(a.v[r]), A(x[c].v[e]), acc[r][c][e]);
        }
    };
    const int ub = q.gp[grp], ue = q.gp[grp + 1];
    // the group's L lanes load KE * L consecutive union entries per round,
    // lane l holding entries l, l + L, ..., and pass them around the group
    // by lane shuffles; two entries' gathers in flight, in union order
    for (int base = ub; base < ue; base += rm.L * KE) {
      int myc[KE];
      Vals4<VT> myv[KE];
#pragma unroll
      for (int u = 0; u < KE; ++u) {
        const int kk = base + rm.gl + rm.L * u;
        myc[u] = r0;
#pragma unroll
        for (int r = 0; r < G; ++r) myv[u].v[r] = VT(0);
        if (kk < ue) {
          myc[u] = q.col[kk];
          myv[u].load(vals, kk);
        }
      }
#pragma unroll
      for (int u = 0; u < KE; ++u) {
        const int cnt = min(rm.L, ue - base - rm.L * u);
        if (cnt <= 0) break;
        int e = 0;
        for (; e + 2 <= cnt; e += 2) {
          const int c0 = __shfl(myc[u], rm.lb + e), c1 = __shfl(myc[u], rm.lb + e + 1);
          const Vals4<VT> a0 = myv[u].from(rm.lb + e), a1 = myv[u].from(rm.lb + e + 1);
          V16<T> x0[C], x1[C];
#pragma unroll
          for (int c = 0; c < C; ++c)
            if (okc[c]) {
              x0[c].load(X + (size_t)c0 * ld + colc[c]);
              x1[c].load(X + (size_t)c1 * ld + colc[c]);
            }
          add(x0, a0);
          add(x1, a1);
        }
        if (e < cnt) {
          const int c0 = __shfl(myc[u], rm.lb + e);
          const Vals4<VT> a0 = myv[u].from(rm.lb + e);
          V16<T> x0[C];
#pragma unroll
          for (int c = 0; c < C; ++c)
            if (okc[c]) x0[c].load(X + (size_t)c0 * ld + colc[c]);
          add(x0, a0);
        }
      }
    }
#pragma unroll
    for (int r = 0; r < G; ++r) {
      const int row = r0 + r;
      if (row >= nn) break;
#pragma unroll
      for (int c = 0; c < C; ++c)
        if (okc[c]) {
          V16<T> out;
          const A* sce = scs + colc[c];
          if (sx) {
            V16<T> xs;
            xs.load_nt(sx + (size_t)row * ld + colc[c]);  // read once per step
            const double* cfe = scf + colc[c];
#pragma unroll
            for (int e = 0; e < VEC; ++e)
              out.v[e] = T(fma(-cfe[e], double(xs.v[e]), double(acc[r][c][e] * sce[e])));
          } else {
#pragma unroll
            for (int e = 0; e < VEC; ++e) out.v[e] = T(acc[r][c][e] * sce[e]);
          }
          out.store_nt(W + (size_t)row * ld + colc[c]);
          if constexpr (FUSED) {
            // the newest window vector is X itself: the row's value is read
            // again (the group's gathers do not keep it)
            V16<T> xd;
            xd.load(X + (size_t)row * ld + colc[c]);
            if constexpr (LDSACC) {
#pragma unroll
              for (int e = 0; e < VEC; ++e) {
                double& slot = red[red_slot<C, VEC>(rm, c, e)];
                slot = fma(double(xd.v[e]), double(out.v[e]), slot);
              }
            } else {
#pragma unroll
              for (int v = 0; v < NF; ++v) {
                V16<T> x;
                if (v == NF - 1)
                  x = xd;
                else
                  x.load(static_cast<const T*>(q.fx[v]) + (size_t)row * ld + colc[c]);
#pragma unroll
                for (int e = 0; e < VEC; ++e)
                  dacc[v][c][e] = fma(double(x.v[e]), double(out.v[e]), dacc[v][c][e]);
              }
            }
          }
        }
    }
  }
  if constexpr (LDSACC) {
    __syncthreads();
    red_partials<C, VEC>(red, rm, ld, q.fmult[0], q.part, (size_t)q.voff * ld, bk, nbk);
  } else if constexpr (FUSED) {
#pragma unroll
    for (int v = 0; v < NF; ++v)
      block_partials<C, VEC>(dacc[v], red, rm, ld, q.fmult[v], q.part, (size_t)(q.voff + v) * ld,
                             bk, nbk);
  }
}

// blocks per CU at which every instance fits its registers without spills
template <typename VT, typename T, int C, int NF>
constexpr int rg_min_blocks() {
  // FP64 values on FP32 blocks keep FP64 sums of 4 elements per chunk
  if (sizeof(VT) == 8 && sizeof(T) == 4 && C == 2) return NF == 2 ? 2 : 3;
  return (C == 1 && sizeof(VT) == 4 && sizeof(T) == 4) ? (NF == 2 ? 4 : 5) : (NF == 2 ? 3 : 4);
}

template <typename VT, typename T, int C, int NF>
__global__ __launch_bounds__(kThreads, (rg_min_blocks<VT, T, C, NF>())) void k_spmm_rg(
    BatchArgs<RgDesc> bt) {
  int r = 0;
  while (r + 1 < bt.count && (int)blockIdx.x >= bt.off[r + 1]) ++r;
  rg_body<VT, T, C, NF>(bt.d[r], (int)blockIdx.x - bt.off[r], bt.off[r + 1] - bt.off[r]);
}

template <typename VT, typename T, int C, int NF>
static hipError_t rg_launch(hipStream_t st, SpmmItem* items, const int* idx, int cnt) {
  auto fn = k_spmm_rg<VT, T, C, NF>;
  BatchArgs<RgDesc> bt{};
  bt.count = cnt;
  int off = 0;
  for (int q = 0; q < cnt; ++q) {
    SpmmItem& it = items[idx[q]];
    const int nb = stream_grid(it.g, (const void*)fn);
    it.nblk = nb;
    RgDesc& d = bt.d[q];
    d.n = it.g.n;
    d.gp = it.rg.gp;
    d.col = it.rg.col;
    d.val = sizeof(VT) == 4 ? static_cast<const void*>(it.rg.val)
                            : static_cast<const void*>(it.rg.val64);
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
    d.ld = it.g.ld;
    d.ncolv = it.g.ncolv;
    d.voff = it.voff;
    d.il = it.g.xil;
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

hipError_t launch_spmm_rg_group(hipStream_t st, SpmmItem* items, const int* idx, int cnt) {
  if (!items || !idx || cnt < 1 || cnt > kMaxBatch) return hipErrorInvalidValue;
  const SpmmItem& it = items[idx[0]];
  for (int q = 0; q < cnt; ++q) {
    const SpmmItem& x = items[idx[q]];
    // FP32 values on FP32 blocks, FP64 values on FP64 or FP32 blocks
    const bool ok = (x.g.xbytes == 4 && (x.vt == VT_F32 || x.vt == VT_F64)) ||
                    (x.g.xbytes == 8 && x.vt == VT_F64);
    const void* val = x.vt == VT_F32 ? static_cast<const void*>(x.rg.val)
                                     : static_cast<const void*>(x.rg.val64);
    if (!x.g.rg || !ok || x.g.xbytes != it.g.xbytes || x.vt != it.vt || x.g.C != it.g.C ||
        x.nf != it.nf || x.g.lges != 0 || x.g.ts != 0 || !x.rg.gp || !x.rg.col || !val ||
        reinterpret_cast<uintptr_t>(val) % 16 != 0)
      return hipErrorInvalidValue;
  }
  const int C = it.g.C, nf = it.nf;
  auto by_nf = [&](auto v, auto t, auto c) -> hipError_t {
    using VT = decltype(v);
    using T = decltype(t);
    constexpr int CC = decltype(c)::value;
    if (nf == 0) return rg_launch<VT, T, CC, 0>(st, items, idx, cnt);
    if (nf == 1) return rg_launch<VT, T, CC, 1>(st, items, idx, cnt);
    return rg_launch<VT, T, CC, 2>(st, items, idx, cnt);
  };
  auto by_c = [&](auto v, auto t) -> hipError_t {
    if (C == 1) return by_nf(v, t, std::integral_constant<int, 1>{});
    if (C == 2) return by_nf(v, t, std::integral_constant<int, 2>{});
    return hipErrorInvalidValue;
  };
  if (it.g.xbytes == 8) return by_c(double{}, double{});
  if (it.vt == VT_F64) return by_c(double{}, float{});
  return by_c(float{}, float{});
}

// ---------------------------------------------------------------------------
// Row groups from the CSR arrays on the device: one thread per group merges
// its rows' sorted column lists.  Pass 1 counts each group's union columns
// (cnt[g]); pass 2, given gp (the exclusive prefix sums), writes the union
// columns and their kRowGroup values (with val, the FP64 values rounded to
// FP32; with val64, as they are; zero where a row has no entry).
// ---------------------------------------------------------------------------
template <bool FILL>
__global__ __launch_bounds__(kThreads) void k_rowgroup_build(int64_t n, const int* __restrict__ rp,
                                                             const int* __restrict__ ci,
                                                             const double* __restrict__ v64,
                                                             int* __restrict__ cnt,
                                                             const int* __restrict__ gp,
                                                             int* __restrict__ col,
                                                             float* __restrict__ val,
                                                             double* __restrict__ val64) {
  const int64_t ng = (n + kRowGroup - 1) / kRowGroup;
  const int64_t g = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (g >= ng) return;
  const int64_t r0 = g * kRowGroup;
  const int nr = (int)min((int64_t)kRowGroup, n - r0);
  int k[kRowGroup], e[kRowGroup];
#pragma unroll
  for (int r = 0; r < kRowGroup; ++r) {
    k[r] = r < nr ? rp[r0 + r] : 0;
    e[r] = r < nr ? rp[r0 + r + 1] : 0;
  }
  int u = FILL ? gp[g] : 0;
  int m = 0;
  for (;;) {
    int c = INT_MAX;  // columns are below n <= INT_MAX
#pragma unroll
    for (int r = 0; r < kRowGroup; ++r)
      if (k[r] < e[r]) c = min(c, ci[k[r]]);
    if (c == INT_MAX) break;
    double vr[kRowGroup] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int r = 0; r < kRowGroup; ++r)
      if (k[r] < e[r] && ci[k[r]] == c) {
        if (FILL) vr[r] = v64[k[r]];
        ++k[r];
      }
    if (FILL) {
      col[u] = c;
      if (val)
        reinterpret_cast<float4*>(val)[u] =
            make_float4((float)vr[0], (float)vr[1], (float)vr[2], (float)vr[3]);
      if (val64) {
        reinterpret_cast<double2*>(val64)[2 * u] = make_double2(vr[0], vr[1]);
        reinterpret_cast<double2*>(val64)[2 * u + 1] = make_double2(vr[2], vr[3]);
      }
      ++u;
    }
    ++m;
  }
  if (!FILL) cnt[g] = m;
}

hipError_t launch_rowgroup_count(hipStream_t st, int64_t n, const int* rp, const int* ci,
                                 int* cnt) {
  if (n < 1 || !rp || !ci || !cnt) return hipErrorInvalidValue;
  const int64_t ng = (n + kRowGroup - 1) / kRowGroup;
  hipLaunchKernelGGL(k_rowgroup_build<false>, dim3((unsigned)((ng + kThreads - 1) / kThreads)),
                     dim3(kThreads), 0, st, n, rp, ci, nullptr, cnt, nullptr, nullptr, nullptr,
                     nullptr);
  return hipGetLastError();
}

hipError_t launch_rowgroup_fill(hipStream_t st, int64_t n, const int* rp, const int* ci,
                                const double* v64, const int* gp, int* col, float* val,
                                double* val64) {
  if (n < 1 || !rp || !ci || !v64 || !gp || !col || (!val && !val64) ||
      reinterpret_cast<uintptr_t>(val) % 16 != 0 || reinterpret_cast<uintptr_t>(val64) % 16 != 0)
    return hipErrorInvalidValue;
  const int64_t ng = (n + kRowGroup - 1) / kRowGroup;
  hipLaunchKernelGGL(k_rowgroup_build<true>, dim3((unsigned)((ng + kThreads - 1) / kThreads)),
                     dim3(kThreads), 0, st, n, rp, ci, v64, nullptr, gp, col, val, val64);
  return hipGetLastError();
}

}  // namespace ld
