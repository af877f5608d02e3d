// Device-side helpers shared by the liblogdet kernels (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ld {

constexpr int kThreads = 256;   // every streaming kernel uses 256-thread blocks
constexpr int kWave = 64;
constexpr int kMaxNv = 8;       // vectors handled by one dots/update launch

// Blocks are dispatched round-robin over the 8 XCDs of the MI355X (block b on
// XCD b % 8), each XCD with its own L2.  Remap so that every XCD owns one
// contiguous range of row blocks: rows that share gathered neighbours (and
// the partial-sum layout) then stay inside one L2.
__device__ inline int xcd_remap(int b, int nb) {
  const int nb8 = nb & ~7;
  if (b >= nb8) return b;
  return (b & 7) * (nb8 >> 3) + (b >> 3);
}

// bf16 storage is the upper half of an IEEE float.
__device__ inline float bf16_to_float(uint16_t v) { return __uint_as_float(uint32_t(v) << 16); }

template <typename T> struct Acc;
template <> struct Acc<double> { using type = double; };
template <> struct Acc<float> { using type = float; };
template <> struct Acc<_Float16> { using type = float; };  // FP16 storage, FP32 sums

template <typename VT, typename A> __device__ inline A value_as(VT v) { return A(v); }
template <> __device__ inline float value_as<uint16_t, float>(uint16_t v) { return bf16_to_float(v); }
template <> __device__ inline double value_as<uint16_t, double>(uint16_t v) { return double(bf16_to_float(v)); }

// 16-byte vector access: 2 doubles, 4 floats or 8 FP16 values per lane.
template <typename T> struct V16;
template <> struct V16<double> {
  static constexpr int N = 2;
  double v[2];
  __device__ inline void load(const double* p) {
    const double2 t = *reinterpret_cast<const double2*>(p);
    v[0] = t.x; v[1] = t.y;
  }
  __device__ inline void store(double* p) const {
    double2 t; t.x = v[0]; t.y = v[1];
    *reinterpret_cast<double2*>(p) = t;
  }
  // streaming load: last use of the line
  __device__ inline void load_nt(const double* p) {
    typedef double d2 __attribute__((ext_vector_type(2)));
    const d2 t = __builtin_nontemporal_load(reinterpret_cast<const d2*>(p));
    v[0] = t.x; v[1] = t.y;
  }
  // streaming store: the line is not kept in the caches for reuse
  __device__ inline void store_nt(double* p) const {
    typedef double d2 __attribute__((ext_vector_type(2)));
    const d2 t = {v[0], v[1]};
    __builtin_nontemporal_store(t, reinterpret_cast<d2*>(p));
  }
};
template <> struct V16<float> {
  static constexpr int N = 4;
  float v[4];
  __device__ inline void load(const float* p) {
    const float4 t = *reinterpret_cast<const float4*>(p);
    v[0] = t.x; v[1] = t.y; v[2] = t.z; v[3] = t.w;
  }
  __device__ inline void store(float* p) const {
    float4 t; t.x = v[0]; t.y = v[1]; t.z = v[2]; t.w = v[3];
    *reinterpret_cast<float4*>(p) = t;
  }
  // streaming load: last use of the line
  __device__ inline void load_nt(const float* p) {
    typedef float f4 __attribute__((ext_vector_type(4)));
    const f4 t = __builtin_nontemporal_load(reinterpret_cast<const f4*>(p));
    v[0] = t.x; v[1] = t.y; v[2] = t.z; v[3] = t.w;
  }
  // streaming store: the line is not kept in the caches for reuse
  __device__ inline void store_nt(float* p) const {
    typedef float f4 __attribute__((ext_vector_type(4)));
    const f4 t = {v[0], v[1], v[2], v[3]};
    __builtin_nontemporal_store(t, reinterpret_cast<f4*>(p));
  }
};

template <> struct V16<_Float16> {
  static constexpr int N = 8;
  typedef _Float16 h8 __attribute__((ext_vector_type(8)));
  _Float16 v[8];
  __device__ inline void load(const _Float16* p) {
    const h8 t = *reinterpret_cast<const h8*>(p);
#pragma unroll
    for (int e = 0; e < 8; ++e) v[e] = t[e];
  }
  __device__ inline void store(_Float16* p) const {
    h8 t;
#pragma unroll
    for (int e = 0; e < 8; ++e) t[e] = v[e];
    *reinterpret_cast<h8*>(p) = t;
  }
  // streaming load: last use of the line
  __device__ inline void load_nt(const _Float16* p) {
    const h8 t = __builtin_nontemporal_load(reinterpret_cast<const h8*>(p));
#pragma unroll
    for (int e = 0; e < 8; ++e) v[e] = t[e];
  }
  // streaming store: the line is not kept in the caches for reuse
  __device__ inline void store_nt(_Float16* p) const {
    h8 t;
#pragma unroll
    for (int e = 0; e < 8; ++e) t[e] = v[e];
    __builtin_nontemporal_store(t, reinterpret_cast<h8*>(p));
  }
};

// Ordering of LDS accesses between lanes of one wave (a wave's LDS
// instructions run in order; this keeps the compiler from moving them).
__device__ inline void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Vectors handed to the multi-vector streaming kernels.  x[v] is a block of
// the same [n][ld] layout as the output; mult[v][col] (may be null -> 1) is
// the per-column factor that turns the stored block into the basis vector.
struct VecSet {
  const void* x[kMaxNv];
  const double* mult[kMaxNv];
};

// ---------------------------------------------------------------------------
// Row mapping shared by the streaming kernels.  Rows are swept in chunks of
// RPI = 256 / L consecutive rows; block b takes chunks b, b + nblk, ... so the
// whole grid advances through the matrix in order (the rows in flight, and
// the probe-vector rows their sparse entries gather, stay within a window
// that the memory-side cache holds).  Inside a chunk L lanes share a row
// and each lane owns C 16-byte chunks of the row's probe vector (chunk c of
// lane l is chunk l + L*c), so L*C chunks cover ld columns with few idle
// lanes (96 FP32 probes: L = 8, C = 3).  Per-block partial sums are stored
// transposed, part[i][block], so the reduction reads contiguous memory.
// ---------------------------------------------------------------------------
// With an entry split ES = 2^lgES (the product only) the L lanes of a row
// form ES groups of Lc = L / ES column lanes; group eg takes every ES-th
// sparse entry of the row and the groups' sums are added at the row's end.
// Without an entry split L need not be a power of two (12 lanes for the 12
// chunks of 96 FP16 probes instead of 16 with 4 idle): rows never straddle a
// wave, each wave holds 64 / L rows and its last 64 mod L lanes are idle
// (on = false).  lb is the wave lane of the row's first lane.
struct RowMap {
  int lg, L, rpi, rg, gl, Lc, cl, eg, lb;
  bool on;
  __device__ RowMap(int lgL, int lgES = 0) : lg(lgL), L(1 << lgL), rpi(kThreads >> lgL) {
    rg = (int)threadIdx.x >> lg;
    gl = (int)threadIdx.x & (L - 1);
    Lc = L >> lgES;
    cl = gl & (Lc - 1);
    eg = lgES ? gl >> (lgL - lgES) : 0;
    lb = ((int)threadIdx.x & 63) & ~(L - 1);
    on = true;
  }
  // any 1 <= L <= 64 (no entry split unless L is a power of two)
  __device__ static RowMap lanes(int L, int lgES) {
    if ((L & (L - 1)) == 0) return RowMap(__builtin_ctz((unsigned)L), lgES);
    RowMap m(0);
    const int rpw = 64 / L, lane = (int)threadIdx.x & 63, rw = lane / L;
    m.lg = -1;
    m.L = L;
    m.rpi = (kThreads / 64) * rpw;
    m.on = rw < rpw;
    m.rg = ((int)threadIdx.x >> 6) * rpw + (m.on ? rw : 0);
    m.gl = lane - rw * L;
    m.Lc = L;
    m.cl = m.gl;
    m.eg = 0;
    m.lb = rw * L;
    return m;
  }
};

// Chunk taken by this block in round j.  The grid is at most one resident
// wave of blocks and, from 8 blocks up, a multiple of 8; blocks are placed
// round-robin on the 8 XCDs (block b on XCD b % 8), so in every round XCD x
// gets one contiguous band of the round's chunks: rows a few chunks apart
// (the +-N neighbours of a stencil) then share that XCD's L2.
__device__ inline int chunk_of(int j, int b, int nb) {
  const int base = j * nb;
  return (nb & 7) ? base + b : base + (b & 7) * (nb >> 3) + (b >> 3);
}

// Column sums of the per-thread slots red[rg][c][gl][e] over the row groups
// of the block, stored as the block's partial sums (times mult[col]).
template <int C, int VEC>
__device__ inline void red_partials(const double* red, const RowMap& rm, int ld, const double* mult,
                                    double* part, size_t row0, int bk, int nbk) {
  const int WC = rm.Lc * C * VEC;
  for (int i = threadIdx.x; i < WC; i += kThreads) {
    double sum = 0.0;
    for (int q = 0; q < rm.rpi; ++q) sum += red[q * WC + i];
    if (i < ld) part[(row0 + i) * nbk + bk] = sum * (mult ? mult[i] : 1.0);
  }
  __syncthreads();
}

// Slot of thread (rg, cl) for chunk c, element e in a [rpi][C*Lc*VEC] array
// (the slot index within a row group is the column).
template <int C, int VEC>
__device__ inline int red_slot(const RowMap& rm, int c, int e) {
  return rm.rg * (rm.Lc * C * VEC) + (c * rm.Lc + rm.cl) * VEC + e;
}

// Sum the per-lane accumulators of one vector over the row groups of the
// block and store the block's partial sums (times mult[col]).
template <int C, int VEC>
__device__ inline void block_partials(const double (&acc)[C][VEC], double* red, const RowMap& rm,
                                      int ld, const double* mult, double* part, size_t row0, int bk,
                                      int nbk) {
  if (rm.eg == 0 && rm.on) {
#pragma unroll
    for (int c = 0; c < C; ++c)
#pragma unroll
      for (int e = 0; e < VEC; ++e) red[red_slot<C, VEC>(rm, c, e)] = acc[c][e];
  }
  __syncthreads();
  red_partials<C, VEC>(red, rm, ld, mult, part, row0, bk, nbk);
}

}  // namespace ld
