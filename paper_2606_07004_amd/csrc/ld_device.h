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

// Vectors handed to the multi-vector streaming kernels.  x[v] is a block of
// the same [n][ld] layout as the output; mult[v][col] (may be null -> 1) is
// the per-column factor that turns the stored block into the basis vector.
struct VecSet {
  const void* x[kMaxNv];
  const double* mult[kMaxNv];
};

}  // namespace ld
