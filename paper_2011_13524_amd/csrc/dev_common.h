// Device-side helpers for the gfx950 kernels: complex arithmetic on
// interleaved (re, im) pairs and the insert-zero index map.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace qsv {

template <typename R>
struct cx {
  R re, im;
};

template <typename R>
__device__ __forceinline__ cx<R> operator+(cx<R> a, cx<R> b) {
  return {a.re + b.re, a.im + b.im};
}
template <typename R>
__device__ __forceinline__ cx<R> operator*(cx<R> a, cx<R> b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
// a * b + c
template <typename R>
__device__ __forceinline__ cx<R> cfma(cx<R> a, cx<R> b, cx<R> c) {
  return {fma(a.re, b.re, fma(-a.im, b.im, c.re)), fma(a.re, b.im, fma(a.im, b.re, c.im))};
}

// 2x2 complex matrix, row-major.
template <typename R>
struct M2 {
  cx<R> m00, m01, m10, m11;
};

// Insert a zero bit at each of the (ascending) positions, turning a dense
// counter into the B0 element it enumerates: bits of i above each position are
// shifted up by one.
__device__ __forceinline__ uint64_t insert_zeros(uint64_t i, const int* pos, int m) {
  for (int j = 0; j < m; ++j) {
    const uint64_t lo = i & ((uint64_t(1) << pos[j]) - 1);
    i = ((i >> pos[j]) << (pos[j] + 1)) | lo;
  }
  return i;
}

// Clang vector types, usable with the non-temporal load/store builtins. State
// amplitudes are streamed once per pass, so HBM traffic uses non-temporal
// accesses (measured on MI355X: ~10% more in-place bandwidth than plain ones).
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ f32x4 nt_load(const f32x4* p) { return __builtin_nontemporal_load(p); }
__device__ __forceinline__ f32x2 nt_load(const f32x2* p) { return __builtin_nontemporal_load(p); }
__device__ __forceinline__ f64x2 nt_load(const f64x2* p) { return __builtin_nontemporal_load(p); }
__device__ __forceinline__ void nt_store(f32x4 v, f32x4* p) { __builtin_nontemporal_store(v, p); }
__device__ __forceinline__ void nt_store(f32x2 v, f32x2* p) { __builtin_nontemporal_store(v, p); }
__device__ __forceinline__ void nt_store(f64x2 v, f64x2* p) { __builtin_nontemporal_store(v, p); }

// Vector access to VEC consecutive amplitudes starting at amplitude index x
// (x must be VEC-aligned in amplitudes when 16-byte vectors are used).
template <typename R, int VEC>
struct AmpIO;

// complex64: a 16-byte vector holds two amplitudes.
template <int VEC>
struct AmpIO<float, VEC> {
  static_assert(VEC == 1 || VEC % 2 == 0, "VEC");
  __device__ __forceinline__ static void load(const float* base, uint64_t x, cx<float>* v) {
    if constexpr (VEC == 1) {
      const f32x2 a = nt_load(reinterpret_cast<const f32x2*>(base + 2 * x));
      v[0] = {a.x, a.y};
    } else {
#pragma unroll
      for (int j = 0; j < VEC / 2; ++j) {
        const f32x4 a = nt_load(reinterpret_cast<const f32x4*>(base + 2 * (x + 2 * j)));
        v[2 * j] = {a.x, a.y};
        v[2 * j + 1] = {a.z, a.w};
      }
    }
  }
  __device__ __forceinline__ static void store(float* base, uint64_t x, const cx<float>* v) {
    if constexpr (VEC == 1) {
      nt_store(f32x2{v[0].re, v[0].im}, reinterpret_cast<f32x2*>(base + 2 * x));
    } else {
#pragma unroll
      for (int j = 0; j < VEC / 2; ++j)
        nt_store(f32x4{v[2 * j].re, v[2 * j].im, v[2 * j + 1].re, v[2 * j + 1].im},
                 reinterpret_cast<f32x4*>(base + 2 * (x + 2 * j)));
    }
  }
};

// complex128: a 16-byte vector holds one amplitude.
template <int VEC>
struct AmpIO<double, VEC> {
  __device__ __forceinline__ static void load(const double* base, uint64_t x, cx<double>* v) {
#pragma unroll
    for (int j = 0; j < VEC; ++j) {
      const f64x2 a = nt_load(reinterpret_cast<const f64x2*>(base + 2 * (x + j)));
      v[j] = {a.x, a.y};
    }
  }
  __device__ __forceinline__ static void store(double* base, uint64_t x, const cx<double>* v) {
#pragma unroll
    for (int j = 0; j < VEC; ++j)
      nt_store(f64x2{v[j].re, v[j].im}, reinterpret_cast<f64x2*>(base + 2 * (x + j)));
  }
};

template <typename R>
__device__ __forceinline__ cx<R> load1(const R* base, uint64_t x) {
  cx<R> v;
  AmpIO<R, 1>::load(base, x, &v);
  return v;
}
template <typename R>
__device__ __forceinline__ void store1(R* base, uint64_t x, cx<R> v) {
  AmpIO<R, 1>::store(base, x, &v);
}

}  // namespace qsv
