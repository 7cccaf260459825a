// Device helpers shared by the HIP sources: MFMA wrappers (gfx950), complex MFMA products,
// vector loads and wave reductions.
#pragma once

#include "ptebd_internal.h"

namespace ptebd {
namespace {

// ---------------------------------------------------------------- MFMA wrappers
// 16x16x4 MFMA.  Operand lane layout (both precisions): lane l supplies A[l%16][l/16] and
// B[l/16][l%16].  Result: 4 values per lane in column l%16; their rows differ between the
// f32 and f64 instructions (checked on gfx950): f32 rows 4*(l/16)+v, f64 rows l/16+4v.
template <class T>
struct Mfma;

template <>
struct Mfma<float> {
  typedef float v4 __attribute__((ext_vector_type(4)));
  __device__ static inline v4 op(float a, float b, v4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  __device__ static inline int row(int lane, int v) { return 4 * (lane >> 4) + v; }
};

template <>
struct Mfma<double> {
  typedef double v4 __attribute__((ext_vector_type(4)));
  __device__ static inline v4 op(double a, double b, v4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  __device__ static inline int row(int lane, int v) { return (lane >> 4) + 4 * v; }
};

// acc += a * b (complex); acc[0] real part, acc[1] imaginary part.
template <class T>
__device__ inline void cmfma(typename Mfma<T>::v4 (&acc)[2], cplx<T> a, cplx<T> b) {
  acc[0] = Mfma<T>::op(a.re, b.re, acc[0]);
  acc[0] = Mfma<T>::op(-a.im, b.im, acc[0]);
  acc[1] = Mfma<T>::op(a.re, b.im, acc[1]);
  acc[1] = Mfma<T>::op(a.im, b.re, acc[1]);
}

// acc += conj(x) * y (complex), the Gram-matrix update.
template <class T>
__device__ inline void gram_mfma(typename Mfma<T>::v4 (&acc)[2], cplx<T> x, cplx<T> y) {
  acc[0] = Mfma<T>::op(x.re, y.re, acc[0]);
  acc[0] = Mfma<T>::op(x.im, y.im, acc[0]);
  acc[1] = Mfma<T>::op(x.re, y.im, acc[1]);
  acc[1] = Mfma<T>::op(-x.im, y.re, acc[1]);
}

template <class T>
__device__ inline cplx<T> czero() {
  cplx<T> z;
  z.re = T(0);
  z.im = T(0);
  return z;
}

// Four consecutive complex entries from 16-byte aligned memory (zeros when !ok).
template <class T>
__device__ inline void load4(bool ok, const cplx<T>* __restrict__ p, cplx<T> (&o)[4]) {
  if (!ok) {
    for (int t = 0; t < 4; ++t) o[t] = czero<T>();
    return;
  }
  if constexpr (sizeof(T) == 4) {
    const float4 u = *reinterpret_cast<const float4*>(p);
    const float4 w = *reinterpret_cast<const float4*>(p + 2);
    o[0].re = u.x; o[0].im = u.y; o[1].re = u.z; o[1].im = u.w;
    o[2].re = w.x; o[2].im = w.y; o[3].re = w.z; o[3].im = w.w;
  } else {
    for (int t = 0; t < 4; ++t) {
      const double2 u = *reinterpret_cast<const double2*>(p + t);
      o[t].re = u.x;
      o[t].im = u.y;
    }
  }
}

__device__ inline double wave_max(double v) {
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
  return v;
}

__device__ inline double wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

}  // namespace
}  // namespace ptebd
