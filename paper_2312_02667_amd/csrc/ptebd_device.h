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

// Device memory reached through a pointer read from a descriptor.  Such a pointer is
// generic to the compiler, and generic (flat) accesses count against the LDS counter as
// well as the vector-memory one: every wait for an LDS result would then also wait for the
// global loads in flight, which defeats prefetching.  Casting it to the global address
// space gives global loads and stores (and the scalar-base + 32-bit offset form).
template <class T>
using gptr = __attribute__((address_space(1))) T*;

// Native vector types for 16-byte global accesses (plain loads and stores, no class copy
// through an address-space-qualified reference).
typedef float vf4 __attribute__((ext_vector_type(4)));
typedef double vd2 __attribute__((ext_vector_type(2)));

template <class T>
__device__ inline gptr<T> as_global(T* p) {
  return (gptr<T>)p;
}

// One complex entry read through a global pointer (by value, for use in expressions that
// mix it with local values).
template <class T>
__device__ inline cplx<T> gload(gptr<const cplx<T>> p) {
  cplx<T> z;
  z.re = p->re;
  z.im = p->im;
  return z;
}

template <class T>
__device__ inline void gstore(gptr<cplx<T>> p, cplx<T> z) {
  p->re = z.re;
  p->im = z.im;
}

// Entry idx of a global complex array addressed by a 32-bit element index (every array
// indexed this way holds well under 2^28 entries), which lets the compiler use the scalar
// base + 32-bit vector offset address form instead of a 64-bit address per lane.
template <class T>
__device__ inline gptr<const cplx<T>> gat(gptr<const cplx<T>> base, uint32_t idx) {
  return (gptr<const cplx<T>>)((gptr<const char>)base + idx * (uint32_t)sizeof(cplx<T>));
}
template <class T>
__device__ inline gptr<cplx<T>> gat(gptr<cplx<T>> base, uint32_t idx) {
  return (gptr<cplx<T>>)((gptr<char>)base + idx * (uint32_t)sizeof(cplx<T>));
}

// Entries idx and idx + 1 (idx even for FP32: one 16-byte load).
template <class T>
__device__ inline void gload_pair(gptr<const cplx<T>> base, uint32_t idx, cplx<T>& a,
                                  cplx<T>& b) {
  if constexpr (sizeof(T) == 4) {
    const vf4 u = *reinterpret_cast<gptr<const vf4>>(gat<T>(base, idx));
    a.re = u.x; a.im = u.y; b.re = u.z; b.im = u.w;
  } else {
    a = gload<T>(gat<T>(base, idx));
    b = gload<T>(gat<T>(base, idx + 1));
  }
}

// z when ok, else 0 (a select, no branch).
template <class T>
__device__ inline cplx<T> cmask(cplx<T> z, bool ok) {
  cplx<T> o;
  o.re = ok ? z.re : T(0);
  o.im = ok ? z.im : T(0);
  return o;
}

// Four consecutive complex entries from 16-byte aligned memory (zeros when !ok).
template <class T>
__device__ inline void load4(bool ok, gptr<const cplx<T>> p, cplx<T> (&o)[4]) {
  if (!ok) {
    for (int t = 0; t < 4; ++t) o[t] = czero<T>();
    return;
  }
  if constexpr (sizeof(T) == 4) {
    const vf4 u = *reinterpret_cast<gptr<const vf4>>(p);
    const vf4 w = *reinterpret_cast<gptr<const vf4>>(p + 2);
    o[0].re = u.x; o[0].im = u.y; o[1].re = u.z; o[1].im = u.w;
    o[2].re = w.x; o[2].im = w.y; o[3].re = w.z; o[3].im = w.w;
  } else {
    for (int t = 0; t < 4; ++t) {
      const vd2 u = *reinterpret_cast<gptr<const vd2>>(p + t);
      o[t].re = u.x;
      o[t].im = u.y;
    }
  }
}

// XCD-aware work order for per-gate tiles, on a one-dimensional grid of `per_gate` slots per
// gate for the gate count rounded up to a multiple of 8 (xcd_grid).  The workgroups of a
// launch are handed to the eight XCDs in turn (workgroup L to XCD L % 8), so giving slot L to
// gate 8 (L / 8 / per_gate) + L % 8 keeps every tile of a gate on one XCD: the operand panels
// its tiles share are read into that XCD's L2 once instead of once per XCD.  A gate index at
// or past the gate count is padding, to be skipped by the caller.
__device__ inline void xcd_gate_tile(int per_gate, int& gate, int& tile) {
  const int slot = (int)(blockIdx.x >> 3);
  gate = (slot / per_gate) * 8 + (int)(blockIdx.x & 7);
  tile = slot % per_gate;
}

inline unsigned xcd_grid(int per_gate, int n_gates) {
  return (unsigned)per_gate * (unsigned)((n_gates + 7) / 8 * 8);
}

// Round-robin (circle method) tournament: player in `slot` during `round`, for an even
// number of players; slot 0 is fixed, the others rotate.  Pairs are (p, nplayers-1-p).
__device__ inline int rr_player(int slot, int round, int nplayers) {
  return slot == 0 ? 0 : 1 + ((slot - 1 + round) % (nplayers - 1));
}

// The same tournament for 32 players and round < 31, without an integer division.
__device__ inline int rr32(int slot, int round) {
  int x = slot - 1 + round;
  x -= (x >= 31) ? 31 : 0;
  return slot == 0 ? 0 : 1 + x;
}

// FP64 reciprocal square root for positive finite arguments: the hardware estimate (relative
// error 2^-24 on gfx950, measured) refined by NEWTON Newton steps, each of which doubles the
// number of correct bits: one step gives 2^-47, two give full double precision.
template <int NEWTON>
__device__ inline double rsqrt_f64(double x) {
  double y = __builtin_amdgcn_rsq(x);
#pragma unroll
  for (int i = 0; i < NEWTON; ++i) y = y * (1.5 - 0.5 * x * y * y);
  return y;
}

// Jacobi rotation of the Hermitian 2x2 block [[a, g], [conj(g), b]] in FP64 (the symmetric
// Schur step with the phase of g factored out): J = [[c, s], [-conj(s), c]] with
// zeta = (b - a) / (2|g|), t = sign(zeta) / (|zeta| + sqrt(1 + zeta^2)), c = 1/sqrt(1+t^2),
// s = t c g/|g|; J^H [[a, g], [conj g, b]] J is diagonal.  With d = |b - a| and
// S = sqrt(d^2 + 4|g|^2) the same rotation is c = sqrt((d + S) / (2S)) and
// s = sign(b - a) g sqrt(2 / (S (d + S))) (sign +1 for b = a), which takes one square root
// and one reciprocal square root, no division, and stays finite for |g| far below |b - a|.
// A block whose entries lie outside [1e-140, 1e140] is first scaled by 2^(+-600) (exact) so
// that d^2 + 4|g|^2 stays a normal number.  Identity when |g| <= thr * sqrt(a b) or g = 0.
// NEWTON: refinement steps of the reciprocal square roots (2 for rotations applied in FP64;
// 1 is exact to 2^-47, ample for rotations rounded to FP32).
template <int NEWTON>
__device__ inline bool jacobi_rotation(double a, double b, double gr, double gi, double thr,
                                       double& c, double& sr, double& si) {
  const double g2 = gr * gr + gi * gi;
  c = 1.0;
  sr = 0.0;
  si = 0.0;
  if (!(g2 > 0.0) || g2 <= thr * thr * fmax(a * b, 0.0)) return false;
  double d = fabs(b - a), xr = gr, xi = gi;
  const double m = fmax(d, fmax(fabs(gr), fabs(gi)));
  if (m < 1e-140 || m > 1e140) {
    const double f = m < 1e-140 ? 0x1p600 : 0x1p-600;
    d *= f;
    xr *= f;
    xi *= f;
  }
  const double dd = fma(d, d, 4.0 * (xr * xr + xi * xi));
  const double S = dd * rsqrt_f64<NEWTON>(dd);
  const double e = d + S;
  const double sf = rsqrt_f64<NEWTON>(0.5 * S * e);
  c = 0.5 * e * sf;
  const double ss = b >= a ? sf : -sf;
  sr = ss * xr;
  si = ss * xi;
  return true;
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
