// Two-site wavefunction theta of one bond update (Sec. II.C) as complex GEMMs on MFMA, for a
// batch of gates (one descriptor each), in the path's precision T.
#include "ptebd_device.h"
#include "ptebd_internal.h"

namespace ptebd {
namespace {

// ---------------------------------------------------------------- theta
// One workgroup computes a 32 (a) x 32 (c) tile of the four products
// M_st = A_s B_t, A_s = diag(Lambda[q]) Gamma[q]_s diag(Lambda[q+1]) (chi_q x chi_{q+1}),
// B_t = Gamma[q+1]_t diag(Lambda[q+2]) (chi_{q+1} x chi_{q+2}), then mixes them with the
// gate: theta[(s',a),(t',c)] = sum_st U[(s't'),(st)] M_st[a,c].  Four waves, each a 16x16
// sub-tile of all four products; K (= chi_{q+1}) staged through LDS in steps of 16, the next
// step's entries loaded into registers while the current step's products run.  Built
// for four waves per SIMD in FP32 (the three-product form's third accumulators fit without
// spills) and two in FP64.  Tiles in the XCD-aware order of xcd_gate_tile: every tile of a
// gate on one XCD, which reads the gate's Gamma panels into its L2 once.
template <class T>
__global__ __launch_bounds__(256, sizeof(T) == 4 ? 4 : 2) void theta_kernel(const GateDesc* __restrict__ descs,
                                                                            int n_gates, int max_tiles) {
  int gate, tile;
  xcd_gate_tile(max_tiles, gate, tile);
  if (gate >= n_gates) return;
  const GateDesc* d = descs + gate;
  const int cl = d->cl, cm = d->cm, cr = d->cr;
  const int tiles_c = (cr + 31) >> 5;
  const int tiles = ((cl + 31) >> 5) * tiles_c;
  if (tile >= tiles) return;
  const int a0 = (tile / tiles_c) * 32, c0 = (tile % tiles_c) * 32;

  __shared__ cplx<T> As[2][16][33];
  __shared__ cplx<T> Bs[2][16][33];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wa = wave >> 1, wc = wave & 1;
  typedef typename Mfma<T>::v4 V4;
  // FP32: three real products per complex one: for a = x + iy, b = u + iv the MFMAs
  // accumulate P1 = x u, P2 = y v and P3 = (x + y)(u + v); Re ab = P1 - P2,
  // Im ab = P3 - P1 - P2.  FP64 keeps the four-product form (acc[.][0] = Re, acc[.][1] = Im):
  // the third accumulator would halve its occupancy.
  constexpr bool k3 = sizeof(T) == 4;
  V4 acc[4][3];
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 3; ++j)
      for (int v = 0; v < 4; ++v) acc[i][j][v] = T(0);
  auto mfma3 = [](V4(&c)[3], cplx<T> a, T as, cplx<T> b, T bs) {
    if constexpr (k3) {
      c[0] = Mfma<T>::op(a.re, b.re, c[0]);
      c[1] = Mfma<T>::op(a.im, b.im, c[1]);
      c[2] = Mfma<T>::op(as, bs, c[2]);
    } else {
      (void)as;
      (void)bs;
      V4 two[2] = {c[0], c[1]};
      cmfma<T>(two, a, b);
      c[0] = two[0];
      c[1] = two[1];
    }
  };

  const gptr<const cplx<T>> __restrict__ gq = as_global((const cplx<T>*)d->gq);
  const gptr<const cplx<T>> __restrict__ gq1 = as_global((const cplx<T>*)d->gq1);
  const gptr<const double> __restrict__ lam_l = as_global(d->lam_l);
  const gptr<const double> __restrict__ lam_m = as_global((const double*)d->lam_m);
  const gptr<const double> __restrict__ lam_r = as_global(d->lam_r);
  const size_t plane_a = (size_t)cl * cm, plane_b = (size_t)cm * cr;

  // The K step's tiles are four A and four B entries per thread: A entry i is plane s = i/2,
  // row a = tid % 32 (fixed), k = tid / 32 + 8 (i % 2); B entry i is plane s = i/2, column
  // c = tid / 16 + 16 (i % 2), k = tid % 16 (fixed).  The next step's raw entries are loaded
  // into registers while this step's products run; the Lambda factors that do not depend on
  // k are loaded once.
  const int ta = tid & 31, tka = tid >> 5, tkb = tid & 15, tcb = tid >> 4;
  const int ga = a0 + ta;
  const bool oka = ga < cl;
  const double la = oka ? lam_l[ga] : 0.0;
  double lr[2];
  for (int h = 0; h < 2; ++h) {
    const int gc = c0 + tcb + 16 * h;
    lr[h] = gc < cr ? lam_r[gc] : 0.0;
  }
  cplx<T> ra[4], rb[4];
  auto fetch = [&](int k0) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int s = i >> 1, h = i & 1;
      const int gk = k0 + tka + 8 * h;
      ra[i] = czero<T>();
      if (oka && gk < cm) ra[i] = gload<T>(gq + (s * plane_a + (size_t)gk * cl + ga));
      const int gc = c0 + tcb + 16 * h, gkb = k0 + tkb;
      rb[i] = czero<T>();
      if (gc < cr && gkb < cm) rb[i] = gload<T>(gq1 + (s * plane_b + (size_t)gc * cm + gkb));
    }
  };
  auto stage = [&](int k0) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int s = i >> 1, h = i & 1;
      const int k = tka + 8 * h, gk = k0 + k;
      const T sa = (T)(la * (gk < cm ? lam_m[gk] : 0.0));
      cplx<T> va;
      va.re = ra[i].re * sa;
      va.im = ra[i].im * sa;
      As[s][k][ta] = va;
      const T sb = (T)lr[h];
      cplx<T> vb;
      vb.re = rb[i].re * sb;
      vb.im = rb[i].im * sb;
      Bs[s][tkb][tcb + 16 * h] = vb;
    }
  };
  fetch(0);
  for (int k0 = 0; k0 < cm; k0 += 16) {
    stage(k0);
    __syncthreads();
    if (k0 + 16 < cm) fetch(k0 + 16);
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) {
      const int kk = ks * 4 + (lane >> 4);
      const cplx<T> a0v = As[0][kk][wa * 16 + (lane & 15)];
      const cplx<T> a1v = As[1][kk][wa * 16 + (lane & 15)];
      const cplx<T> b0v = Bs[0][kk][wc * 16 + (lane & 15)];
      const cplx<T> b1v = Bs[1][kk][wc * 16 + (lane & 15)];
      const T a0s = a0v.re + a0v.im, a1s = a1v.re + a1v.im;
      const T b0s = b0v.re + b0v.im, b1s = b1v.re + b1v.im;
      mfma3(acc[0], a0v, a0s, b0v, b0s);
      mfma3(acc[1], a0v, a0s, b1v, b1s);
      mfma3(acc[2], a1v, a1s, b0v, b0s);
      mfma3(acc[3], a1v, a1s, b1v, b1s);
    }
    __syncthreads();
  }

  const int has_gate = d->has_gate, transposed = d->transposed, R = d->R;
  T ur[16], ui[16];
  if (has_gate) {
    for (int i = 0; i < 16; ++i) {
      ur[i] = (T)as_global(d->gate)[2 * i];
      ui[i] = (T)as_global(d->gate)[2 * i + 1];
    }
  }
  const gptr<cplx<T>> __restrict__ w = as_global((cplx<T>*)d->w);
  for (int v = 0; v < 4; ++v) {
    const int a = a0 + wa * 16 + Mfma<T>::row(lane, v);
    const int c = c0 + wc * 16 + (lane & 15);
    if (a >= cl || c >= cr) continue;
    T mr[4], mi[4];
    for (int st = 0; st < 4; ++st) {
      if constexpr (k3) {
        mr[st] = acc[st][0][v] - acc[st][1][v];
        mi[st] = acc[st][2][v] - acc[st][0][v] - acc[st][1][v];
      } else {
        mr[st] = acc[st][0][v];
        mi[st] = acc[st][1][v];
      }
    }
    for (int sp = 0; sp < 2; ++sp) {
      for (int tp = 0; tp < 2; ++tp) {
        T tr, ti;
        if (has_gate) {
          tr = T(0);
          ti = T(0);
          const int row = (sp * 2 + tp) * 4;
          for (int st = 0; st < 4; ++st) {
            tr += ur[row + st] * mr[st] - ui[row + st] * mi[st];
            ti += ur[row + st] * mi[st] + ui[row + st] * mr[st];
          }
        } else {
          tr = mr[sp * 2 + tp];
          ti = mi[sp * 2 + tp];
        }
        const int row = sp * cl + a, col = tp * cr + c;
        cplx<T> o;
        o.re = tr;
        if (!transposed) {
          o.im = ti;
          gstore<T>(w + ((size_t)col * R + row), o);
        } else {
          o.im = -ti;
          gstore<T>(w + ((size_t)row * R + col), o);
        }
      }
    }
  }
}

}  // namespace

template <class T>
void launch_theta(const GateDesc* d_desc, int n_gates, int max_tiles, hipStream_t stream) {
  if (n_gates <= 0 || max_tiles <= 0) return;
  hipLaunchKernelGGL(theta_kernel<T>, dim3(xcd_grid(max_tiles, n_gates)), dim3(256), 0, stream,
                     d_desc, n_gates, max_tiles);
}

template void launch_theta<float>(const GateDesc*, int, int, hipStream_t);
template void launch_theta<double>(const GateDesc*, int, int, hipStream_t);

}  // namespace ptebd
