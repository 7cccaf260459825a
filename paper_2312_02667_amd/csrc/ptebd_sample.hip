// HIP kernels of the measurement step that follows Canonicalize in Algorithm 1:
//   sample_site_kernel -- one site of perfect sampling (Ferris and Vidal) for a batch of bit
//                         strings: a (samples x chi_q) by (chi_q x 2 chi_{q+1}) complex
//                         product on MFMA, FP64 conditional probabilities and decisions
//   scale_state_kernel -- the normalization of a canonical form: Lambda[i] / n on the inner
//                         bonds, n Gamma[q] on the inner sites
#include <algorithm>

#include "ptebd_device.h"
#include "ptebd_internal.h"

namespace ptebd {
namespace {

// Perfect sampling at site q for samples [16 b, 16 b + 16) (b = blockIdx.x).
// The previous site left, per sample i, the unnormalized row W_prev[i, :] (plane 0 then
// plane 1, cl values each), the chosen plane sel[i] and 1 / sqrt(p_sel); the prefix vector
// is v_i = W_prev[i, sel_i cl + a] * scale_i (v_i = (1) at site 0).  This site forms
//   W[i, p cm + c] = sum_a v_i[a] Gamma[q]_{a p c} Lambda[q+1]_c          (p = 0, 1)
// with B = Gamma Lambda right-isometric in the canonical form, p_p = sum_c |W[i, p cm + c]|^2
// in FP64, and bit q of sample i = (u_i < p_0 / (p_0 + p_1)) ? 0 : 1.
// Four waves; each takes groups of four 16-column output tiles; K = cl in steps of 4.
template <class T>
__global__ __launch_bounds__(256) void sample_site_kernel(SampleSite a) {
  typedef typename Mfma<T>::v4 V4;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int col = lane & 15, grp = lane >> 4;
  const int i0 = blockIdx.x * 16;
  const int cl = a.cl, cm = a.cm, ncols = 2 * cm;
  const cplx<T>* __restrict__ G = (const cplx<T>*)a.gamma;
  const cplx<T>* __restrict__ win = (const cplx<T>*)a.w_in;
  cplx<T>* __restrict__ wout = (cplx<T>*)a.w_out;
  __shared__ double part[4][16][2];

  // A operand: lane supplies row `col` (sample i0 + col), k = k0 + grp
  const int my_i = i0 + col;
  const bool row_ok = my_i < a.n_samples;
  const cplx<T>* __restrict__ vrow = nullptr;
  T vscale = T(1);
  if (row_ok && !a.first) {
    vrow = win + (size_t)my_i * a.ldw + (size_t)a.sel_in[my_i] * cl;
    vscale = (T)a.scale_in[my_i];
  }
  double np0[4] = {0.0, 0.0, 0.0, 0.0}, np1[4] = {0.0, 0.0, 0.0, 0.0};
  for (int cb = wave * 64; cb < ncols; cb += 256) {
    V4 acc[4][2];
    for (int t = 0; t < 4; ++t)
      for (int v = 0; v < 4; ++v) {
        acc[t][0][v] = T(0);
        acc[t][1][v] = T(0);
      }
    // B operand columns of this lane, one per tile
    int boff[4];
    T blam[4];
    for (int t = 0; t < 4; ++t) {
      const int j = cb + 16 * t + col;
      if (j < ncols) {
        const int p = j >= cm ? 1 : 0;
        const int c = j - p * cm;
        boff[t] = p * cl * cm + c * cl;
        blam[t] = (T)a.lam_r[c];
      } else {
        boff[t] = -1;
        blam[t] = T(0);
      }
    }
    for (int k0 = 0; k0 < cl; k0 += 4) {
      const int k = k0 + grp;
      cplx<T> av = czero<T>();
      if (row_ok && k < cl) {
        if (a.first) {
          av.re = k == 0 ? T(1) : T(0);
        } else {
          const cplx<T> z = vrow[k];
          av.re = z.re * vscale;
          av.im = z.im * vscale;
        }
      }
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        cplx<T> bv = czero<T>();
        if (boff[t] >= 0 && k < cl) {
          const cplx<T> g = G[boff[t] + k];
          bv.re = g.re * blam[t];
          bv.im = g.im * blam[t];
        }
        cmfma<T>(acc[t], av, bv);
      }
    }
    for (int t = 0; t < 4; ++t) {
      const int j = cb + 16 * t + col;
      if (j >= ncols) continue;
      for (int v = 0; v < 4; ++v) {
        const int i = i0 + Mfma<T>::row(lane, v);
        const T re = acc[t][0][v], im = acc[t][1][v];
        if (i < a.n_samples) {
          cplx<T> z;
          z.re = re;
          z.im = im;
          wout[(size_t)i * a.ldw + j] = z;
        }
        const double w2 = (double)re * (double)re + (double)im * (double)im;
        if (j < cm)
          np0[v] += w2;
        else
          np1[v] += w2;
      }
    }
  }
  // lanes with equal grp hold the same rows: reduce over the 16 columns, then over waves
  for (int v = 0; v < 4; ++v)
    for (int o = 1; o < 16; o <<= 1) {
      np0[v] += __shfl_xor(np0[v], o);
      np1[v] += __shfl_xor(np1[v], o);
    }
  if (col == 0)
    for (int v = 0; v < 4; ++v) {
      const int r = Mfma<T>::row(lane, v);
      part[wave][r][0] = np0[v];
      part[wave][r][1] = np1[v];
    }
  __syncthreads();
  if (tid < 16) {
    const int i = i0 + tid;
    if (i < a.n_samples) {
      const double p0 = (part[0][tid][0] + part[1][tid][0]) + (part[2][tid][0] + part[3][tid][0]);
      const double p1 = (part[0][tid][1] + part[1][tid][1]) + (part[2][tid][1] + part[3][tid][1]);
      const double tot = p0 + p1;
      const double u = a.u[(size_t)i * a.ustride];
      int b = 0;
      if (!(tot > 0.0) || !isfinite(tot)) {
        atomicOr(a.err, 1);
      } else {
        b = (u < p0 / tot) ? 0 : 1;
      }
      const double pb = b ? p1 : p0;
      a.bits[(size_t)i * a.bstride] = (uint8_t)b;
      a.sel_out[i] = b;
      a.scale_out[i] = pb > 0.0 ? 1.0 / sqrt(pb) : 0.0;
    }
  }
}

// Lambda[i] /= n for the inner bonds i = 1..N-1 and Gamma[q] *= n for the inner sites
// q = 1..N-2 (blockIdx.y = site / bond index).
template <class T>
__global__ void scale_state_kernel(void* gamma_base, size_t slot_elems, double* lam_base,
                                   int lam_stride, const int32_t* __restrict__ dims,
                                   int n_sites, double nrm) {
  const int q = blockIdx.y;
  const double inv = 1.0 / nrm;
  if (q >= 1 && q <= n_sites - 2) {
    cplx<T>* g = (cplx<T>*)gamma_base + (size_t)q * slot_elems;
    const size_t cnt = 2 * (size_t)dims[q] * dims[q + 1];
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < cnt;
         e += (size_t)gridDim.x * blockDim.x) {
      cplx<T> z = g[e];
      z.re = (T)((double)z.re * nrm);
      z.im = (T)((double)z.im * nrm);
      g[e] = z;
    }
  }
  if (q >= 1 && q <= n_sites - 1 && blockIdx.x == 0) {
    double* l = lam_base + (size_t)q * lam_stride;
    for (int j = threadIdx.x; j < dims[q]; j += blockDim.x) l[j] *= inv;
  }
}

}  // namespace

template <class T>
void launch_sample_site(const SampleSite& a, hipStream_t stream) {
  const int blocks = (a.n_samples + 15) / 16;
  hipLaunchKernelGGL(sample_site_kernel<T>, dim3(blocks), dim3(256), 0, stream, a);
}

template <class T>
void launch_scale_state(void* gamma_base, size_t slot_elems, double* lam_base, int lam_stride,
                        const int32_t* d_dims, int n_sites, int max_elems, double nrm,
                        hipStream_t stream) {
  const int bx = std::max(1, std::min(64, (max_elems + 255) / 256));
  hipLaunchKernelGGL(scale_state_kernel<T>, dim3(bx, n_sites), dim3(256), 0, stream, gamma_base,
                     slot_elems, lam_base, lam_stride, d_dims, n_sites, nrm);
}

template void launch_sample_site<float>(const SampleSite&, hipStream_t);
template void launch_sample_site<double>(const SampleSite&, hipStream_t);
template void launch_scale_state<float>(void*, size_t, double*, int, const int32_t*, int, int,
                                        double, hipStream_t);
template void launch_scale_state<double>(void*, size_t, double*, int, const int32_t*, int, int,
                                         double, hipStream_t);

}  // namespace ptebd
