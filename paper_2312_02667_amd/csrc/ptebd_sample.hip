// HIP kernels of the measurement step that follows Canonicalize in Algorithm 1:
//   sample_contract_kernel, sample_decide_kernel
//                      -- one site of perfect sampling (Ferris and Vidal) for a batch of bit
//                         strings: a (samples x chi_q) by (chi_q x 2 chi_{q+1}) complex
//                         product on MFMA in 32 x 32 tiles with FP64 partial norms, then the
//                         FP64 conditional probabilities and decisions
//   scale_state_kernel -- the normalization of a canonical form: Lambda[i] / n on the inner
//                         bonds, n Gamma[q] on the inner sites
#include <algorithm>

#include "ptebd_device.h"
#include "ptebd_internal.h"

namespace ptebd {
namespace {

// Perfect sampling at site q, step 1: the contraction.  The previous site left, per sample
// i, the unnormalized row W_prev[i, :] (plane 0 then plane 1, cl values each), the chosen
// plane sel[i] and 1 / sqrt(p_sel); the prefix vector is v_i = W_prev[i, sel_i cl + a] *
// scale_i (v_i = (1) at site 0).  This kernel forms
//   W[i, p cm + c] = sum_a v_i[a] Gamma[q]_{a p c} Lambda[q+1]_c          (p = 0, 1)
// for a 32-sample x 32-column tile per workgroup (blockIdx.x: samples, blockIdx.y: columns
// of the two planes), with B = Gamma Lambda right-isometric in the canonical form, and the
// tile's partial sums of |W[i, .]|^2 over its plane-0 and plane-1 columns in FP64.  K = cl
// is staged through LDS in steps of 16; four waves, each a 16 x 16 sub-tile on MFMA.
template <class T>
__global__ __launch_bounds__(256) void sample_contract_kernel(SampleSite a) {
  typedef typename Mfma<T>::v4 V4;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wa = wave >> 1, wc = wave & 1;
  const int col = lane & 15, grp = lane >> 4;
  const int i0 = blockIdx.x * 32, j0 = blockIdx.y * 32;
  const int cl = a.cl, cm = a.cm, ncols = 2 * cm, S = a.n_samples;
  const cplx<T>* __restrict__ G = (const cplx<T>*)a.gamma;
  const cplx<T>* __restrict__ win = (const cplx<T>*)a.w_in;
  cplx<T>* __restrict__ wout = (cplx<T>*)a.w_out;
  __shared__ cplx<T> As[16][33];  // [k][sample]
  __shared__ cplx<T> Bs[16][33];  // [k][column]
  __shared__ double red[2][32][2];  // [column half][sample][plane]

  // each thread stages two A and two B elements per K step: k = tid & 15, row / column
  // (tid >> 4) and (tid >> 4) + 16 of the tile
  const int lk = tid & 15, lr = tid >> 4;
  const cplx<T>* rowp[2];
  T rsc[2];
  bool rok[2];
  int boff[2];
  T blam[2];
  bool cok[2];
  for (int h = 0; h < 2; ++h) {
    const int i = i0 + lr + 16 * h;
    rok[h] = i < S;
    const int ic = rok[h] ? i : 0;
    rowp[h] = a.first ? win : win + (size_t)ic * a.ldw + (size_t)a.sel_in[ic] * cl;
    rsc[h] = a.first ? T(1) : (T)a.scale_in[ic];
    const int j = j0 + lr + 16 * h;
    cok[h] = j < ncols;
    const int p = j >= cm ? 1 : 0, c = cok[h] ? j - p * cm : 0;
    boff[h] = p * cl * cm + c * cl;
    blam[h] = (T)a.lam_r[c];
  }
  V4 acc[2];
  for (int v = 0; v < 4; ++v) {
    acc[0][v] = T(0);
    acc[1][v] = T(0);
  }
  for (int k0 = 0; k0 < cl; k0 += 16) {
    const int k = k0 + lk;
    const bool kok = k < cl;
    for (int h = 0; h < 2; ++h) {
      cplx<T> av = czero<T>();
      if (rok[h] && kok) {
        if (a.first) {
          av.re = k == 0 ? T(1) : T(0);
        } else {
          const cplx<T> z = rowp[h][k];
          av.re = z.re * rsc[h];
          av.im = z.im * rsc[h];
        }
      }
      As[lk][lr + 16 * h] = av;
      cplx<T> bv = czero<T>();
      if (cok[h] && kok) {
        const cplx<T> g = G[boff[h] + k];
        bv.re = g.re * blam[h];
        bv.im = g.im * blam[h];
      }
      Bs[lk][lr + 16 * h] = bv;
    }
    __syncthreads();
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) {
      const int kk = ks * 4 + grp;
      cmfma<T>(acc, As[kk][wa * 16 + col], Bs[kk][wc * 16 + col]);
    }
    __syncthreads();
  }
  // W rows out; per-sample partial sums over this lane's column, then over the 16 columns
  // of the sub-tile (lanes with equal grp hold the same samples), then over the two waves
  // of a column half
  const int j = j0 + wc * 16 + col;
  double np0[4], np1[4];
  for (int v = 0; v < 4; ++v) {
    const int i = i0 + wa * 16 + Mfma<T>::row(lane, v);
    const T re = acc[0][v], im = acc[1][v];
    if (i < S && j < ncols) {
      cplx<T> z;
      z.re = re;
      z.im = im;
      wout[(size_t)i * a.ldw + j] = z;
    }
    const double w2 = j < ncols ? (double)re * (double)re + (double)im * (double)im : 0.0;
    np0[v] = j < cm ? w2 : 0.0;
    np1[v] = j < cm ? 0.0 : w2;
  }
  for (int v = 0; v < 4; ++v)
    for (int o = 1; o < 16; o <<= 1) {
      np0[v] += __shfl_xor(np0[v], o);
      np1[v] += __shfl_xor(np1[v], o);
    }
  if (col == 0)
    for (int v = 0; v < 4; ++v) {
      const int r = wa * 16 + Mfma<T>::row(lane, v);
      red[wc][r][0] = np0[v];
      red[wc][r][1] = np1[v];
    }
  __syncthreads();
  if (tid < 32) {
    const int i = i0 + tid;
    if (i < S) {
      double* pt = a.part + ((size_t)i * a.ntiles + blockIdx.y) * 2;
      pt[0] = red[0][tid][0] + red[1][tid][0];
      pt[1] = red[0][tid][1] + red[1][tid][1];
    }
  }
}

// Step 2: per sample, p_0 and p_1 summed over the column tiles in order (deterministic),
// bit q = (u_i < p_0 / (p_0 + p_1)) ? 0 : 1 in FP64, the chosen plane and 1 / sqrt(p_bit)
// for the next site.
__global__ __launch_bounds__(256) void sample_decide_kernel(SampleSite a) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.n_samples) return;
  const double* pt = a.part + (size_t)i * a.ntiles * 2;
  double p0 = 0.0, p1 = 0.0;
  for (int t = 0; t < a.ntiles; ++t) {
    p0 += pt[2 * t];
    p1 += pt[2 * t + 1];
  }
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
  // a.ntiles = ceil(2 cm / 32) column tiles; a.part holds n_samples x ntiles x 2 doubles
  const int row_tiles = (a.n_samples + 31) / 32;
  hipLaunchKernelGGL(sample_contract_kernel<T>, dim3(row_tiles, a.ntiles), dim3(256), 0, stream,
                     a);
  hipLaunchKernelGGL(sample_decide_kernel, dim3((a.n_samples + 255) / 256), dim3(256), 0, stream,
                     a);
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
