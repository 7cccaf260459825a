// FP64 kernels behind the exact queries (norm, overlap, <Z>, canonical distance): a small
// column-major complex GEMM, the Lambda-scaled site tensor in FP64, and two reductions.
// The queries are sequential transfer-matrix sweeps over the sites (the quantum-map
// recursion used in the proof of Lemma 2, with no projectors), off the hot path.
#include "ptebd_internal.h"

namespace ptebd {
namespace {

__device__ inline cplx<double> cmul(cplx<double> a, cplx<double> b) {
  cplx<double> r;
  r.re = a.re * b.re - a.im * b.im;
  r.im = a.re * b.im + a.im * b.re;
  return r;
}

__device__ inline cplx<double> load_op(const cplx<double>* p, int ld, char op, int i, int j,
                                       int rows, int cols) {
  // element (i, j) of op(P), op(P) is rows x cols
  cplx<double> z;
  z.re = 0.0;
  z.im = 0.0;
  if (i >= rows || j >= cols) return z;
  if (op == 'N') return p[(size_t)j * ld + i];
  z = p[(size_t)i * ld + j];
  if (op == 'C') z.im = -z.im;
  return z;
}

__global__ __launch_bounds__(256) void zgemm_kernel(char opa, char opb, int m, int n, int k,
                                                    double alpha, const cplx<double>* a,
                                                    int lda, const cplx<double>* b, int ldb,
                                                    double beta, cplx<double>* c, int ldc) {
  __shared__ cplx<double> As[16][17];
  __shared__ cplx<double> Bs[16][17];
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  const int i0 = blockIdx.x * 16, j0 = blockIdx.y * 16;
  cplx<double> acc;
  acc.re = 0.0;
  acc.im = 0.0;
  for (int k0 = 0; k0 < k; k0 += 16) {
    As[ty][tx] = load_op(a, lda, opa, i0 + tx, k0 + ty, m, k);
    Bs[ty][tx] = load_op(b, ldb, opb, k0 + tx, j0 + ty, k, n);
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < 16; ++kk) {
      const cplx<double> p = cmul(As[kk][tx], Bs[ty][kk]);
      acc.re += p.re;
      acc.im += p.im;
    }
    __syncthreads();
  }
  const int i = i0 + tx, j = j0 + ty;
  if (i < m && j < n) {
    cplx<double>* dst = c + (size_t)j * ldc + i;
    cplx<double> r;
    r.re = alpha * acc.re;
    r.im = alpha * acc.im;
    if (beta != 0.0) {
      r.re += beta * dst->re;
      r.im += beta * dst->im;
    }
    *dst = r;
  }
}

template <class T>
__global__ void site_a_kernel(const cplx<T>* __restrict__ gamma, const double* lam_left,
                              const double* lam_right, int cl, int cm, double sl, double sr,
                              cplx<double>* __restrict__ out) {
  const size_t total = 2 * (size_t)cl * cm;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (size_t)gridDim.x * blockDim.x) {
    const int a = (int)(e % cl);
    const int m = (int)((e / cl) % cm);
    double sc = sl * sr;
    if (lam_left) sc *= lam_left[a];
    if (lam_right) sc *= lam_right[m];
    const cplx<T> g = gamma[e];
    cplx<double> z;
    z.re = (double)g.re * sc;
    z.im = (double)g.im * sc;
    out[e] = z;
  }
}

// out[0] = sum_ij |x_ij - delta_ij|^2 over an n x n matrix (one workgroup, fixed order).
__global__ __launch_bounds__(1024) void frob_minus_identity_kernel(const cplx<double>* x, int n,
                                                                   double* out) {
  __shared__ double red[1024];
  double s = 0.0;
  const size_t total = (size_t)n * n;
  for (size_t e = threadIdx.x; e < total; e += 1024) {
    const size_t i = e % n, j = e / n;
    const double re = x[e].re - (i == j ? 1.0 : 0.0), im = x[e].im;
    s += re * re + im * im;
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int o = 512; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = red[0];
}

// out[0] += weight * Re sum_i conj(a_i) b_i (one workgroup, fixed order).
__global__ __launch_bounds__(1024) void dot_conj_kernel(const cplx<double>* a,
                                                        const cplx<double>* b, int count,
                                                        double weight, double* out) {
  __shared__ double red[1024];
  double s = 0.0;
  for (int e = threadIdx.x; e < count; e += 1024) s += a[e].re * b[e].re + a[e].im * b[e].im;
  red[threadIdx.x] = s;
  __syncthreads();
  for (int o = 512; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] += weight * red[0];
}

__global__ void set_scalar_kernel(cplx<double>* x, double value) {
  x[0].re = value;
  x[0].im = 0.0;
}

}  // namespace

void launch_zgemm(char opa, char opb, int m, int n, int k, double alpha_re,
                  const cplx<double>* a, int lda, const cplx<double>* b, int ldb,
                  double beta_re, cplx<double>* c, int ldc, hipStream_t stream) {
  if (m <= 0 || n <= 0) return;
  dim3 grid((m + 15) / 16, (n + 15) / 16);
  hipLaunchKernelGGL(zgemm_kernel, grid, dim3(256), 0, stream, opa, opb, m, n, k, alpha_re, a,
                     lda, b, ldb, beta_re, c, ldc);
}

template <class T>
void launch_site_a(const void* gamma, const double* lam_left, const double* lam_right, int cl,
                   int cm, double scale_left, double scale_right, cplx<double>* out,
                   hipStream_t stream) {
  const size_t total = 2 * (size_t)cl * cm;
  int blocks = (int)((total + 255) / 256);
  if (blocks > 1024) blocks = 1024;
  hipLaunchKernelGGL(site_a_kernel<T>, dim3(blocks), dim3(256), 0, stream,
                     (const cplx<T>*)gamma, lam_left, lam_right, cl, cm, scale_left,
                     scale_right, out);
}

void launch_frob_minus_identity(const cplx<double>* x, int n, double* out, hipStream_t stream) {
  hipLaunchKernelGGL(frob_minus_identity_kernel, dim3(1), dim3(1024), 0, stream, x, n, out);
}

void launch_dot_conj(const cplx<double>* a, const cplx<double>* b, int count, double weight,
                     double* out_re, hipStream_t stream) {
  hipLaunchKernelGGL(dot_conj_kernel, dim3(1), dim3(1024), 0, stream, a, b, count, weight,
                     out_re);
}

void launch_set_identity_scalar(cplx<double>* x, double value, hipStream_t stream) {
  hipLaunchKernelGGL(set_scalar_kernel, dim3(1), dim3(1), 0, stream, x, value);
}

template void launch_site_a<float>(const void*, const double*, const double*, int, int, double,
                                   double, cplx<double>*, hipStream_t);
template void launch_site_a<double>(const void*, const double*, const double*, int, int, double,
                                    double, cplx<double>*, hipStream_t);

}  // namespace ptebd

namespace ptebd {
namespace {
template <class T>
__global__ void init_product_kernel(char* gamma_base, const size_t* gamma_offsets, int n_sites,
                                    double* lam_base, const size_t* lam_offsets, int n_bonds) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n_sites) {
    cplx<T>* g = (cplx<T>*)(gamma_base + gamma_offsets[i]);
    g[0].re = T(1);
    g[0].im = T(0);
    g[1].re = T(0);
    g[1].im = T(0);
  }
  if (i < n_bonds) lam_base[lam_offsets[i]] = 1.0;
}
}  // namespace

// |0...0>: Gamma[q] = e_0 (shape 1 x 2 x 1) at every listed slot, Lambda = (1) at every
// listed bond slot.  Offsets: bytes for Gamma slots, doubles for Lambda slots.
template <class T>
void launch_init_product(void* gamma_base, const size_t* d_gamma_offsets, int n_sites,
                         double* lam_base, const size_t* d_lam_offsets, int n_bonds,
                         hipStream_t stream) {
  const int n = n_sites > n_bonds ? n_sites : n_bonds;
  if (n <= 0) return;
  hipLaunchKernelGGL(init_product_kernel<T>, dim3((n + 255) / 256), dim3(256), 0, stream,
                     (char*)gamma_base, d_gamma_offsets, n_sites, lam_base, d_lam_offsets,
                     n_bonds);
}
template void launch_init_product<float>(void*, const size_t*, int, double*, const size_t*, int,
                                         hipStream_t);
template void launch_init_product<double>(void*, const size_t*, int, double*, const size_t*, int,
                                          hipStream_t);
}  // namespace ptebd
