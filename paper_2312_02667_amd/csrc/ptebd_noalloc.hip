// ptebd_svd_batched_noalloc: the batched Jacobi SVD of ptebd_svd_batched with every device
// buffer (descriptors, work matrices, rotation matrices, per-matrix outputs, the input and
// output staging) carved out of one file-scope device array, `scratch`, instead of hipMalloc.
//
// The array's host-side name is only a stand-in for the symbol: its device address is taken
// once per device with hipGetSymbolAddress (with that device current) and kept in g_scratch;
// every kernel argument and copy below uses that address.  Every call on one device shares
// that device's array, so calls that overlap on one device race; the array keeps the last
// call's contents, and everything a call reads is written by that call first (the input copy,
// the descriptor and load kernels, and jacobi_init for the convergence state and counters).
#include <algorithm>
#include <cstdio>
#include <mutex>

#include "ptebd.h"
#include "ptebd_device.h"
#include "ptebd_internal.h"

namespace {

using ptebd::cplx;
using ptebd::GateDesc;
using ptebd::LayerOut;

__device__ __align__(256) unsigned char scratch[PTEBD_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch[kMaxDevices] = {};

// Device address of this device's scratch array, taken on the first call on the device.
int scratch_address(int dev, void** out) {
  if (dev < 0 || dev >= kMaxDevices)
    return ptebd::report_error(PTEBD_EDEVICE, "device index beyond the scratch table");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return ptebd::report_error(PTEBD_EDEVICE, "hipGetSymbolAddress of the scratch array failed");
    g_scratch[dev] = p;
  }
  *out = g_scratch[dev];
  return PTEBD_OK;
}

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// Byte offsets of the pieces of one call inside the scratch array.
struct Plan {
  size_t desc, out, w, v, a_in, s_out, u_out, vh_out, total;
};

Plan plan_for(size_t celem, int batch, int m, int n) {
  const size_t R = (size_t)(m > n ? m : n), C = (size_t)(m < n ? m : n), b = (size_t)batch;
  Plan p;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off += align256(bytes);
    return o;
  };
  p.desc = take(sizeof(GateDesc) * b);
  p.out = take(ptebd::layer_out_bytes(batch, (int)C));
  p.w = take(celem * R * C * b);
  p.v = take(celem * C * C * b);
  p.a_in = take(16 * (size_t)m * n * b);
  p.s_out = take(sizeof(double) * C * b);
  p.u_out = take(16 * (size_t)m * C * b);
  p.vh_out = take(16 * C * (size_t)n * b);
  p.total = off;
  return p;
}

// One descriptor per matrix: W = a (or a^H when n > m) and V, column-major, no truncation.
__global__ void na_desc_kernel(GateDesc* __restrict__ d, int batch, int R, int C, int tr,
                               char* w_base, char* v_base, size_t w_bytes, size_t v_bytes) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= batch) return;
  GateDesc g;
  g.cl = g.cm = g.cr = 0;
  g.R = R;
  g.C = C;
  g.transposed = tr;
  g.has_gate = 0;
  g.chi_max = 0;
  g.stabilize = 0;
  g.eps_mode = 0;
  g.gq = g.gq1 = nullptr;
  g.lam_l = g.lam_r = nullptr;
  g.lam_m = nullptr;
  g.w = w_base + w_bytes * b;
  g.v = v_base + v_bytes * b;
  g.gate = nullptr;
  g.gram = g.left = nullptr;
  d[b] = g;
}

// a[b] (complex128 row-major m x n) into W[b] (R x C, column-major, precision T):
// W(i, j) = a(i, j) when m >= n, W(j, i) = conj(a(i, j)) otherwise.
template <class T>
__global__ void na_load_kernel(const double* __restrict__ a, int batch, int m, int n, int R,
                               int tr, cplx<T>* __restrict__ w) {
  const size_t per = (size_t)m * n, total = per * batch;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (size_t)gridDim.x * blockDim.x) {
    const size_t b = e / per, r = e % per;
    const int i = (int)(r / n), j = (int)(r % n);
    cplx<T> z;
    z.re = (T)a[2 * e];
    z.im = tr ? (T)(-a[2 * e + 1]) : (T)a[2 * e + 1];
    const size_t dst = tr ? (size_t)i * R + j : (size_t)j * R + i;
    w[b * per + dst] = z;
  }
}

// Singular values and vectors in the caller's layout (as ptebd_svd_batched): s[b, j],
// u[b] row-major m x C, vh[b] row-major C x n, from the sorted columns of W and V.
template <class T>
__global__ void na_extract_kernel(const cplx<T>* __restrict__ w, const cplx<T>* __restrict__ v,
                                  LayerOut out, int batch, int m, int n, int R, int C, int tr,
                                  double* __restrict__ s, double* __restrict__ u,
                                  double* __restrict__ vh) {
  const int b = blockIdx.y;
  const int j = blockIdx.x;
  if (b >= batch || j >= C) return;
  const double sj = out.sig[(size_t)b * C + j];
  const int pj = out.perm[(size_t)b * C + j];
  const double inv = sj > 0 ? 1.0 / sj : 0.0;
  const cplx<T>* wb = w + (size_t)b * R * C;
  const cplx<T>* vb = v + (size_t)b * C * C;
  if (threadIdx.x == 0) s[(size_t)b * C + j] = sj;
  for (int i = threadIdx.x; i < m; i += blockDim.x) {
    double re, im;
    if (!tr) {
      const cplx<T> z = wb[(size_t)pj * R + i];
      re = z.re * inv;
      im = z.im * inv;
    } else {
      const cplx<T> z = vb[(size_t)pj * C + i];
      re = z.re;
      im = z.im;
    }
    const size_t o = 2 * (((size_t)b * m + i) * C + j);
    u[o] = re;
    u[o + 1] = im;
  }
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    double re, im;
    if (!tr) {
      const cplx<T> z = vb[(size_t)pj * C + i];
      re = z.re;
      im = -z.im;
    } else {
      const cplx<T> z = wb[(size_t)pj * R + i];
      re = z.re * inv;
      im = -z.im * inv;
    }
    const size_t o = 2 * (((size_t)b * C + j) * n + i);
    vh[o] = re;
    vh[o + 1] = im;
  }
}

#define NA_HIP(expr)                                                            \
  do {                                                                          \
    if ((expr) != hipSuccess) return ptebd::report_error(PTEBD_EDEVICE, #expr); \
  } while (0)

template <class T>
int svd_noalloc_t(int precision, int batch, int m, int n, const double* a, double* s, double* u,
                  double* vh, int32_t* sweeps, int max_sweeps, double tol_factor,
                  hipStream_t stream, char* base, const Plan& p) {
  const int tr = n > m ? 1 : 0;
  const int R = m > n ? m : n, C = m < n ? m : n;
  const size_t wb = sizeof(cplx<T>) * (size_t)R * C, vb = sizeof(cplx<T>) * (size_t)C * C;
  GateDesc* d = (GateDesc*)(base + p.desc);
  NA_HIP(hipMemcpyAsync(base + p.a_in, a, 16 * (size_t)m * n * batch, hipMemcpyHostToDevice,
                        stream));
  hipLaunchKernelGGL(na_desc_kernel, dim3((batch + 255) / 256), dim3(256), 0, stream, d, batch,
                     R, C, tr, base + p.w, base + p.v, wb, vb);
  const size_t total = (size_t)m * n * batch;
  const int blocks = (int)std::min<size_t>((total + 255) / 256, 4096);
  hipLaunchKernelGGL(na_load_kernel<T>, dim3(blocks), dim3(256), 0, stream,
                     (const double*)(base + p.a_in), batch, m, n, R, tr, (cplx<T>*)(base + p.w));
  NA_HIP(hipGetLastError());
  const LayerOut lo = ptebd::layer_out_at(base + p.out, batch, C);
  int32_t counter = 0;
  int n_unconv = 0;
  // the same schedule as ptebd_svd_batched: one inner sweep, no repeat threshold, sorted pairs
  const int st = ptebd::jacobi_sweeps<T>(stream, d, batch, C, lo, precision, max_sweeps,
                                         tol_factor, 1, 0.0, 1, &counter, &n_unconv);
  if (st < 0) return st;
  ptebd::launch_finalize<T>(d, batch, 0.0, lo, stream);
  double* s_d = (double*)(base + p.s_out);
  double* u_d = (double*)(base + p.u_out);
  double* vh_d = (double*)(base + p.vh_out);
  hipLaunchKernelGGL(na_extract_kernel<T>, dim3(C, batch), dim3(256), 0, stream,
                     (const cplx<T>*)(base + p.w), (const cplx<T>*)(base + p.v), lo, batch, m, n,
                     R, C, tr, s_d, u_d, vh_d);
  NA_HIP(hipGetLastError());
  NA_HIP(hipMemcpyAsync(s, s_d, sizeof(double) * C * (size_t)batch, hipMemcpyDeviceToHost,
                        stream));
  if (u)
    NA_HIP(hipMemcpyAsync(u, u_d, 16 * (size_t)m * C * batch, hipMemcpyDeviceToHost, stream));
  if (vh)
    NA_HIP(hipMemcpyAsync(vh, vh_d, 16 * (size_t)C * n * batch, hipMemcpyDeviceToHost, stream));
  if (sweeps)
    NA_HIP(hipMemcpyAsync(sweeps, lo.sweeps, sizeof(int32_t) * batch, hipMemcpyDeviceToHost,
                          stream));
  NA_HIP(hipStreamSynchronize(stream));
  if (n_unconv > 0) return ptebd::report_error(PTEBD_WNOCONV, "some SVDs reached the sweep cap");
  return PTEBD_OK;
}

}  // namespace

extern "C" int ptebd_svd_batched_noalloc(int precision, int batch, int m, int n, const double* a,
                                         double* s, double* u, double* vh, int32_t* sweeps,
                                         int max_sweeps, double tol_factor, void* hip_stream) {
  if (precision == PTEBD_BF16X3)
    return ptebd::report_error(PTEBD_EINVAL,
                               "PTEBD_BF16X3 is not built in this library (use PTEBD_FP32)");
  if (precision != PTEBD_FP64 && precision != PTEBD_FP32)
    return ptebd::report_error(PTEBD_EINVAL, "bad precision");
  if (batch < 1 || m < 1 || n < 1 || (m < n ? m : n) > 1024 || batch > 65535)
    return ptebd::report_error(PTEBD_EINVAL,
                               "bad sizes (batch in [1, 65535], min(m, n) <= 1024)");
  if (!a || !s) return ptebd::report_error(PTEBD_EINVAL, "null input / output");
  if (max_sweeps < 1 || !(tol_factor > 0.0))
    return ptebd::report_error(PTEBD_EINVAL, "bad sweep controls");
  const size_t celem = precision == PTEBD_FP64 ? sizeof(cplx<double>) : sizeof(cplx<float>);
  const Plan p = plan_for(celem, batch, m, n);
  if (p.total > (size_t)PTEBD_NOALLOC_SCRATCH_BYTES) {
    char msg[160];
    std::snprintf(msg, sizeof(msg),
                  "batch needs %zu bytes of scratch, more than the %zu of the allocation-free "
                  "array (PTEBD_NOALLOC_SCRATCH_BYTES)",
                  p.total, (size_t)PTEBD_NOALLOC_SCRATCH_BYTES);
    return ptebd::report_error(PTEBD_EINVAL, msg);
  }
  const size_t cnt = 2 * (size_t)batch * m * n;
  for (size_t i = 0; i < cnt; ++i)
    if (!(a[i] - a[i] == 0.0)) return ptebd::report_error(PTEBD_EINVAL, "non-finite input");
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return ptebd::report_error(PTEBD_EDEVICE, "no HIP device");
  void* base = nullptr;
  const int st = scratch_address(dev, &base);
  if (st < 0) return st;
  if (precision == PTEBD_FP64)
    return svd_noalloc_t<double>(precision, batch, m, n, a, s, u, vh, sweeps, max_sweeps,
                                 tol_factor, (hipStream_t)hip_stream, (char*)base, p);
  return svd_noalloc_t<float>(precision, batch, m, n, a, s, u, vh, sweeps, max_sweeps,
                              tol_factor, (hipStream_t)hip_stream, (char*)base, p);
}
