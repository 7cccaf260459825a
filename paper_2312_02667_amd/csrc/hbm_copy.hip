// Plain device copy of a known size, the reference for the HBM byte counters (FETCH_SIZE,
// WRITE_SIZE) that measure the layer kernels' traffic: a profiler pass that covers one
// hbm_copy_kernel dispatch of B bytes reads B bytes and writes B bytes, so what the counters
// report for it fixes their unit.  Built as its own library (libhbmcopy.so), apart from the
// pTEBD library: it is measurement support, not part of the layer's path.
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace {

__global__ __launch_bounds__(256) void hbm_copy_kernel(const float4* __restrict__ src,
                                                        float4* __restrict__ dst, size_t n) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
    dst[i] = src[i];
}

__global__ __launch_bounds__(256) void hbm_fill_kernel(float4* __restrict__ dst, size_t n) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
    dst[i] = make_float4(1.f, 2.f, 3.f, 4.f);
}

}  // namespace

// Allocate two buffers of `mib` MiB on the current device, fill the source, then run `reps`
// copies of it into the destination (each dispatch reads and writes mib MiB) and free both.
// Returns 0, -1 for bad arguments (mib outside [1, 65536], reps outside [1, 100]) or the HIP
// error code of the failing call.
extern "C" int hbm_copy_run(int mib, int reps) {
  if (mib < 1 || mib > 65536 || reps < 1 || reps > 100) return -1;
  const size_t bytes = (size_t)mib << 20;
  const size_t n = bytes / sizeof(float4);
  float4* src = nullptr;
  float4* dst = nullptr;
  hipError_t e = hipMalloc((void**)&src, bytes);
  if (e != hipSuccess) return (int)e;
  e = hipMalloc((void**)&dst, bytes);
  if (e != hipSuccess) {
    (void)hipFree(src);
    return (int)e;
  }
  const int blocks = 8192;  // 32 per CU over 256 CUs, grid-stride over the rest
  hipLaunchKernelGGL(hbm_fill_kernel, dim3(blocks), dim3(256), 0, nullptr, src, n);
  for (int r = 0; r < reps; ++r)
    hipLaunchKernelGGL(hbm_copy_kernel, dim3(blocks), dim3(256), 0, nullptr, src, dst, n);
  e = hipGetLastError();
  if (e == hipSuccess) e = hipDeviceSynchronize();
  (void)hipFree(src);
  (void)hipFree(dst);
  return (int)e;
}
