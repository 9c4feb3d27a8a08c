// Bandwidth probe: a plain streaming kernel with the read:write mix of the
// stage kernel (three arrays read for one written), timed with HIP events.
// It is the measured ceiling that the stage kernel's HBM rate is set
// against, beside the chip's published peak.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <string>

#include "dgswe.h"

namespace {

// d[i] = a[i] + b[i] + c[i] (n_read = 3), a[i] + b[i] (2) or a[i] (1), in
// 16-byte vectors; grid-stride, every vector touched once per launch
__global__ __launch_bounds__(256) void stream_kernel(const float4* __restrict__ a, const float4* __restrict__ b,
                                                     const float4* __restrict__ c, float4* __restrict__ d,
                                                     long long n4, int n_read) {
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n4; i += stride) {
    float4 v = a[i];
    if (n_read > 1) {
      const float4 w = b[i];
      v.x += w.x; v.y += w.y; v.z += w.z; v.w += w.w;
    }
    if (n_read > 2) {
      const float4 w = c[i];
      v.x += w.x; v.y += w.y; v.z += w.z; v.w += w.w;
    }
    d[i] = v;
  }
}

}  // namespace

extern "C" int dgswe_stream_probe(int32_t n_read, int64_t bytes, int32_t reps, double* gbs) {
  if (n_read < 1 || n_read > 3 || bytes < 4096 || reps < 1 || !gbs) return DGSWE_EINVAL;
  const long long n4 = bytes / 16;
  float4* buf[4] = {nullptr, nullptr, nullptr, nullptr};
  hipStream_t s = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  int rc = DGSWE_OK;
  auto chk = [&](hipError_t e) {
    if (e != hipSuccess && rc == DGSWE_OK) rc = e == hipErrorOutOfMemory ? DGSWE_ENOMEM : DGSWE_EHIP;
    return e == hipSuccess;
  };
  for (int i = 0; i < n_read + 1 && rc == DGSWE_OK; ++i)
    if (chk(hipMalloc(&buf[i], size_t(n4) * 16))) chk(hipMemset(buf[i], 0, size_t(n4) * 16));
  if (rc == DGSWE_OK) chk(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
  if (rc == DGSWE_OK) chk(hipEventCreate(&e0));
  if (rc == DGSWE_OK) chk(hipEventCreate(&e1));
  if (rc == DGSWE_OK) {
    int dev = 0, cus = 256;
    chk(hipGetDevice(&dev));
    chk(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    const int grid = std::max(1, cus) * 16;
    float4* out = buf[n_read];
    const float4* b = n_read > 1 ? buf[1] : buf[0];
    const float4* c = n_read > 2 ? buf[2] : buf[0];
    hipLaunchKernelGGL(stream_kernel, dim3(grid), dim3(256), 0, s, buf[0], b, c, out, n4, int(n_read));  // warm-up
    chk(hipEventRecord(e0, s));
    for (int r = 0; r < reps; ++r)
      hipLaunchKernelGGL(stream_kernel, dim3(grid), dim3(256), 0, s, buf[0], b, c, out, n4, int(n_read));
    chk(hipGetLastError());
    chk(hipEventRecord(e1, s));
    chk(hipEventSynchronize(e1));
    float ms = 0.f;
    chk(hipEventElapsedTime(&ms, e0, e1));
    if (rc == DGSWE_OK) *gbs = double(n_read + 1) * double(n4) * 16.0 * reps / (double(ms) * 1e-3) / 1e9;
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (s) (void)hipStreamDestroy(s);
  for (auto* p : buf)
    if (p) (void)hipFree(p);
  return rc;
}
