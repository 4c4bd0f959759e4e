// Autotuning of the split-mode trailing update (the FP32 matrix-core part of the LU of
// Eq. (3)): every tiling times the widest update of an LU (K = 2 NB over the trailing
// (npad - 2 NB)^2 block) on a synthetic batch of that shape.
#include <algorithm>
#include <vector>

#include "lsms_internal.h"

namespace lsms {

__global__ void tune_fill_kernel(float2* a, int64_t n, float scale) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  // a small integer hash gives values in [-scale, scale): finite under repeated updates
  uint32_t h = (uint32_t)(i * 2654435761ull) ^ (uint32_t)(i >> 32);
  h ^= h >> 15;
  h *= 2246822519u;
  h ^= h >> 13;
  const float u = (float)(h & 0xffff) / 32768.0f - 1.0f, v = (float)(h >> 16) / 32768.0f - 1.0f;
  a[i] = make_float2(scale * u, scale * v);
}

int gemm_f32_autotune(int npad, int batch, hipStream_t s, float* ms, int* best) {
  const int64_t per = (int64_t)npad * npad;
  float2* a = nullptr;
  JobDesc* jd = nullptr;
  if (hipMalloc((void**)&a, (size_t)(per * batch) * sizeof(float2)) != hipSuccess) return -1;
  if (hipMalloc((void**)&jd, (size_t)batch * sizeof(JobDesc)) != hipSuccess) {
    hipFree(a);
    return -1;
  }
  int rc = 0;
  std::vector<JobDesc> host(batch);
  for (int j = 0; j < batch; ++j) {
    JobDesc d{};
    d.a_off = per * j;
    d.n = npad;
    d.npad = npad;
    host[j] = d;
  }
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipMemcpyAsync(jd, host.data(), host.size() * sizeof(JobDesc), hipMemcpyHostToDevice, s) != hipSuccess ||
      hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    rc = -1;
  } else {
    const int64_t n = per * batch;
    tune_fill_kernel<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(a, n, 1.0f / (float)npad);
    const int k = 0, kd = 2 * NB, rows = npad - kd;
    *best = -1;
    for (int v = 0; v < gemm_f32_variants() && rc == 0; ++v) {
      launch_gemm_f32(v, jd, batch, rows, rows, k, kd, kd, kd, 0, a, s);  // warm-up
      float t = 1e30f;
      for (int rep = 0; rep < 3; ++rep) {
        hipEventRecord(e0, s);
        launch_gemm_f32(v, jd, batch, rows, rows, k, kd, kd, kd, 0, a, s);
        hipEventRecord(e1, s);
        float x = 0.f;
        if (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&x, e0, e1) != hipSuccess) {
          rc = -1;
          break;
        }
        t = std::min(t, x);
      }
      ms[v] = t;
      if (*best < 0 || t < ms[*best]) *best = v;
    }
  }
  if (e0) hipEventDestroy(e0);
  if (e1) hipEventDestroy(e1);
  hipStreamSynchronize(s);
  hipFree(jd);
  hipFree(a);
  return rc;
}

}  // namespace lsms
