// Peak-rate probes of the device, so that the roofline fractions the library's measurements
// are compared with can be checked against what the chip sustains: streams of independent
// matrix-core instructions (FP64 16x16x4, FP32 16x16x4 and 32x32x2), dependent FP64 vector
// FMAs, and a device-to-device copy.  Each arithmetic launch puts four four-wave workgroups
// on every compute unit (four waves per SIMD, all resident at once, so no workgroup waits for
// a second round); results are summed into one output per thread so nothing is dead code.
#include <algorithm>

#include "lsms_internal.h"

namespace lsms {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef float f16v __attribute__((ext_vector_type(16)));

constexpr int PROBE_CHAINS = 8;

__global__ __launch_bounds__(256) void probe_mfma_f64_kernel(int iters, double* out) {
  const int t = threadIdx.x;
  const double a = 1.0 + 1e-3 * (t & 7), b = 1.0 - 1e-3 * (t & 3);
  d4 acc[PROBE_CHAINS];
#pragma unroll
  for (int c = 0; c < PROBE_CHAINS; ++c) acc[c] = d4{0, 0, 0, 0};
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int c = 0; c < PROBE_CHAINS; ++c) acc[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[c], 0, 0, 0);
  }
  double s = 0.0;
#pragma unroll
  for (int c = 0; c < PROBE_CHAINS; ++c) s += acc[c][0] + acc[c][1] + acc[c][2] + acc[c][3];
  out[blockIdx.x * 256 + t] = s;
}

__global__ __launch_bounds__(256) void probe_mfma_f32_kernel(int iters, double* out) {
  const int t = threadIdx.x;
  const float a = 1.0f + 1e-3f * (t & 7), b = 1.0f - 1e-3f * (t & 3);
  f4 acc[PROBE_CHAINS];
#pragma unroll
  for (int c = 0; c < PROBE_CHAINS; ++c) acc[c] = f4{0, 0, 0, 0};
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int c = 0; c < PROBE_CHAINS; ++c) acc[c] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc[c], 0, 0, 0);
  }
  float s = 0.f;
#pragma unroll
  for (int c = 0; c < PROBE_CHAINS; ++c) s += acc[c][0] + acc[c][1] + acc[c][2] + acc[c][3];
  out[blockIdx.x * 256 + t] = s;
}

__global__ __launch_bounds__(256) void probe_mfma_f32_32_kernel(int iters, double* out) {
  const int t = threadIdx.x;
  const float a = 1.0f + 1e-3f * (t & 7), b = 1.0f - 1e-3f * (t & 3);
  f16v acc[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) acc[c] = f16v{};
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int c = 0; c < 4; ++c) acc[c] = __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, acc[c], 0, 0, 0);
  }
  float s = 0.f;
#pragma unroll
  for (int c = 0; c < 4; ++c)
#pragma unroll
    for (int r = 0; r < 16; ++r) s += acc[c][r];
  out[blockIdx.x * 256 + t] = s;
}

__global__ __launch_bounds__(256) void probe_fma_f64_kernel(int iters, double* out) {
  const int t = threadIdx.x;
  double x[PROBE_CHAINS];
#pragma unroll
  for (int c = 0; c < PROBE_CHAINS; ++c) x[c] = 1.0 + 1e-6 * (t + c);
  const double m = 0.999999, q = 1e-7;
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int c = 0; c < PROBE_CHAINS; ++c) x[c] = fma(x[c], m, q);
  }
  double s = 0.0;
#pragma unroll
  for (int c = 0; c < PROBE_CHAINS; ++c) s += x[c];
  out[blockIdx.x * 256 + t] = s;
}

__global__ __launch_bounds__(256) void probe_copy_kernel(const float4* __restrict__ src, float4* __restrict__ dst,
                                                         int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    dst[i] = src[i];
}

__global__ __launch_bounds__(256) void probe_fill_kernel(float4* __restrict__ dst, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    dst[i] = make_float4((float)i, 0.f, 0.f, 1.f);
}

__global__ __launch_bounds__(256) void probe_read_kernel(const float4* __restrict__ src, int64_t n, float* out) {
  float s = 0.f;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const float4 v = src[i];
    s += v.x + v.y + v.z + v.w;
  }
  if (s == 12345.678f) out[0] = s;  // keeps the loads; never true for the filled values
}

// what: 0 FP64 MFMA 16x16x4, 1 FP32 MFMA 16x16x4, 2 FP32 MFMA 32x32x2 (TFLOP/s), 3 FP64
// vector FMA (TFLOP/s), 4 device-to-device copy of 1 GiB (GB/s, bytes read + written),
// 5 writes of 1 GiB, 6 reads of 1 GiB (GB/s).
// Best of three timed launches after one warm-up; returns 0, or -1 on a HIP error.
int peak_probe(int what, int cu_count, hipStream_t s, double* value) {
  const int blocks = cu_count * 4;
  double* out = nullptr;
  float4* buf = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  int rc = -1;
  const int64_t copy_elems = (1ll << 30) / 16;
  if (hipMalloc((void**)&out, (size_t)blocks * 256 * sizeof(double)) != hipSuccess) return -1;
  if (what >= 4 && hipMalloc((void**)&buf, (size_t)copy_elems * 2 * 16) != hipSuccess) {
    hipFree(out);
    return -1;
  }
  if (hipEventCreate(&e0) == hipSuccess && hipEventCreate(&e1) == hipSuccess) {
    const int iters = what == 3 ? 200000 : 20000;
    auto launch = [&]() {
      switch (what) {
        case 0: probe_mfma_f64_kernel<<<blocks, 256, 0, s>>>(iters, out); break;
        case 1: probe_mfma_f32_kernel<<<blocks, 256, 0, s>>>(iters, out); break;
        case 2: probe_mfma_f32_32_kernel<<<blocks, 256, 0, s>>>(iters, out); break;
        case 3: probe_fma_f64_kernel<<<blocks, 256, 0, s>>>(iters, out); break;
        case 4: probe_copy_kernel<<<cu_count * 16, 256, 0, s>>>(buf, buf + copy_elems, copy_elems); break;
        case 5: probe_fill_kernel<<<cu_count * 16, 256, 0, s>>>(buf, copy_elems); break;
        default: probe_read_kernel<<<cu_count * 16, 256, 0, s>>>(buf, copy_elems, (float*)out);
      }
    };
    // work per launch: waves x iterations x instructions x flops per instruction
    const double waves = (double)blocks * 4;
    double work = 0.0;
    switch (what) {
      case 0: work = waves * iters * PROBE_CHAINS * (2.0 * 16 * 16 * 4); break;
      case 1: work = waves * iters * PROBE_CHAINS * (2.0 * 16 * 16 * 4); break;
      case 2: work = waves * iters * 4 * (2.0 * 32 * 32 * 2); break;
      case 3: work = waves * 64.0 * iters * PROBE_CHAINS * 2.0; break;
      case 4: work = 2.0 * 16.0 * (double)copy_elems; break;
      default: work = 16.0 * (double)copy_elems;
    }
    if (what == 6) probe_fill_kernel<<<cu_count * 16, 256, 0, s>>>(buf, copy_elems);
    launch();
    float best = 1e30f;
    bool ok = hipGetLastError() == hipSuccess;
    for (int rep = 0; rep < 3 && ok; ++rep) {
      hipEventRecord(e0, s);
      launch();
      hipEventRecord(e1, s);
      float ms = 0.f;
      ok = hipEventSynchronize(e1) == hipSuccess && hipEventElapsedTime(&ms, e0, e1) == hipSuccess;
      best = std::min(best, ms);
    }
    if (ok) {
      *value = work / (best * 1e-3) / (what >= 4 ? 1e9 : 1e12);
      rc = 0;
    }
  }
  if (e0) hipEventDestroy(e0);
  if (e1) hipEventDestroy(e1);
  hipStreamSynchronize(s);
  hipFree(buf);
  hipFree(out);
  return rc;
}

}  // namespace lsms
