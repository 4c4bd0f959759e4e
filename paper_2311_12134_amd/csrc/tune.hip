// Autotuning of the blocked LU of Eq. (3) (whose inverse dominates the cost, Sec. II.A):
// every tiling of a trailing update, or both variants of a split-mode panel, is timed on a
// synthetic batch of the shape it will meet, and the caller keeps the fastest.
//   kind 1 (wide): the widest update of an LU with G panels per group, K = G NB over the
//   trailing (npad - G NB)^2 block;
//   kind 0 (narrow): the update of a group's last panel, K = (G - 1) NB over
//   (npad - (G - 1) NB) rows x NB columns;
//   panels: the split-mode panel of a given height (its NB columns only) with 256-thread
//   workgroups and 8-wide leaves against 512-thread workgroups and 16-wide leaves.
// Values are bounded pseudo-random numbers (an integer hash), so repeated updates stay finite.
#include <algorithm>
#include <vector>

#include "lsms_internal.h"

namespace lsms {

template <typename T>
__global__ void tune_fill_kernel(T* a, int64_t n, float scale) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  uint32_t h = (uint32_t)(i * 2654435761ull) ^ (uint32_t)(i >> 32);
  h ^= h >> 15;
  h *= 2246822519u;
  h ^= h >> 13;
  const float u = (float)(h & 0xffff) / 32768.0f - 1.0f, v = (float)(h >> 16) / 32768.0f - 1.0f;
  a[i].x = scale * u;
  a[i].y = scale * v;
}

namespace {
// A synthetic batch of `batch` systems of padded size npad with their job descriptors,
// pivot and status arrays; freed by the destructor.  cols > 0: only the first cols columns
// of each system are stored (leading dimension cols), enough for a panel at k = 0.
struct TuneBatch {
  void* a = nullptr;
  JobDesc* jd = nullptr;
  int32_t* piv = nullptr;
  int32_t* info = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  bool ok = false;
  int64_t per = 0;  // elements per system
  TuneBatch(int npad, int batch, size_t elem, hipStream_t s, int cols = 0) {
    per = (int64_t)npad * (cols > 0 ? cols : npad);
    std::vector<JobDesc> host(batch);
    for (int j = 0; j < batch; ++j) {
      JobDesc d{};
      d.a_off = per * j;
      d.piv_off = piv_ints(npad) * j;
      d.n = npad;
      d.npad = npad;
      d.nl = npad / NL;
      d.ld = cols > 0 ? cols : 0;
      host[j] = d;
    }
    if (hipMalloc(&a, (size_t)(per * batch) * elem) != hipSuccess) return;
    if (hipMalloc((void**)&jd, (size_t)batch * sizeof(JobDesc)) != hipSuccess) return;
    if (hipMalloc((void**)&piv, (size_t)(piv_ints(npad) * batch) * 4) != hipSuccess) return;
    if (hipMalloc((void**)&info, (size_t)batch * 4) != hipSuccess) return;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return;
    if (hipMemcpyAsync(jd, host.data(), host.size() * sizeof(JobDesc), hipMemcpyHostToDevice, s) != hipSuccess)
      return;
    if (hipStreamSynchronize(s) != hipSuccess) return;  // the host staging goes out of scope
    ok = true;
  }
  ~TuneBatch() {
    if (e0) hipEventDestroy(e0);
    if (e1) hipEventDestroy(e1);
    hipFree(info);
    hipFree(piv);
    hipFree(jd);
    hipFree(a);
  }
  // best of three launches of f() (after one warm-up), in ms; < 0 on error
  template <typename F>
  float time(F f, hipStream_t s) {
    f();
    float t = 1e30f;
    for (int rep = 0; rep < 3; ++rep) {
      hipEventRecord(e0, s);
      f();
      hipEventRecord(e1, s);
      float x = 0.f;
      if (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&x, e0, e1) != hipSuccess) return -1.f;
      t = std::min(t, x);
    }
    return t;
  }
};
}  // namespace

int update_autotune(int precision, int kind, int npad, int batch, int group, hipStream_t s, float* ms, int* best) {
  const bool f64 = precision == 0;
  TuneBatch tb(npad, batch, f64 ? sizeof(double2) : sizeof(float2), s);
  if (!tb.ok) return -1;
  const int64_t n = (int64_t)npad * npad * batch;
  if (f64)
    tune_fill_kernel<double2><<<(unsigned)((n + 255) / 256), 256, 0, s>>>((double2*)tb.a, n, 1.0f / (float)npad);
  else
    tune_fill_kernel<float2><<<(unsigned)((n + 255) / 256), 256, 0, s>>>((float2*)tb.a, n, 1.0f / (float)npad);
  const int kd = kind == 1 ? group * NB : (group - 1) * NB;
  const int rows = npad - kd, cols = kind == 1 ? rows : NB, c_end = kind == 1 ? 0 : kd + NB;
  const int nv = f64 ? gemm_f64_variants() : gemm_f32_variants_all();
  *best = -1;
  for (int v = 0; v < nv; ++v) {
    const float t = tb.time(
        [&]() {
          if (f64)
            launch_gemm_f64_variant(v, tb.jd, batch, rows, cols, 0, kd, kd, kd, c_end, (double2*)tb.a, s);
          else
            launch_gemm_f32_any(v, tb.jd, batch, rows, cols, 0, kd, kd, kd, c_end, (float2*)tb.a, s);
        },
        s);
    if (t < 0.f) return -1;
    ms[v] = t;
    if (*best < 0 || t < ms[*best]) *best = v;
  }
  return hipStreamSynchronize(s) == hipSuccess ? 0 : -1;
}

int panel_autotune(int rows, int batch, hipStream_t s, float* ms) {
  TuneBatch tb(rows, batch, sizeof(float2), s, NB);
  if (!tb.ok) return -1;
  const int64_t n = tb.per * batch;
  for (int v = 0; v < 2; ++v) {
    float t = tb.time(
        [&]() {
          // fresh values each launch: the panel factors its columns in place
          tune_fill_kernel<float2><<<(unsigned)((n + 255) / 256), 256, 0, s>>>((float2*)tb.a, n, 1.0f);
          launch_panel_f32_variant(v, tb.jd, batch, rows, (float2*)tb.a, tb.piv, tb.info, s);
        },
        s);
    const float tf = tb.time(
        [&]() { tune_fill_kernel<float2><<<(unsigned)((n + 255) / 256), 256, 0, s>>>((float2*)tb.a, n, 1.0f); }, s);
    if (t < 0.f || tf < 0.f) return -1;
    ms[v] = std::max(t - tf, 0.f);
  }
  return hipStreamSynchronize(s) == hipSuccess ? 0 : -1;
}

}  // namespace lsms
