// Trailing update A22 -= L21 U12 of the blocked LU (the O(n^3) part of the tau inverse
// of Eq. (3)) on the matrix cores, batched over the jobs of a wave.
//
// For job j the launch updates rows [r_begin, npad) x columns [c_begin, c_end) (c_end = 0:
// to npad) with K = kd columns of L starting at column k and the matching kd rows of U.
// Storage is row-major, leading dimension npad, complex interleaved.
#include "lsms_internal.h"

namespace lsms {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

// ------------------------------------------------------------------------------------
// trailing update A22 -= L21 U12, FP64 MFMA (4 real products per complex product)
// 64 x 64 complex tile per workgroup, 4 waves of 32 x 32, K = NB in chunks of 16.
// v_mfma_f64_16x16x4: A lane l -> (row l%16, k l/16); B lane l -> (k l/16, col l%16);
// D lane l, register r -> (row l/16 + 4r, col l%16).
// ------------------------------------------------------------------------------------
__global__ __launch_bounds__(256) void gemm_f64_kernel(const JobDesc* jobs, int k, int kd, int r_begin, int c_begin,
                                                   int c_end, double2* work) {
  const JobDesc jd = jobs[blockIdx.z];
  const int row0 = r_begin + blockIdx.y * 64, col0 = c_begin + blockIdx.x * 64;
  if (row0 >= jd.npad || col0 >= jd.npad || (c_end > 0 && col0 >= c_end)) return;  // uniform
  double2* A = work + jd.a_off;
  const int64_t ld = jd.npad;
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int wr = wave >> 1, wc = wave & 1;
  __shared__ double2 sA[16][64 + 1];
  __shared__ double2 sB[16][64 + 1];
  d4 are[2][2], aim[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      are[i][j] = d4{0, 0, 0, 0};
      aim[i][j] = d4{0, 0, 0, 0};
    }
  const int ii = lane & 15, kq = lane >> 4;
  for (int kc = 0; kc < kd; kc += 16) {
    {
      const int i = t >> 2, k4 = (t & 3) * 4;
      const double2* src = A + (row0 + i) * ld + k + kc + k4;
#pragma unroll
      for (int u = 0; u < 4; ++u) sA[k4 + u][i] = src[u];
      const int kk = t >> 4, j4 = (t & 15) * 4;
      const double2* srb = A + (k + kc + kk) * ld + col0 + j4;
#pragma unroll
      for (int u = 0; u < 4; ++u) sB[kk][j4 + u] = srb[u];
    }
    __syncthreads();
#pragma unroll
    for (int k4 = 0; k4 < 16; k4 += 4) {
      double2 a[2], b[2];
#pragma unroll
      for (int rb = 0; rb < 2; ++rb) a[rb] = sA[k4 + kq][wr * 32 + rb * 16 + ii];
#pragma unroll
      for (int cb = 0; cb < 2; ++cb) b[cb] = sB[k4 + kq][wc * 32 + cb * 16 + ii];
#pragma unroll
      for (int rb = 0; rb < 2; ++rb)
#pragma unroll
        for (int cb = 0; cb < 2; ++cb) {
          are[rb][cb] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[rb].x, b[cb].x, are[rb][cb], 0, 0, 0);
          are[rb][cb] = __builtin_amdgcn_mfma_f64_16x16x4f64(-a[rb].y, b[cb].y, are[rb][cb], 0, 0, 0);
          aim[rb][cb] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[rb].x, b[cb].y, aim[rb][cb], 0, 0, 0);
          aim[rb][cb] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[rb].y, b[cb].x, aim[rb][cb], 0, 0, 0);
        }
    }
    __syncthreads();
  }
#pragma unroll
  for (int rb = 0; rb < 2; ++rb)
#pragma unroll
    for (int cb = 0; cb < 2; ++cb)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = row0 + wr * 32 + rb * 16 + kq + 4 * r;
        const int col = col0 + wc * 32 + cb * 16 + ii;
        double2* cp = A + row * ld + col;
        double2 cv = *cp;
        cv.x -= are[rb][cb][r];
        cv.y -= aim[rb][cb][r];
        *cp = cv;
      }
}

// ------------------------------------------------------------------------------------
// trailing update, split mode: FP32 storage, FP32 MFMA with three real products.
// v_mfma_f32_16x16x4: A lane l -> (row l%16, k l/16); B lane l -> (k l/16, col l%16);
// D lane l, register r -> (row 4(l/16) + r, col l%16).
// ------------------------------------------------------------------------------------
__global__ __launch_bounds__(256) void gemm_f32_3m_kernel(const JobDesc* jobs, int k, int kd, int r_begin, int c_begin,
                                                   int c_end, float2* work) {
  const JobDesc jd = jobs[blockIdx.z];
  const int row0 = r_begin + blockIdx.y * 64, col0 = c_begin + blockIdx.x * 64;
  if (row0 >= jd.npad || col0 >= jd.npad || (c_end > 0 && col0 >= c_end)) return;  // uniform
  float2* A = work + jd.a_off;
  const int64_t ld = jd.npad;
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int wr = wave >> 1, wc = wave & 1;
  __shared__ float2 sA[16][64 + 1];
  __shared__ float2 sB[16][64 + 1];
  f4 t1[2][2], t2[2][2], t3[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      t1[i][j] = f4{0, 0, 0, 0};
      t2[i][j] = f4{0, 0, 0, 0};
      t3[i][j] = f4{0, 0, 0, 0};
    }
  const int ii = lane & 15, kq = lane >> 4;
  for (int kc = 0; kc < kd; kc += 16) {
    {
      const int i = t >> 2, k4 = (t & 3) * 4;
      const float2* src = A + (row0 + i) * ld + k + kc + k4;
#pragma unroll
      for (int u = 0; u < 4; ++u) sA[k4 + u][i] = src[u];
      const int kk = t >> 4, j4 = (t & 15) * 4;
      const float2* srb = A + (k + kc + kk) * ld + col0 + j4;
#pragma unroll
      for (int u = 0; u < 4; ++u) sB[kk][j4 + u] = srb[u];
    }
    __syncthreads();
#pragma unroll
    for (int k4 = 0; k4 < 16; k4 += 4) {
      float2 a[2], b[2];
#pragma unroll
      for (int rb = 0; rb < 2; ++rb) a[rb] = sA[k4 + kq][wr * 32 + rb * 16 + ii];
#pragma unroll
      for (int cb = 0; cb < 2; ++cb) b[cb] = sB[k4 + kq][wc * 32 + cb * 16 + ii];
#pragma unroll
      for (int rb = 0; rb < 2; ++rb)
#pragma unroll
        for (int cb = 0; cb < 2; ++cb) {
          t1[rb][cb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[rb].x, b[cb].x, t1[rb][cb], 0, 0, 0);
          t2[rb][cb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[rb].y, b[cb].y, t2[rb][cb], 0, 0, 0);
          t3[rb][cb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[rb].x + a[rb].y, b[cb].x + b[cb].y, t3[rb][cb],
                                                            0, 0, 0);
        }
    }
    __syncthreads();
  }
#pragma unroll
  for (int rb = 0; rb < 2; ++rb)
#pragma unroll
    for (int cb = 0; cb < 2; ++cb)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = row0 + wr * 32 + rb * 16 + 4 * kq + r;
        const int col = col0 + wc * 32 + cb * 16 + ii;
        float2* cp = A + row * ld + col;
        float2 cv = *cp;
        cv.x -= t1[rb][cb][r] - t2[rb][cb][r];
        cv.y -= t3[rb][cb][r] - t1[rb][cb][r] - t2[rb][cb][r];
        *cp = cv;
      }
}

void launch_gemm_f64(dim3 grid, const JobDesc* jobs, int k, int kd, int r_begin, int c_begin, int c_end,
                     double2* work, hipStream_t s) {
  gemm_f64_kernel<<<grid, 256, 0, s>>>(jobs, k, kd, r_begin, c_begin, c_end, work);
}

void launch_gemm_f32(dim3 grid, const JobDesc* jobs, int k, int kd, int r_begin, int c_begin, int c_end,
                     float2* work, hipStream_t s) {
  gemm_f32_3m_kernel<<<grid, 256, 0, s>>>(jobs, k, kd, r_begin, c_begin, c_end, work);
}

}  // namespace lsms
