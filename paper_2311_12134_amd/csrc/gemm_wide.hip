// Split-mode trailing update A22 -= L21 U12 (the FP32 matrix-core part of the LU of Eq. (3))
// with workgroups of more than four waves: a TM x TN complex tile per workgroup of
// (TM / 32) x (TN / 32) waves, each wave one 32 x 32 block on FP32 MFMA 16x16x4 with the three
// real products, exactly as tiling 2 of gemm.hip computes it (so every element sums in the
// same order).  A larger tile stages fewer L21 / U12 bytes through LDS per product: (TM + TN)
// x 16 complex per K chunk of 16 for TM x TN x 16 products, against 128 x 16 for 64 x 64.
// K chunks go through two LDS buffers with register prefetch one chunk ahead, or with DEPTH 2
// two chunks ahead through two register sets (one barrier per chunk either way); tiles
// reaching past npad or c_end load zeros there and store nothing; the one-dimensional grid
// is remapped so that consecutive tiles of one job run on the same XCD.
#include "lsms_internal.h"

namespace lsms {

typedef float f4 __attribute__((ext_vector_type(4)));

template <int TM, int TN, int DEPTH, int SWZ = 0>
__global__ __launch_bounds__((TM / 32) * (TN / 32) * 64) void gemm_f32_3m_big(const JobDesc* jobs, int tiles_x,
                                                                                int tiles_y, int k, int kd,
                                                                                int r_begin, int c_begin, int c_end,
                                                                                float2* work) {
  constexpr int KC = 16;
  constexpr int WAVES_N = TN / 32, NT = (TM / 32) * (TN / 32) * 64;
  constexpr int AQ = KC / 4, BQ = TN / 4;  // complex quads per row of the A / B stage
  constexpr int AQN = TM * AQ, BQN = KC * BQ;
  constexpr int AP = (AQN + NT - 1) / NT, BP = (BQN + NT - 1) / NT;
  constexpr int LA = TM + 16, LB = TN + 16;
  int T = blockIdx.x;
  {
    const int N = gridDim.x, q = N >> 3, r = N & 7, x = T & 7;
    T = x * q + min(x, r) + (T >> 3);
  }
  int tx, ty, job;
  if (SWZ > 0) {  // a job's tiles in bands of SWZ tile rows, column by column within a band
    const int tpj = tiles_x * tiles_y;
    job = T / tpj;
    const int u = T - job * tpj;
    const int band = u / (SWZ * tiles_x), rem = u - band * SWZ * tiles_x;
    const int rows = min(SWZ, tiles_y - band * SWZ);
    tx = rem / rows;
    ty = band * SWZ + (rem - tx * rows);
  } else {
    tx = T % tiles_x;
    T /= tiles_x;
    ty = T % tiles_y;
    job = T / tiles_y;
  }
  const JobDesc jd = jobs[job];
  const int row0 = r_begin + ty * TM, col0 = c_begin + tx * TN;
  const int npad = jd.npad;
  const int cmax = c_end > 0 ? min(c_end, npad) : npad;
  if (row0 >= npad || col0 >= cmax) return;  // uniform
  float2* A = work + jd.a_off;
  const int64_t ld = npad;
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int wm = wave / WAVES_N, wn = wave % WAVES_N;
  const bool active = (row0 + wm * 32 < npad) && (col0 + wn * 32 < cmax);
  __shared__ float2 sA[2][KC][LA];
  __shared__ float2 sB[2][KC][LB];
  auto aswz = [](int kk) { return ((kk >> 2) & 3) << 4; };
  float2 ra_[DEPTH][AP][4], rb_[DEPTH][BP][4];
  auto load = [&](int kc, int set) {
    float2(&ra)[AP][4] = ra_[set];
    float2(&rb)[BP][4] = rb_[set];
#pragma unroll
    for (int p = 0; p < AP; ++p) {
      const int q = t + NT * p, i = q / AQ, kk = (q % AQ) * 4, row = row0 + i;
      if (q < AQN && row < npad) {
        const float4* src = (const float4*)(A + (int64_t)row * ld + k + kc + kk);
        const float4 v0 = src[0], v1 = src[1];
        ra[p][0] = make_float2(v0.x, v0.y);
        ra[p][1] = make_float2(v0.z, v0.w);
        ra[p][2] = make_float2(v1.x, v1.y);
        ra[p][3] = make_float2(v1.z, v1.w);
      } else {
#pragma unroll
        for (int u = 0; u < 4; ++u) ra[p][u] = make_float2(0.f, 0.f);
      }
    }
#pragma unroll
    for (int p = 0; p < BP; ++p) {
      const int q = t + NT * p, kk = q / BQ, j = (q % BQ) * 4;
      if (q < BQN && col0 + j < cmax) {
        const float4* src = (const float4*)(A + (int64_t)(k + kc + kk) * ld + col0 + j);
        const float4 v0 = src[0], v1 = src[1];
        rb[p][0] = make_float2(v0.x, v0.y);
        rb[p][1] = make_float2(v0.z, v0.w);
        rb[p][2] = make_float2(v1.x, v1.y);
        rb[p][3] = make_float2(v1.z, v1.w);
      } else {
#pragma unroll
        for (int u = 0; u < 4; ++u) rb[p][u] = make_float2(0.f, 0.f);
      }
    }
  };
  auto store = [&](int buf, int set) {
    float2(&ra)[AP][4] = ra_[set];
    float2(&rb)[BP][4] = rb_[set];
#pragma unroll
    for (int p = 0; p < AP; ++p) {
      const int q = t + NT * p, i = q / AQ, kk = (q % AQ) * 4;
      if (q < AQN) {
#pragma unroll
        for (int u = 0; u < 4; ++u) sA[buf][kk + u][i ^ aswz(kk + u)] = ra[p][u];
      }
    }
#pragma unroll
    for (int p = 0; p < BP; ++p) {
      const int q = t + NT * p, kk = q / BQ, j = (q % BQ) * 4;
      if (q < BQN) {
#pragma unroll
        for (int u = 0; u < 4; ++u) sB[buf][kk][j + u] = rb[p][u];
      }
    }
  };
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
  load(0, 0);
  store(0, 0);
  if (DEPTH == 2 && KC < kd) load(KC, 0);  // chunk 1 in flight during chunk 0
  __syncthreads();
  int cur = 0;
  for (int kc = 0, c = 0; kc < kd; kc += KC, ++c) {
    const bool more = kc + KC < kd;
    if (DEPTH == 1) {
      if (more) load(kc + KC, 0);
    } else if (kc + 2 * KC < kd) {
      load(kc + 2 * KC, (c + 1) & 1);  // chunk c + 2 into the other register set
    }
#pragma unroll
    for (int k4 = 0; k4 < KC; k4 += 4) {
      float2 a[2], b[2];
      float as[2], bs[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        a[i] = sA[cur][k4 + kq][(wm * 32 + i * 16 + ii) ^ aswz(k4)];
        as[i] = a[i].x + a[i].y;
      }
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        b[j] = sB[cur][k4 + kq][wn * 32 + j * 16 + ii];
        bs[j] = b[j].x + b[j].y;
      }
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          t1[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i].x, b[j].x, t1[i][j], 0, 0, 0);
          t2[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i].y, b[j].y, t2[i][j], 0, 0, 0);
          t3[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(as[i], bs[j], t3[i][j], 0, 0, 0);
        }
    }
    if (more) store(cur ^ 1, DEPTH == 1 ? 0 : (c & 1));  // chunk c + 1, loaded a chunk (or two) ago
    __syncthreads();
    cur ^= 1;
  }
  if (!active) return;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int rbase = row0 + wm * 32 + i * 16, cbase = col0 + wn * 32 + j * 16;
      if (rbase < npad && cbase < cmax) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          float2* cp = A + (int64_t)(rbase + 4 * kq + r) * ld + cbase + ii;
          float2 cv = *cp;
          cv.x -= t1[i][j][r] - t2[i][j][r];
          cv.y -= t3[i][j][r] - t1[i][j][r] - t2[i][j][r];
          *cp = cv;
        }
      }
    }
}

template <int TM, int TN, int DEPTH, int SWZ>
void launch_big(const JobDesc* jobs, int njobs, int rows, int cols, int k, int kd, int r_begin, int c_begin,
                int c_end, float2* work, hipStream_t s) {
  const int tx = (cols + TN - 1) / TN, ty = (rows + TM - 1) / TM;
  const int64_t n = (int64_t)tx * ty * njobs;
  gemm_f32_3m_big<TM, TN, DEPTH, SWZ><<<(unsigned)n, (TM / 32) * (TN / 32) * 64, 0, s>>>(jobs, tx, ty, k, kd, r_begin,
                                                                                        c_begin, c_end, work);
}

template void launch_big<128, 64, 1, 0>(const JobDesc*, int, int, int, int, int, int, int, int, float2*, hipStream_t);
template void launch_big<64, 128, 1, 0>(const JobDesc*, int, int, int, int, int, int, int, int, float2*, hipStream_t);
template void launch_big<128, 128, 1, 0>(const JobDesc*, int, int, int, int, int, int, int, int, float2*, hipStream_t);
template void launch_big<64, 64, 2, 0>(const JobDesc*, int, int, int, int, int, int, int, int, float2*, hipStream_t);
template void launch_big<64, 128, 2, 0>(const JobDesc*, int, int, int, int, int, int, int, int, float2*, hipStream_t);
template void launch_big<64, 128, 1, 8>(const JobDesc*, int, int, int, int, int, int, int, int, float2*, hipStream_t);

}  // namespace lsms
