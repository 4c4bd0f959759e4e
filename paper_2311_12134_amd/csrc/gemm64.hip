// Trailing update A22 -= L21 U12 of the FP64-mode blocked LU (the O(n^3) part of the tau
// inverse of Eq. (3)) on the FP64 matrix cores: a family of tilings the autotuner chooses
// from.  Same launch contract as the FP32 family (gemm.hip): for job j the launch updates
// rows [r_begin, npad) x columns [c_begin, c_end) (c_end = 0: to npad) with K = kd columns
// of L starting at column k and the matching kd rows of U; row-major, ld = npad.
//
// TM x TN complex tile per workgroup of four waves, each wave WM x WN as (WM/16) x (WN/16)
// blocks of v_mfma_f64_16x16x4 with the four real products of a complex product
// (re += ar br - ai bi, im += ar bi + ai br: plain FP64 arithmetic, no three-product form).
// K is staged through LDS in chunks of KC with two buffers: the global loads of chunk i+1
// are issued before the products of chunk i and stored to the other buffer after them, so
// one barrier per chunk suffices.  Rows or columns of a tile past npad (or c_end) load as
// zero and are not stored.  With XCD the one-dimensional workgroup index is remapped so
// that consecutive tiles of a job, which read the same L21 and U12 panels, run on the same
// XCD and share its L2.
// v_mfma_f64_16x16x4: A lane l -> (row l%16, k l/16); B lane l -> (k l/16, col l%16);
// D lane l, register r -> (row l/16 + 4r, col l%16).
#include "lsms_internal.h"

namespace lsms {

typedef double d4 __attribute__((ext_vector_type(4)));

// Tiles of up to 64 x 64 are held to four waves per SIMD: left alone the compiler keeps the
// accumulators in AGPRs and ends at three (104 VGPRs + 64 AGPRs); bounded, they fit 111 VGPRs
// with no spills.
template <int TM, int TN, int WM, int WN, bool XCD, int KC>
__global__ __launch_bounds__(256, TM * TN <= 64 * 64 ? 4 : 1) void gemm_f64_tiled(const JobDesc* jobs, int tiles_x,
                                                                                 int tiles_y, int k, int kd,
                                                                                 int r_begin, int c_begin, int c_end,
                                                                                 double2* work) {
  constexpr int WAVES_N = TN / WN;
  static_assert((TM / WM) * (TN / WN) == 4, "four waves per workgroup");
  constexpr int BM = WM / 16, BN = WN / 16;
  constexpr int AQ = KC / 2, BQ = TN / 2;  // complex pairs per row of the A / B stage
  constexpr int AP = (TM * AQ + 255) / 256;  // A passes, one pair per thread and pass
  constexpr int BP = (KC * BQ + 255) / 256;  // B passes
  static_assert((TM * AQ) % 64 == 0 && (KC * BQ) % 64 == 0, "staging in whole wavefronts");
  constexpr int LA = TM + 4, LB = TN + 4;  // LDS row lengths (64-byte offset between k rows)

  int T = blockIdx.x;
  if (XCD) {
    const int N = gridDim.x, q = N >> 3, r = N & 7, x = T & 7;
    T = x * q + min(x, r) + (T >> 3);
  }
  const int tx = T % tiles_x;
  T /= tiles_x;
  const int ty = T % tiles_y;
  const int job = T / tiles_y;
  const JobDesc jd = jobs[job];
  const int row0 = r_begin + ty * TM, col0 = c_begin + tx * TN;
  const int npad = jd.npad;
  const int cmax = c_end > 0 ? min(c_end, npad) : npad;
  if (row0 >= npad || col0 >= cmax) return;  // uniform
  double2* A = work + jd.a_off;
  const int64_t ld = npad;
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int wm = wave / WAVES_N, wn = wave % WAVES_N;

  __shared__ double2 sA[2][KC][LA];  // k-major: the A tile transposed
  __shared__ double2 sB[2][KC][LB];

  // global -> register staging: thread t takes pair t + 256 p of the A stage (row q / AQ,
  // k 2 (q % AQ)) and of the B stage (k q / BQ, column 2 (q % BQ))
  double2 ra[AP][2], rb[BP][2];
  auto load = [&](int kc) {
#pragma unroll
    for (int p = 0; p < AP; ++p) {
      const int q = t + 256 * p, i = q / AQ, kk = (q % AQ) * 2, row = row0 + i;
      if (q >= TM * AQ) break;
      if (row < npad) {
        const double2* src = A + (int64_t)row * ld + k + kc + kk;
        ra[p][0] = src[0];
        ra[p][1] = src[1];
      } else {
        ra[p][0] = ra[p][1] = make_double2(0.0, 0.0);
      }
    }
#pragma unroll
    for (int p = 0; p < BP; ++p) {
      const int q = t + 256 * p, kk = q / BQ, j = (q % BQ) * 2;
      if (q >= KC * BQ) break;
      if (col0 + j < cmax) {
        const double2* src = A + (int64_t)(k + kc + kk) * ld + col0 + j;
        rb[p][0] = src[0];
        rb[p][1] = src[1];
      } else {
        rb[p][0] = rb[p][1] = make_double2(0.0, 0.0);
      }
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int p = 0; p < AP; ++p) {
      const int q = t + 256 * p, i = q / AQ, kk = (q % AQ) * 2;
      if (q >= TM * AQ) break;
      sA[buf][kk][i] = ra[p][0];
      sA[buf][kk + 1][i] = ra[p][1];
    }
#pragma unroll
    for (int p = 0; p < BP; ++p) {
      const int q = t + 256 * p, kk = q / BQ, j = (q % BQ) * 2;
      if (q >= KC * BQ) break;
      sB[buf][kk][j] = rb[p][0];
      sB[buf][kk][j + 1] = rb[p][1];
    }
  };

  d4 are[BM][BN], aim[BM][BN];
#pragma unroll
  for (int i = 0; i < BM; ++i)
#pragma unroll
    for (int j = 0; j < BN; ++j) {
      are[i][j] = d4{0, 0, 0, 0};
      aim[i][j] = d4{0, 0, 0, 0};
    }
  const int ii = lane & 15, kq = lane >> 4;

  load(0);
  store(0);
  __syncthreads();
  int cur = 0;
  for (int kc = 0; kc < kd; kc += KC) {
    const bool more = kc + KC < kd;
    if (more) load(kc + KC);
#pragma unroll
    for (int k4 = 0; k4 < KC; k4 += 4) {
      double2 a[BM], b[BN];
#pragma unroll
      for (int i = 0; i < BM; ++i) a[i] = sA[cur][k4 + kq][wm * WM + i * 16 + ii];
#pragma unroll
      for (int j = 0; j < BN; ++j) b[j] = sB[cur][k4 + kq][wn * WN + j * 16 + ii];
#pragma unroll
      for (int i = 0; i < BM; ++i)
#pragma unroll
        for (int j = 0; j < BN; ++j) {
          are[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i].x, b[j].x, are[i][j], 0, 0, 0);
          are[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(-a[i].y, b[j].y, are[i][j], 0, 0, 0);
          aim[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i].x, b[j].y, aim[i][j], 0, 0, 0);
          aim[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i].y, b[j].x, aim[i][j], 0, 0, 0);
        }
    }
    if (more) store(cur ^ 1);
    __syncthreads();
    cur ^= 1;
  }
#pragma unroll
  for (int i = 0; i < BM; ++i)
#pragma unroll
    for (int j = 0; j < BN; ++j) {
      const int rbase = row0 + wm * WM + i * 16, cbase = col0 + wn * WN + j * 16;
      if (rbase < npad && cbase < cmax) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          double2* cp = A + (int64_t)(rbase + kq + 4 * r) * ld + cbase + ii;
          double2 cv = *cp;
          cv.x -= are[i][j][r];
          cv.y -= aim[i][j][r];
          *cp = cv;
        }
      }
    }
}

template <int TM, int TN, int WM, int WN, bool XCD, int KC>
static void launch_tiled64(const JobDesc* jobs, int njobs, int rows, int cols, int k, int kd, int r_begin,
                           int c_begin, int c_end, double2* work, hipStream_t s) {
  const int tx = (cols + TN - 1) / TN, ty = (rows + TM - 1) / TM;
  const int64_t n = (int64_t)tx * ty * njobs;
  gemm_f64_tiled<TM, TN, WM, WN, XCD, KC><<<(unsigned)n, 256, 0, s>>>(jobs, tx, ty, k, kd, r_begin, c_begin, c_end,
                                                                      work);
}

int gemm_f64_variants() { return 6; }

// 0: the single-buffered 64 x 64 kernel (gemm.hip); 1: 64 x 64, two LDS stages of K = 8, XCD
// order; 2: 32 x 64 (waves of 16 x 32, more workgroups per CU); 3: 128 x 64 (waves of 64 x 32);
// 4: 64 x 128 (waves of 32 x 64); 5: as 1 without the XCD order.
void launch_gemm_f64_variant(int variant, const JobDesc* jobs, int njobs, int rows, int cols, int k, int kd,
                             int r_begin, int c_begin, int c_end, double2* work, hipStream_t s) {
  switch (variant) {
    case 1: launch_tiled64<64, 64, 32, 32, true, 8>(jobs, njobs, rows, cols, k, kd, r_begin, c_begin, c_end, work, s); break;
    case 2: launch_tiled64<32, 64, 16, 32, true, 8>(jobs, njobs, rows, cols, k, kd, r_begin, c_begin, c_end, work, s); break;
    case 3: launch_tiled64<128, 64, 64, 32, true, 8>(jobs, njobs, rows, cols, k, kd, r_begin, c_begin, c_end, work, s); break;
    case 4: launch_tiled64<64, 128, 32, 64, true, 8>(jobs, njobs, rows, cols, k, kd, r_begin, c_begin, c_end, work, s); break;
    case 5: launch_tiled64<64, 64, 32, 32, false, 8>(jobs, njobs, rows, cols, k, kd, r_begin, c_begin, c_end, work, s); break;
    default: launch_gemm_f64(jobs, njobs, rows, cols, k, kd, r_begin, c_begin, c_end, work, s);
  }
}

}  // namespace lsms
