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

// ------------------------------------------------------------------------------------
// split-mode trailing update, tiled family.  TM x TN complex tile per workgroup of four
// waves, each wave a WM x WN sub-tile of (WM/16) x (WN/16) blocks on FP32 MFMA 16x16x4 with
// the three real products.  K is staged through LDS in chunks of 16 with two buffers: the
// global loads of chunk i+1 are issued before the MFMAs of chunk i and written to the other
// buffer after them, so one barrier per chunk suffices and the load latency overlaps the
// matrix-core work.  Tiles may reach past npad by 64 rows or columns (npad is a multiple of
// 64): those rows and columns load as zero (their MFMAs run on zeros, so the accumulators
// never pass through a branch) and nothing is stored there.  The grid is one-dimensional over (job, tile row, tile column); with
// XCD = true the workgroup index is remapped so that consecutive tiles of one job, which
// share L21 and U12 panels, run on the same XCD (workgroups are dealt to the eight XCDs
// round-robin) and hit the same L2.
// ------------------------------------------------------------------------------------
template <int TM, int TN, int WM, int WN, bool XCD, int KC = 16, bool PFC = false, bool TRI = false, bool M32 = false,
          int SWZ = 0>
__global__ __launch_bounds__(256) void gemm_f32_3m_tiled(const JobDesc* jobs, int tiles_x, int tiles_y, int k, int kd,
                                                         int r_begin, int c_begin, int c_end, float2* work) {
  // KC: K chunk per LDS stage.  PFC: the wave's C elements are loaded two chunks before
  // the end, so their latency overlaps the last chunks' MFMAs instead of the epilogue.
  // TRI: only the tiles on and below the diagonal of the (square) updated block, numbered
  // row by row (tile row y holds y + 1 tiles) -- the symmetric factorization's update.
  // M32: each wave's 32 x 32 block on FP32 MFMA 32x32x2 (three 32 x 32 real products, two
  // k per step; A lane l -> (row l%32, k l/32), B lane l -> (k l/32, column l%32), D lane l,
  // register r -> (row 8(r/4) + 4(l/32) + r%4, column l%32)): half the MFMA instructions.
  // SWZ > 0: a job's tiles are numbered in bands of SWZ tile rows, column by column within a
  // band, so the workgroups resident on one XCD at a time (consecutive numbers) cover a
  // SWZ-row by (resident / SWZ)-column block and read SWZ row panels of L21 and that many
  // column panels of U12, which stay in the XCD's L2 while K grows (row by row, a block
  // of four tile rows needs every column panel of U12).
  constexpr int WAVES_N = TN / WN;
  static_assert((TM / WM) * (TN / WN) == 4, "four waves per workgroup");
  constexpr int BM = WM / 16, BN = WN / 16;
  constexpr int AQ = KC / 4, BQ = TN / 4;  // complex quads per row of the A / B stage
  constexpr int AP = TM * AQ / 256;      // A passes, one quad per thread and pass
  constexpr int BP = KC * BQ / 256;      // B passes
  constexpr int LA = TM + 16, LB = TN + 16;  // LDS row lengths (k-step offset of 32 banks)

  int T = blockIdx.x;
  if (XCD) {
    const int N = gridDim.x, q = N >> 3, r = N & 7, x = T & 7;
    T = x * q + min(x, r) + (T >> 3);
  }
  int tx, ty, job;
  if (TRI) {
    const int per = tiles_y * (tiles_y + 1) / 2, u = T % per;
    job = T / per;
    int y = (int)((sqrtf(8.0f * (float)u + 1.0f) - 1.0f) * 0.5f);
    while (y * (y + 1) / 2 > u) --y;
    while ((y + 1) * (y + 2) / 2 <= u) ++y;
    ty = y;
    tx = u - y * (y + 1) / 2;
  } else if (SWZ > 0) {
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
  const bool active = (row0 + wm * WM < npad) && (col0 + wn * WN < cmax);

  __shared__ float2 sA[2][KC][LA];
  __shared__ float2 sB[2][KC][LB];
  // A is stored transposed (k-major): the four k-quads a wavefront writes would hit the
  // same LDS banks, so rows are XOR-swizzled by 16 (k / 4); all four k of one MFMA step
  // share the swizzle, so the 16 rows a read touches stay consecutive
  auto aswz = [](int kk) { return ((kk >> 2) & 3) << 4; };

  // global -> register staging of one chunk: thread t takes quad t + 256 p of the A stage
  // (row q / AQ, k 4 (q % AQ)) and of the B stage (k q / BQ, column 4 (q % BQ))
  float2 ra[AP][4], rb[BP][4];
  auto load = [&](int kc) {
#pragma unroll
    for (int p = 0; p < AP; ++p) {
      const int q = t + 256 * p, i = q / AQ, kk = (q % AQ) * 4, row = row0 + i;
      if (row < npad) {
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
      const int q = t + 256 * p, kk = q / BQ, j = (q % BQ) * 4;
      if (col0 + j < cmax) {
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
  auto store = [&](int buf) {
#pragma unroll
    for (int p = 0; p < AP; ++p) {
      const int q = t + 256 * p, i = q / AQ, kk = (q % AQ) * 4;
#pragma unroll
      for (int u = 0; u < 4; ++u) sA[buf][kk + u][i ^ aswz(kk + u)] = ra[p][u];
    }
#pragma unroll
    for (int p = 0; p < BP; ++p) {
      const int q = t + 256 * p, kk = q / BQ, j = (q % BQ) * 4;
#pragma unroll
      for (int u = 0; u < 4; ++u) sB[buf][kk][j + u] = rb[p][u];
    }
  };

  static_assert(!M32 || (WM == 32 && WN == 32 && !PFC), "32x32x2 form: one 32 x 32 block per wave");
  typedef float f16v __attribute__((ext_vector_type(16)));
  constexpr int BM_ = M32 ? 1 : BM, BN_ = M32 ? 1 : BN;
  f4 t1[BM_][BN_], t2[BM_][BN_], t3[BM_][BN_];
  f16v u1, u2, u3;  // the 32x32x2 form's accumulators
#pragma unroll
  for (int i = 0; i < BM_; ++i)
#pragma unroll
    for (int j = 0; j < BN_; ++j) {
      t1[i][j] = f4{0, 0, 0, 0};
      t2[i][j] = f4{0, 0, 0, 0};
      t3[i][j] = f4{0, 0, 0, 0};
    }
  u1 = f16v{};
  u2 = f16v{};
  u3 = f16v{};
  const int ii = lane & 15, kq = lane >> 4;

  load(0);
  store(0);
  __syncthreads();
  int cur = 0;
  float2 cpre[PFC ? BM : 1][PFC ? BN : 1][4];
  auto load_c = [&]() {
#pragma unroll
    for (int i = 0; i < BM; ++i)
#pragma unroll
      for (int j = 0; j < BN; ++j) {
        const int rbase = row0 + wm * WM + i * 16, cbase = col0 + wn * WN + j * 16;
        const bool ok = rbase < npad && cbase < cmax;
#pragma unroll
        for (int r = 0; r < 4; ++r)
          cpre[PFC ? i : 0][PFC ? j : 0][r] =
              ok ? A[(int64_t)(rbase + 4 * kq + r) * ld + cbase + ii] : make_float2(0.f, 0.f);
      }
  };
  for (int kc = 0; kc < kd; kc += KC) {
    const bool more = kc + KC < kd;
    if (more) load(kc + KC);
    if (PFC && kc == (kd > 2 * KC ? kd - 2 * KC : 0)) load_c();
    if constexpr (M32) {
#pragma unroll
      for (int k2 = 0; k2 < KC; k2 += 2) {
        const int kk = k2 + (lane >> 5), i32 = lane & 31;
        const float2 a = sA[cur][kk][(wm * WM + i32) ^ aswz(kk)];
        const float2 b = sB[cur][kk][wn * WN + i32];
        u1 = __builtin_amdgcn_mfma_f32_32x32x2f32(a.x, b.x, u1, 0, 0, 0);
        u2 = __builtin_amdgcn_mfma_f32_32x32x2f32(a.y, b.y, u2, 0, 0, 0);
        u3 = __builtin_amdgcn_mfma_f32_32x32x2f32(a.x + a.y, b.x + b.y, u3, 0, 0, 0);
      }
    } else
#pragma unroll
    for (int k4 = 0; k4 < KC; k4 += 4) {
      float2 a[BM], b[BN];
      float as[BM], bs[BN];
#pragma unroll
      for (int i = 0; i < BM; ++i) {
        a[i] = sA[cur][k4 + kq][(wm * WM + i * 16 + ii) ^ aswz(k4)];
        as[i] = a[i].x + a[i].y;
      }
#pragma unroll
      for (int j = 0; j < BN; ++j) {
        b[j] = sB[cur][k4 + kq][wn * WN + j * 16 + ii];
        bs[j] = b[j].x + b[j].y;
      }
#pragma unroll
      for (int i = 0; i < BM; ++i)
#pragma unroll
        for (int j = 0; j < BN; ++j) {
          t1[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i].x, b[j].x, t1[i][j], 0, 0, 0);
          t2[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i].y, b[j].y, t2[i][j], 0, 0, 0);
          t3[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(as[i], bs[j], t3[i][j], 0, 0, 0);
        }
    }
    if (more) store(cur ^ 1);
    __syncthreads();
    cur ^= 1;
  }
  if (!active) return;
  if constexpr (M32) {
    const int rbase = row0 + wm * WM, cbase = col0 + wn * WN + (lane & 31);
    if (cbase < cmax) {
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int row = rbase + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
        if (row < npad) {
          float2* cp = A + (int64_t)row * ld + cbase;
          float2 cv = *cp;
          cv.x -= u1[r] - u2[r];
          cv.y -= u3[r] - u1[r] - u2[r];
          *cp = cv;
        }
      }
    }
    return;
  }
  // D lane l, register r -> (row 4(l/16) + r, col l%16) of each 16 x 16 block
#pragma unroll
  for (int i = 0; i < BM; ++i)
#pragma unroll
    for (int j = 0; j < BN; ++j) {
      const int rbase = row0 + wm * WM + i * 16, cbase = col0 + wn * WN + j * 16;
      if (rbase < npad && cbase < cmax) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          float2* cp = A + (int64_t)(rbase + 4 * kq + r) * ld + cbase + ii;
          float2 cv = PFC ? cpre[PFC ? i : 0][PFC ? j : 0][r] : *cp;
          cv.x -= t1[i][j][r] - t2[i][j][r];
          cv.y -= t3[i][j][r] - t1[i][j][r] - t2[i][j][r];
          *cp = cv;
        }
      }
    }
}

void launch_gemm_f64(const JobDesc* jobs, int njobs, int rows, int cols, int k, int kd, int r_begin, int c_begin,
                     int c_end, double2* work, hipStream_t s) {
  dim3 grid(cols / 64, rows / 64, njobs);
  gemm_f64_kernel<<<grid, 256, 0, s>>>(jobs, k, kd, r_begin, c_begin, c_end, work);
}

template <int TM, int TN, int WM, int WN, bool XCD, int KC = 16, bool PFC = false, bool TRI = false, bool M32 = false,
          int SWZ = 0>
static void launch_tiled(const JobDesc* jobs, int njobs, int rows, int cols, int k, int kd, int r_begin,
                         int c_begin, int c_end, float2* work, hipStream_t s) {
  const int tx = (cols + TN - 1) / TN, ty = (rows + TM - 1) / TM;
  const int64_t n = TRI ? (int64_t)ty * (ty + 1) / 2 * njobs : (int64_t)tx * ty * njobs;
  gemm_f32_3m_tiled<TM, TN, WM, WN, XCD, KC, PFC, TRI, M32, SWZ>
      <<<(unsigned)n, 256, 0, s>>>(jobs, tx, ty, k, kd, r_begin, c_begin, c_end, work);
}

// Tiling 2 with the tiles of a job numbered in bands of eight tile rows (see SWZ above).
void launch_gemm_f32_banded(const JobDesc* jobs, int njobs, int rows, int cols, int k, int kd, int r_begin,
                            int c_begin, int c_end, float2* work, hipStream_t s) {
  launch_tiled<64, 64, 32, 32, true, 16, false, false, false, 8>(jobs, njobs, rows, cols, k, kd, r_begin, c_begin,
                                                                 c_end, work, s);
}

// Lower-triangle tiles only (rows and columns start together): the update
// A22 -= L21 (D L21^T) of the symmetric factorization, 64 x 64 tiles, XCD-ordered.
void launch_gemm_f32_lower(const JobDesc* jobs, int njobs, int rows, int k, int kd, int rc_begin, float2* work,
                           hipStream_t s) {
  launch_tiled<64, 64, 32, 32, true, 16, false, true>(jobs, njobs, rows, rows, k, kd, rc_begin, rc_begin, 0, work, s);
}

int gemm_f32_variants() { return 10; }

void launch_gemm_f32(int variant, const JobDesc* jobs, int njobs, int rows, int cols, int k, int kd, int r_begin,
                     int c_begin, int c_end, float2* work, hipStream_t s) {
  switch (variant) {
    case 1: launch_tiled<64, 64, 32, 32, false>(jobs, njobs, rows, cols, k, kd, r_begin, c_begin, c_end, work, s); break;
    case 2: launch_tiled<64, 64, 32, 32, true>(jobs, njobs, rows, cols, k, kd, r_begin, c_begin, c_end, work, s); break;
    case 3: launch_tiled<128, 64, 32, 64, true>(jobs, njobs, rows, cols, k, kd, r_begin, c_begin, c_end, work, s); break;
    case 4: launch_tiled<64, 128, 64, 32, true>(jobs, njobs, rows, cols, k, kd, r_begin, c_begin, c_end, work, s); break;
    case 5: launch_tiled<128, 128, 64, 64, true>(jobs, njobs, rows, cols, k, kd, r_begin, c_begin, c_end, work, s); break;
    case 6: launch_tiled<128, 128, 64, 64, false>(jobs, njobs, rows, cols, k, kd, r_begin, c_begin, c_end, work, s); break;
    case 7: launch_tiled<64, 64, 32, 32, true, 16, true>(jobs, njobs, rows, cols, k, kd, r_begin, c_begin, c_end, work, s); break;
    case 8: launch_tiled<64, 64, 32, 32, true, 32, false>(jobs, njobs, rows, cols, k, kd, r_begin, c_begin, c_end, work, s); break;
    case 9: launch_tiled<64, 64, 32, 32, true, 16, false, false, true>(jobs, njobs, rows, cols, k, kd, r_begin, c_begin, c_end, work, s); break;
    default: {
      dim3 grid(cols / 64, rows / 64, njobs);
      gemm_f32_3m_kernel<<<grid, 256, 0, s>>>(jobs, k, kd, r_begin, c_begin, c_end, work);
    }
  }
}

}  // namespace lsms
