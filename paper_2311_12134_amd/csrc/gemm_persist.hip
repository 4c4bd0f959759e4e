// Persistent form of the split-mode trailing update A22 -= L21 U12 (the FP32 matrix-core
// part of the LU of Eq. (3)): a fixed grid of resident workgroups loops over
// the 64 x 64 complex tiles of every job of the wave, so no workgroup is launched per tile
// and the matrix cores see one continuous stream of products.  The arithmetic is that of
// the tiled kernel in gemm.hip (64 x 64 tile, four waves of 32 x 32, FP32 MFMA 16x16x4 with
// the three real products, K chunks of 16 through two LDS buffers), so every element sums
// in the same order and the results are identical to those of that tiling.
//
// Tiles are numbered job by job, row by row; workgroup b lives on XCD b % 8 (workgroups are
// dealt to the eight XCDs round-robin) and takes tiles from that XCD's contiguous share of
// the numbering, so the tiles of one job, which read the same L21 and U12 panels, stay in
// one L2.  With PFC the wave's C elements are loaded two chunks before the end of a tile.
#include <algorithm>

#include "lsms_internal.h"

namespace lsms {

typedef float f4 __attribute__((ext_vector_type(4)));

template <bool PFC>
__global__ __launch_bounds__(256) void gemm_f32_3m_persist(const JobDesc* jobs, int tiles_x, int tiles_y, int ntiles,
                                                           int k, int kd, int r_begin, int c_begin, int c_end,
                                                           float2* work) {
  constexpr int TM = 64, TN = 64, WM = 32, WN = 32, KC = 16;
  constexpr int BM = WM / 16, BN = WN / 16;
  constexpr int AQ = KC / 4, BQ = TN / 4;
  constexpr int AP = TM * AQ / 256, BP = KC * BQ / 256;
  constexpr int LA = TM + 16, LB = TN + 16;
  __shared__ float2 sA[2][KC][LA];
  __shared__ float2 sB[2][KC][LB];
  auto aswz = [](int kk) { return ((kk >> 2) & 3) << 4; };
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int wm = wave / 2, wn = wave % 2;
  const int ii = lane & 15, kq = lane >> 4;

  // this XCD's share of the tile numbering, and this workgroup's place among the XCD's
  const int G = gridDim.x, xcd = blockIdx.x & 7, per = G >> 3, slot = blockIdx.x >> 3;
  const int q = ntiles >> 3, r = ntiles & 7;
  const int lo = xcd * q + min(xcd, r), hi = lo + q + (xcd < r ? 1 : 0);

  for (int T = lo + slot; T < hi; T += per) {
    int u = T;
    const int tx = u % tiles_x;
    u /= tiles_x;
    const int ty = u % tiles_y;
    const int job = u / tiles_y;
    const JobDesc jd = jobs[job];
    const int row0 = r_begin + ty * TM, col0 = c_begin + tx * TN;
    const int npad = jd.npad;
    const int cmax = c_end > 0 ? min(c_end, npad) : npad;
    if (row0 >= npad || col0 >= cmax) continue;  // uniform over the workgroup
    float2* A = work + jd.a_off;
    const int64_t ld = npad;
    const bool active = (row0 + wm * WM < npad) && (col0 + wn * WN < cmax);

    float2 ra[AP][4], rb[BP][4];
    auto load = [&](int kc) {
#pragma unroll
      for (int p = 0; p < AP; ++p) {
        const int qq = t + 256 * p, i = qq / AQ, kk = (qq % AQ) * 4, row = row0 + i;
        if (row < npad) {
          const float4* src = (const float4*)(A + (int64_t)row * ld + k + kc + kk);
          const float4 v0 = src[0], v1 = src[1];
          ra[p][0] = make_float2(v0.x, v0.y);
          ra[p][1] = make_float2(v0.z, v0.w);
          ra[p][2] = make_float2(v1.x, v1.y);
          ra[p][3] = make_float2(v1.z, v1.w);
        } else {
#pragma unroll
          for (int uu = 0; uu < 4; ++uu) ra[p][uu] = make_float2(0.f, 0.f);
        }
      }
#pragma unroll
      for (int p = 0; p < BP; ++p) {
        const int qq = t + 256 * p, kk = qq / BQ, j = (qq % BQ) * 4;
        if (col0 + j < cmax) {
          const float4* src = (const float4*)(A + (int64_t)(k + kc + kk) * ld + col0 + j);
          const float4 v0 = src[0], v1 = src[1];
          rb[p][0] = make_float2(v0.x, v0.y);
          rb[p][1] = make_float2(v0.z, v0.w);
          rb[p][2] = make_float2(v1.x, v1.y);
          rb[p][3] = make_float2(v1.z, v1.w);
        } else {
#pragma unroll
          for (int uu = 0; uu < 4; ++uu) rb[p][uu] = make_float2(0.f, 0.f);
        }
      }
    };
    auto store = [&](int buf) {
#pragma unroll
      for (int p = 0; p < AP; ++p) {
        const int qq = t + 256 * p, i = qq / AQ, kk = (qq % AQ) * 4;
#pragma unroll
        for (int uu = 0; uu < 4; ++uu) sA[buf][kk + uu][i ^ aswz(kk + uu)] = ra[p][uu];
      }
#pragma unroll
      for (int p = 0; p < BP; ++p) {
        const int qq = t + 256 * p, kk = qq / BQ, j = (qq % BQ) * 4;
#pragma unroll
        for (int uu = 0; uu < 4; ++uu) sB[buf][kk][j + uu] = rb[p][uu];
      }
    };
    f4 t1[BM][BN], t2[BM][BN], t3[BM][BN];
#pragma unroll
    for (int i = 0; i < BM; ++i)
#pragma unroll
      for (int j = 0; j < BN; ++j) {
        t1[i][j] = f4{0, 0, 0, 0};
        t2[i][j] = f4{0, 0, 0, 0};
        t3[i][j] = f4{0, 0, 0, 0};
      }
    float2 cpre[PFC ? BM : 1][PFC ? BN : 1][4];
    auto load_c = [&]() {
#pragma unroll
      for (int i = 0; i < BM; ++i)
#pragma unroll
        for (int j = 0; j < BN; ++j) {
          const int rbase = row0 + wm * WM + i * 16, cbase = col0 + wn * WN + j * 16;
          const bool ok = rbase < npad && cbase < cmax;
#pragma unroll
          for (int rr = 0; rr < 4; ++rr)
            cpre[PFC ? i : 0][PFC ? j : 0][rr] =
                ok ? A[(int64_t)(rbase + 4 * kq + rr) * ld + cbase + ii] : make_float2(0.f, 0.f);
        }
    };
    // the previous tile's last products may still read the buffers
    __syncthreads();
    load(0);
    store(0);
    __syncthreads();
    int cur = 0;
    for (int kc = 0; kc < kd; kc += KC) {
      const bool more = kc + KC < kd;
      if (more) load(kc + KC);
      if (PFC && kc == (kd > 2 * KC ? kd - 2 * KC : 0)) load_c();
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
    if (!active) continue;
#pragma unroll
    for (int i = 0; i < BM; ++i)
#pragma unroll
      for (int j = 0; j < BN; ++j) {
        const int rbase = row0 + wm * WM + i * 16, cbase = col0 + wn * WN + j * 16;
        if (rbase < npad && cbase < cmax) {
#pragma unroll
          for (int rr = 0; rr < 4; ++rr) {
            float2* cp = A + (int64_t)(rbase + 4 * kq + rr) * ld + cbase + ii;
            float2 cv = PFC ? cpre[PFC ? i : 0][PFC ? j : 0][rr] : *cp;
            cv.x -= t1[i][j][rr] - t2[i][j][rr];
            cv.y -= t3[i][j][rr] - t1[i][j][rr] - t2[i][j][rr];
            *cp = cv;
          }
        }
      }
  }
}

// Workgroups of the persistent grid: as many as are resident at once on every compute unit
// (a workgroup that waited for a second round would serialise its whole share of tiles),
// a multiple of 8 so each XCD gets the same number.
template <bool PFC>
static int persist_grid() {
  static int wgs = 0;
  if (wgs == 0) {
    int dev = 0, cus = 0, per_cu = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess &&
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, gemm_f32_3m_persist<PFC>, 256, 0) == hipSuccess &&
        cus > 0 && per_cu > 0)
      wgs = per_cu * cus;
    else
      wgs = 256;
    wgs = std::max(8, wgs / 8 * 8);
  }
  return wgs;
}

int gemm_f32_variants_all() { return gemm_f32_variants() + 2; }

// Variants past the tiled family of gemm.hip: 10 the persistent 64 x 64 form, 11 the same
// with the C tile loaded two chunks early.
void launch_gemm_f32_any(int variant, const JobDesc* jobs, int njobs, int rows, int cols, int k, int kd, int r_begin,
                         int c_begin, int c_end, float2* work, hipStream_t s) {
  const int base = gemm_f32_variants();
  if (variant < base) {
    launch_gemm_f32(variant, jobs, njobs, rows, cols, k, kd, r_begin, c_begin, c_end, work, s);
    return;
  }
  const int tx = (cols + 63) / 64, ty = (rows + 63) / 64;
  const int64_t nt = (int64_t)tx * ty * njobs;
  const int wgs = variant == base ? persist_grid<false>() : persist_grid<true>();
  const int grid = (int)std::min<int64_t>(wgs, (nt + 7) / 8 * 8);
  if (variant == base)
    gemm_f32_3m_persist<false><<<grid, 256, 0, s>>>(jobs, tx, ty, (int)nt, k, kd, r_begin, c_begin, c_end, work);
  else
    gemm_f32_3m_persist<true><<<grid, 256, 0, s>>>(jobs, tx, ty, (int)nt, k, kd, r_begin, c_begin, c_end, work);
}

}  // namespace lsms
