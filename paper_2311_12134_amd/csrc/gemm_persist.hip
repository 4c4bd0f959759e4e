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

// Streaming form of the persistent update: the same resident grid and tile order, but the
// first K chunk of a workgroup's next tile is loaded during the last chunk of the current
// one (and written to the free LDS buffer before the closing barrier), so no tile starts
// with an exposed global-load latency; with PFC the C tile is loaded at the start of the
// last chunk, so the epilogue's read latency overlaps that chunk's products.  Per tile
// the arithmetic and its order are those of the 64 x 64 tiled kernel.
template <bool PFC>
__global__ __launch_bounds__(256, PFC ? 3 : 4) void gemm_f32_3m_stream(const JobDesc* jobs, int tiles_x, int tiles_y, int ntiles,
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

  const int G = gridDim.x, xcd = blockIdx.x & 7, per = G >> 3, slot = blockIdx.x >> 3;
  const int q = ntiles >> 3, r = ntiles & 7;
  const int lo = xcd * q + min(xcd, r), hi = lo + q + (xcd < r ? 1 : 0);

  // a tile of the numbering: its corner, its job's size and matrix (uniform values)
  struct Tile {
    int row0, col0, npad, cmax;
    float2* A;
  };
  // advances T (by per) to the next tile that lies inside its job's matrix; false past hi
  auto find = [&](int& T, Tile& tl) -> bool {
    for (; T < hi; T += per) {
      int u = T;
      const int tx = u % tiles_x;
      u /= tiles_x;
      const int ty = u % tiles_y;
      const JobDesc& jd = jobs[u / tiles_y];
      tl.row0 = r_begin + ty * TM;
      tl.col0 = c_begin + tx * TN;
      tl.npad = jd.npad;
      tl.cmax = c_end > 0 ? min(c_end, tl.npad) : tl.npad;
      tl.A = work + jd.a_off;
      if (tl.row0 < tl.npad && tl.col0 < tl.cmax) return true;
    }
    return false;
  };

  float2 ra[AP][4], rb[BP][4];
  auto load = [&](const Tile& tl, int kc) {
    const int64_t ld = tl.npad;
#pragma unroll
    for (int p = 0; p < AP; ++p) {
      const int qq = t + 256 * p, i = qq / AQ, kk = (qq % AQ) * 4, row = tl.row0 + i;
      if (row < tl.npad) {
        const float4* src = (const float4*)(tl.A + (int64_t)row * ld + k + kc + kk);
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
      if (tl.col0 + j < tl.cmax) {
        const float4* src = (const float4*)(tl.A + (int64_t)(k + kc + kk) * ld + tl.col0 + j);
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
  float2 cpre[PFC ? BM : 1][PFC ? BN : 1][4];
  auto load_c = [&](const Tile& tl) {
    const int64_t ld = tl.npad;
#pragma unroll
    for (int i = 0; i < BM; ++i)
#pragma unroll
      for (int j = 0; j < BN; ++j) {
        const int rbase = tl.row0 + wm * WM + i * 16, cbase = tl.col0 + wn * WN + j * 16;
        const bool ok = rbase < tl.npad && cbase < tl.cmax;
#pragma unroll
        for (int rr = 0; rr < 4; ++rr)
          cpre[PFC ? i : 0][PFC ? j : 0][rr] =
              ok ? tl.A[(int64_t)(rbase + 4 * kq + rr) * ld + cbase + ii] : make_float2(0.f, 0.f);
      }
  };

  int T = lo + slot;
  Tile cur_t;
  if (!find(T, cur_t)) return;  // uniform
  load(cur_t, 0);
  store(0);
  __syncthreads();
  int cur = 0;
  while (true) {
    int Tn = T + per;
    Tile nxt;
    const bool has_next = find(Tn, nxt);
    f4 t1[BM][BN], t2[BM][BN], t3[BM][BN];
#pragma unroll
    for (int i = 0; i < BM; ++i)
#pragma unroll
      for (int j = 0; j < BN; ++j) {
        t1[i][j] = f4{0, 0, 0, 0};
        t2[i][j] = f4{0, 0, 0, 0};
        t3[i][j] = f4{0, 0, 0, 0};
      }
    for (int kc = 0; kc < kd; kc += KC) {
      const bool more = kc + KC < kd;
      if (more)
        load(cur_t, kc + KC);
      else if (has_next)
        load(nxt, 0);
      if (PFC && !more) load_c(cur_t);
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
      if (more || has_next) store(cur ^ 1);  // the next chunk, or the next tile's first
      __syncthreads();
      cur ^= 1;
    }
    const int64_t ld = cur_t.npad;
#pragma unroll
    for (int i = 0; i < BM; ++i)
#pragma unroll
      for (int j = 0; j < BN; ++j) {
        const int rbase = cur_t.row0 + wm * WM + i * 16, cbase = cur_t.col0 + wn * WN + j * 16;
        if (rbase < cur_t.npad && cbase < cur_t.cmax) {
#pragma unroll
          for (int rr = 0; rr < 4; ++rr) {
            float2* cp = cur_t.A + (int64_t)(rbase + 4 * kq + rr) * ld + cbase + ii;
            float2 cv = PFC ? cpre[PFC ? i : 0][PFC ? j : 0][rr] : *cp;
            cv.x -= t1[i][j][rr] - t2[i][j][rr];
            cv.y -= t3[i][j][rr] - t1[i][j][rr] - t2[i][j][rr];
            *cp = cv;
          }
        }
      }
    if (!has_next) break;
    T = Tn;
    cur_t = nxt;
  }
}

// Workgroups of the persistent grid: as many as are resident at once on every compute unit
// (a workgroup that waited for a second round would serialise its whole share of tiles),
// a multiple of 8 so each XCD gets the same number.
// (one cached figure per kernel: ID tells them apart).
template <int ID, typename K>
static int persist_grid(K kernel) {
  static int wgs = 0;
  if (wgs == 0) {
    int dev = 0, cus = 0, per_cu = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess &&
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, 256, 0) == hipSuccess &&
        cus > 0 && per_cu > 0)
      wgs = per_cu * cus;
    else
      wgs = 256;
    wgs = std::max(8, wgs / 8 * 8);
  }
  return wgs;
}

template <int TM, int TN, int DEPTH, int SWZ>
void launch_big(const JobDesc* jobs, int njobs, int rows, int cols, int k, int kd, int r_begin, int c_begin,
                int c_end, float2* work, hipStream_t s);  // gemm_wide.hip

void launch_gemm_f32_banded(const JobDesc* jobs, int njobs, int rows, int cols, int k, int kd, int r_begin,
                            int c_begin, int c_end, float2* work, hipStream_t s);  // gemm.hip

int gemm_f32_variants_all() { return gemm_f32_variants() + 11; }

// Variants past the tiled family of gemm.hip: 10 the persistent 64 x 64 form, 11 the same
// with the C tile loaded two chunks early; 12, 13, 14 the 128 x 64, 64 x 128 and 128 x 128
// tiles of eight and sixteen waves; 15, 16 the 64 x 64 and 64 x 128 tiles with the K chunks
// prefetched two ahead (gemm_wide.hip); 17, 18 the streaming persistent form without and
// with the C tile loaded at the start of a tile's last chunk; 19 tiling 2 with the tiles of
// a job in bands of eight tile rows (gemm.hip); 20 the 64 x 128 tile (13) in bands of eight
// tile rows (gemm_wide.hip).
void launch_gemm_f32_any(int variant, const JobDesc* jobs, int njobs, int rows, int cols, int k, int kd, int r_begin,
                         int c_begin, int c_end, float2* work, hipStream_t s) {
  const int base = gemm_f32_variants();
  if (variant < base) {
    launch_gemm_f32(variant, jobs, njobs, rows, cols, k, kd, r_begin, c_begin, c_end, work, s);
    return;
  }
  if (variant == base + 9) {
    launch_gemm_f32_banded(jobs, njobs, rows, cols, k, kd, r_begin, c_begin, c_end, work, s);
    return;
  }
  if (variant == base + 10) {
    launch_big<64, 128, 1, 8>(jobs, njobs, rows, cols, k, kd, r_begin, c_begin, c_end, work, s);
    return;
  }
  if (variant >= base + 2 && variant < base + 7) {
    if (variant == base + 2)
      launch_big<128, 64, 1, 0>(jobs, njobs, rows, cols, k, kd, r_begin, c_begin, c_end, work, s);
    else if (variant == base + 3)
      launch_big<64, 128, 1, 0>(jobs, njobs, rows, cols, k, kd, r_begin, c_begin, c_end, work, s);
    else if (variant == base + 4)
      launch_big<128, 128, 1, 0>(jobs, njobs, rows, cols, k, kd, r_begin, c_begin, c_end, work, s);
    else if (variant == base + 5)
      launch_big<64, 64, 2, 0>(jobs, njobs, rows, cols, k, kd, r_begin, c_begin, c_end, work, s);
    else
      launch_big<64, 128, 2, 0>(jobs, njobs, rows, cols, k, kd, r_begin, c_begin, c_end, work, s);
    return;
  }
  const int tx = (cols + 63) / 64, ty = (rows + 63) / 64;
  const int64_t nt = (int64_t)tx * ty * njobs;
  int wgs;
  switch (variant - base) {
    case 0: wgs = persist_grid<0>(gemm_f32_3m_persist<false>); break;
    case 1: wgs = persist_grid<1>(gemm_f32_3m_persist<true>); break;
    case 7: wgs = persist_grid<7>(gemm_f32_3m_stream<false>); break;
    default: wgs = persist_grid<8>(gemm_f32_3m_stream<true>);
  }
  const int grid = (int)std::min<int64_t>(wgs, (nt + 7) / 8 * 8);
  switch (variant - base) {
    case 0:
      gemm_f32_3m_persist<false><<<grid, 256, 0, s>>>(jobs, tx, ty, (int)nt, k, kd, r_begin, c_begin, c_end, work);
      break;
    case 1:
      gemm_f32_3m_persist<true><<<grid, 256, 0, s>>>(jobs, tx, ty, (int)nt, k, kd, r_begin, c_begin, c_end, work);
      break;
    case 7:
      gemm_f32_3m_stream<false><<<grid, 256, 0, s>>>(jobs, tx, ty, (int)nt, k, kd, r_begin, c_begin, c_end, work);
      break;
    default:
      gemm_f32_3m_stream<true><<<grid, 256, 0, s>>>(jobs, tx, ty, (int)nt, k, kd, r_begin, c_begin, c_end, work);
  }
}

}  // namespace lsms
