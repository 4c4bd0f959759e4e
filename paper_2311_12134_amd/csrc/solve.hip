// Solves with the blocked LU factors, and the FP64 residual / update of the
// split-precision iterative refinement.
//
// The factorization is the product M = P_1^T L_1 P_2^T L_2 ... P_K^T L_K U of panel
// interchanges P_p and unit-lower panel factors L_p (stored in the panel's columns,
// never re-permuted by later panels).  Hence
//   M X = B   :  X = U^-1 L_K^-1 P_K ... L_1^-1 P_1 B          (trans = 0)
//   M^T X = B :  X = P_1^T L_1^-T ... P_K^T L_K^-T U^-T B      (trans = 1)
// One workgroup per job walks the panels.  Each panel's interchanges are applied as one
// gather of at most 2 NB rows (the permutation list written by the panel kernel), the
// diagonal NB x NB triangle is solved by one wavefront with cross-lane shuffles (tri.h),
// and the off-diagonal blocks stream through LDS one coalesced NB x NB tile at a time.
// Arithmetic is FP64 for both storage types.
#include "lsms_internal.h"
#include "tri.h"

namespace lsms {

// Per-thread share of an NB x NRHS block: entry u of thread t is idx = t + 256 u,
// row idx / NRHS, column idx % NRHS.
template <int NRHS>
struct Blk {
  static constexpr int PER = NB * NRHS / 256;
};

template <typename T, int NRHS, int TRANS>
__global__ __launch_bounds__(256) void solve_kernel(const JobDesc* jobs, const T* work, const int32_t* piv,
                                                    double2* xbuf, int64_t col_off, const int32_t* skip) {
  const int job = blockIdx.x;
  if (skip && skip[job]) return;
  const JobDesc jd = jobs[job];
  const T* A = work + jd.a_off;
  const int64_t ld = jd.npad;
  const int npad = jd.npad;
  const int32_t* pv = piv + jd.piv_off;
  double2* X = xbuf + jd.x_off + col_off;
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  constexpr int PER = Blk<NRHS>::PER;
  constexpr int HELD = PERM_MAX * NRHS / 256;
  __shared__ double2 s_T[NB][NB + 1];  // diagonal block, or one NB x NB tile of L / U
  __shared__ double2 s_X[NB][NRHS];    // right-hand sides of the current panel rows
  __shared__ double2 s_C[NB][NRHS];    // a chunk of other right-hand-side rows
  __shared__ int s_dst[PERM_MAX], s_src[PERM_MAX];
  auto xrow = [&](int r) { return X + (int64_t)r * NRHS_MAX; };

  // apply the permutation of panel k to X (gather dst <- src), or its inverse
  auto permute = [&](int k, bool inverse) {
    const int32_t* lst = pv + perm_off(npad, k);
    const int cnt = lst[0];
    for (int i = t; i < cnt; i += 256) {
      s_dst[i] = lst[2 + i];
      s_src[i] = lst[2 + PERM_MAX + i];
    }
    __syncthreads();
    double2 held[HELD];
#pragma unroll
    for (int u = 0; u < HELD; ++u) {
      const int idx = t + 256 * u, i = idx / NRHS, c = idx % NRHS;
      if (i < cnt) held[u] = xrow(inverse ? s_dst[i] : s_src[i])[c];
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < HELD; ++u) {
      const int idx = t + 256 * u, i = idx / NRHS, c = idx % NRHS;
      if (i < cnt) xrow(inverse ? s_src[i] : s_dst[i])[c] = held[u];
    }
    __syncthreads();
  };
  auto load_diag = [&](int k, int which) {  // 0: strict lower (L), 1: upper with diagonal (U)
    for (int idx = t; idx < NB * NB; idx += 256) {
      const int q = idx / NB, pp = idx % NB;
      const bool keep = which ? (pp >= q) : (pp < q);
      s_T[q][pp] = keep ? ld2(A + (k + q) * ld + k + pp) : make_double2(0.0, 0.0);
    }
  };
  auto load_tile = [&](int r0, int c0) {  // s_T = A[r0 .. r0+NB, c0 .. c0+NB)
    for (int idx = t; idx < NB * NB; idx += 256) {
      const int q = idx / NB, pp = idx % NB;
      s_T[q][pp] = ld2(A + (int64_t)(r0 + q) * ld + c0 + pp);
    }
  };
  auto load_rows = [&](double2 (*dst)[NRHS], int r0) {
    for (int idx = t; idx < NB * NRHS; idx += 256) dst[idx / NRHS][idx % NRHS] = xrow(r0 + idx / NRHS)[idx % NRHS];
  };
  auto store_rows = [&](double2 (*src)[NRHS], int r0) {
    for (int idx = t; idx < NB * NRHS; idx += 256) xrow(r0 + idx / NRHS)[idx % NRHS] = src[idx / NRHS][idx % NRHS];
  };

  if (TRANS == 0) {
    // X <- L_K^-1 P_K ... L_1^-1 P_1 X
    for (int k = 0; k < npad; k += NB) {
      permute(k, false);
      load_diag(k, 0);
      load_rows(s_X, k);
      __syncthreads();
      if (wave == 0) tri_unit_lower<NRHS>(&s_T[0][0], NB + 1, &s_X[0][0], NRHS, 0, lane);
      __syncthreads();
      store_rows(s_X, k);
      __syncthreads();
      for (int r0 = k + NB; r0 < npad; r0 += NB) {  // rows below: X -= L21 X_p
        load_tile(r0, k);
        load_rows(s_C, r0);
        __syncthreads();
#pragma unroll
        for (int u = 0; u < PER; ++u) {
          const int idx = t + 256 * u, rr = idx / NRHS, c = idx % NRHS;
          double2 acc = s_C[rr][c];
#pragma unroll 8
          for (int q = 0; q < NB; ++q) acc = cfms(acc, s_T[rr][q], s_X[q][c]);
          xrow(r0 + rr)[c] = acc;
        }
        __syncthreads();
      }
    }
    // X <- U^-1 X
    for (int k = npad - NB; k >= 0; k -= NB) {
      double2 acc[PER];
#pragma unroll
      for (int u = 0; u < PER; ++u) {
        const int idx = t + 256 * u;
        acc[u] = xrow(k + idx / NRHS)[idx % NRHS];
      }
      for (int c0 = k + NB; c0 < npad; c0 += NB) {  // X_p -= U12 X_right
        load_tile(k, c0);
        load_rows(s_C, c0);
        __syncthreads();
#pragma unroll
        for (int u = 0; u < PER; ++u) {
          const int idx = t + 256 * u, q = idx / NRHS, c = idx % NRHS;
#pragma unroll 8
          for (int cc = 0; cc < NB; ++cc) acc[u] = cfms(acc[u], s_T[q][cc], s_C[cc][c]);
        }
        __syncthreads();
      }
#pragma unroll
      for (int u = 0; u < PER; ++u) {
        const int idx = t + 256 * u;
        s_X[idx / NRHS][idx % NRHS] = acc[u];
      }
      load_diag(k, 1);
      __syncthreads();
      if (wave == 0) tri_upper<NRHS>(&s_T[0][0], NB + 1, &s_X[0][0], NRHS, 0, lane);
      __syncthreads();
      store_rows(s_X, k);
      __syncthreads();
    }
  } else {
    // X <- U^-T X (forward over panels)
    for (int k = 0; k < npad; k += NB) {
      load_diag(k, 1);
      load_rows(s_X, k);
      __syncthreads();
      if (wave == 0) tri_upper_trans<NRHS>(&s_T[0][0], NB + 1, &s_X[0][0], NRHS, 0, lane);
      __syncthreads();
      store_rows(s_X, k);
      __syncthreads();
      for (int r0 = k + NB; r0 < npad; r0 += NB) {  // X_r -= U12^T X_p
        load_tile(k, r0);
        load_rows(s_C, r0);
        __syncthreads();
#pragma unroll
        for (int u = 0; u < PER; ++u) {
          const int idx = t + 256 * u, rr = idx / NRHS, c = idx % NRHS;
          double2 a = s_C[rr][c];
#pragma unroll 8
          for (int q = 0; q < NB; ++q) a = cfms(a, s_T[q][rr], s_X[q][c]);
          xrow(r0 + rr)[c] = a;
        }
        __syncthreads();
      }
    }
    // X <- P_1^T L_1^-T ... P_K^T L_K^-T X (backward over panels)
    for (int k = npad - NB; k >= 0; k -= NB) {
      double2 acc[PER];
#pragma unroll
      for (int u = 0; u < PER; ++u) {
        const int idx = t + 256 * u;
        acc[u] = xrow(k + idx / NRHS)[idx % NRHS];
      }
      for (int r0 = k + NB; r0 < npad; r0 += NB) {  // X_p -= L21^T X_below
        load_tile(r0, k);
        load_rows(s_C, r0);
        __syncthreads();
#pragma unroll
        for (int u = 0; u < PER; ++u) {
          const int idx = t + 256 * u, q = idx / NRHS, c = idx % NRHS;
#pragma unroll 8
          for (int rr = 0; rr < NB; ++rr) acc[u] = cfms(acc[u], s_T[rr][q], s_C[rr][c]);
        }
        __syncthreads();
      }
#pragma unroll
      for (int u = 0; u < PER; ++u) {
        const int idx = t + 256 * u;
        s_X[idx / NRHS][idx % NRHS] = acc[u];
      }
      load_diag(k, 0);
      __syncthreads();
      if (wave == 0) tri_unit_lower_trans<NRHS>(&s_T[0][0], NB + 1, &s_X[0][0], NRHS, 0, lane);
      __syncthreads();
      store_rows(s_X, k);
      __syncthreads();
      permute(k, true);
    }
  }
}

template <typename T>
static void solve_dispatch(const JobDesc* jobs, int njobs, const T* work, const int32_t* piv, double2* x,
                           int64_t col_off, int nrhs, int trans, const int32_t* skip, hipStream_t s) {
  if (nrhs == 16) {
    if (trans)
      solve_kernel<T, 16, 1><<<njobs, 256, 0, s>>>(jobs, work, piv, x, col_off, skip);
    else
      solve_kernel<T, 16, 0><<<njobs, 256, 0, s>>>(jobs, work, piv, x, col_off, skip);
  } else {
    if (trans)
      solve_kernel<T, 32, 1><<<njobs, 256, 0, s>>>(jobs, work, piv, x, col_off, skip);
    else
      solve_kernel<T, 32, 0><<<njobs, 256, 0, s>>>(jobs, work, piv, x, col_off, skip);
  }
}

void lu_solve_f64(const JobDesc* jobs, int njobs, const double2* work, const int32_t* piv, double2* x,
                  int64_t x_col_off, int nrhs, int trans, hipStream_t s) {
  solve_dispatch<double2>(jobs, njobs, work, piv, x, x_col_off, nrhs, trans, nullptr, s);
}

void lu_solve_f32(const JobDesc* jobs, int njobs, const float2* work, const int32_t* piv, double2* x,
                  int64_t x_col_off, int nrhs, int trans, hipStream_t s) {
  solve_dispatch<float2>(jobs, njobs, work, piv, x, x_col_off, nrhs, trans, nullptr, s);
}

void lu_solve_f32_skip(const JobDesc* jobs, int njobs, const float2* work, const int32_t* piv, double2* x,
                       const int32_t* skip, hipStream_t s) {
  solve_dispatch<float2>(jobs, njobs, work, piv, x, 0, 16, 0, skip, s);
}

}  // namespace lsms
