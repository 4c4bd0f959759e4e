// Solves with the blocked LU factors, and the FP64 residual / update of the
// split-precision iterative refinement.
//
// The factorization is the product M = P_1^T L_1 P_2^T L_2 ... P_K^T L_K U of panel
// interchanges P_p and unit-lower panel factors L_p (stored in the panel's columns,
// never re-permuted by later panels).  Hence
//   M X = B   :  X = U^-1 L_K^-1 P_K ... L_1^-1 P_1 B          (trans = 0)
//   M^T X = B :  X = P_1^T L_1^-T ... P_K^T L_K^-T U^-T B      (trans = 1)
// One workgroup per job walks the panels.  The diagonal NB x NB triangles are solved by
// one wavefront holding the right-hand sides in registers (lane = column + NRHS * group)
// and broadcasting each finished row with cross-lane shuffles; the off-diagonal blocks
// are applied by the whole workgroup.  Arithmetic is FP64 for both storage types.
#include "lsms_internal.h"

namespace lsms {

template <int NRHS>
struct SolveShape {
  static constexpr int G = 64 / NRHS;   // row groups per wavefront
  static constexpr int RPL = NB / G;    // rows per lane
};

// Forward substitution with a unit lower triangle (s_T strictly lower) on s_X, by wave 0.
template <int NRHS>
__device__ inline void diag_unit_lower(double2 (*s_T)[NB + 1], double2 (*s_X)[NRHS], int lane) {
  constexpr int G = SolveShape<NRHS>::G, RPL = SolveShape<NRHS>::RPL;
  const int c = lane % NRHS, g = lane / NRHS;
  double2 xr[RPL];
#pragma unroll
  for (int s = 0; s < RPL; ++s) xr[s] = s_X[g + G * s][c];
#pragma unroll
  for (int sr = 0; sr < RPL; ++sr) {
    for (int gr = 0; gr < G; ++gr) {
      const int r = G * sr + gr;
      const int src = c + NRHS * gr;
      double2 xv;
      xv.x = __shfl(xr[sr].x, src);
      xv.y = __shfl(xr[sr].y, src);
#pragma unroll
      for (int s = sr; s < RPL; ++s) {
        const int q = g + G * s;
        if (q > r) xr[s] = cfms(xr[s], s_T[q][r], xv);
      }
    }
  }
#pragma unroll
  for (int s = 0; s < RPL; ++s) s_X[g + G * s][c] = xr[s];
}

// Backward substitution with a non-unit upper triangle (s_T upper incl. diagonal), by wave 0.
template <int NRHS>
__device__ inline void diag_upper(double2 (*s_T)[NB + 1], double2 (*s_X)[NRHS], int lane) {
  constexpr int G = SolveShape<NRHS>::G, RPL = SolveShape<NRHS>::RPL;
  const int c = lane % NRHS, g = lane / NRHS;
  double2 xr[RPL];
#pragma unroll
  for (int s = 0; s < RPL; ++s) xr[s] = s_X[g + G * s][c];
#pragma unroll
  for (int sr = RPL - 1; sr >= 0; --sr) {
    for (int gr = G - 1; gr >= 0; --gr) {
      const int r = G * sr + gr;
      if (g == gr) xr[sr] = cmul(xr[sr], cinv(s_T[r][r]));
      const int src = c + NRHS * gr;
      double2 xv;
      xv.x = __shfl(xr[sr].x, src);
      xv.y = __shfl(xr[sr].y, src);
#pragma unroll
      for (int s = 0; s <= sr; ++s) {
        const int q = g + G * s;
        if (q < r) xr[s] = cfms(xr[s], s_T[q][r], xv);
      }
    }
  }
#pragma unroll
  for (int s = 0; s < RPL; ++s) s_X[g + G * s][c] = xr[s];
}

// Forward substitution with U^T (lower, non-unit): x_r /= U[r][r]; x_q -= U[r][q] x_r (q > r).
template <int NRHS>
__device__ inline void diag_upper_trans(double2 (*s_T)[NB + 1], double2 (*s_X)[NRHS], int lane) {
  constexpr int G = SolveShape<NRHS>::G, RPL = SolveShape<NRHS>::RPL;
  const int c = lane % NRHS, g = lane / NRHS;
  double2 xr[RPL];
#pragma unroll
  for (int s = 0; s < RPL; ++s) xr[s] = s_X[g + G * s][c];
#pragma unroll
  for (int sr = 0; sr < RPL; ++sr) {
    for (int gr = 0; gr < G; ++gr) {
      const int r = G * sr + gr;
      if (g == gr) xr[sr] = cmul(xr[sr], cinv(s_T[r][r]));
      const int src = c + NRHS * gr;
      double2 xv;
      xv.x = __shfl(xr[sr].x, src);
      xv.y = __shfl(xr[sr].y, src);
#pragma unroll
      for (int s = sr; s < RPL; ++s) {
        const int q = g + G * s;
        if (q > r) xr[s] = cfms(xr[s], s_T[r][q], xv);
      }
    }
  }
#pragma unroll
  for (int s = 0; s < RPL; ++s) s_X[g + G * s][c] = xr[s];
}

// Backward substitution with L^T (unit upper): x_q -= L[r][q] x_r (q < r).
template <int NRHS>
__device__ inline void diag_unit_lower_trans(double2 (*s_T)[NB + 1], double2 (*s_X)[NRHS], int lane) {
  constexpr int G = SolveShape<NRHS>::G, RPL = SolveShape<NRHS>::RPL;
  const int c = lane % NRHS, g = lane / NRHS;
  double2 xr[RPL];
#pragma unroll
  for (int s = 0; s < RPL; ++s) xr[s] = s_X[g + G * s][c];
#pragma unroll
  for (int sr = RPL - 1; sr >= 0; --sr) {
    for (int gr = G - 1; gr >= 0; --gr) {
      const int r = G * sr + gr;
      const int src = c + NRHS * gr;
      double2 xv;
      xv.x = __shfl(xr[sr].x, src);
      xv.y = __shfl(xr[sr].y, src);
#pragma unroll
      for (int s = 0; s <= sr; ++s) {
        const int q = g + G * s;
        if (q < r) xr[s] = cfms(xr[s], s_T[r][q], xv);
      }
    }
  }
#pragma unroll
  for (int s = 0; s < RPL; ++s) s_X[g + G * s][c] = xr[s];
}

template <typename T, int NRHS, int TRANS>
__global__ __launch_bounds__(256) void solve_kernel(const JobDesc* jobs, const T* work, const int32_t* piv,
                                                    double2* xbuf, int64_t col_off, const int32_t* skip) {
  const int job = blockIdx.x;
  if (skip && skip[job]) return;
  const JobDesc jd = jobs[job];
  const T* A = work + jd.a_off;
  const int64_t ld = jd.npad;
  const int npad = jd.npad;
  const int32_t* ip = piv + jd.piv_off;
  double2* X = xbuf + jd.x_off + col_off;
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  __shared__ double2 s_T[NB][NB + 1];
  __shared__ double2 s_X[NB][NRHS];

  auto swap_rows = [&](int k, bool reverse) {
    if (t < NRHS) {
      for (int qq = 0; qq < NB; ++qq) {
        const int q = reverse ? NB - 1 - qq : qq;
        const int d = k + q, p = ip[d];
        if (p != d && p > d && p < npad) {
          const double2 a = X[(int64_t)d * NRHS_MAX + t];
          const double2 b = X[(int64_t)p * NRHS_MAX + t];
          X[(int64_t)d * NRHS_MAX + t] = b;
          X[(int64_t)p * NRHS_MAX + t] = a;
        }
      }
    }
  };

  if (TRANS == 0) {
    // L phase
    for (int k = 0; k < npad; k += NB) {
      swap_rows(k, false);
      __syncthreads();
      for (int idx = t; idx < NB * NB; idx += 256) {
        const int q = idx / NB, pp = idx % NB;
        s_T[q][pp] = pp < q ? ld2(A + (k + q) * ld + k + pp) : make_double2(0.0, 0.0);
      }
      for (int idx = t; idx < NB * NRHS; idx += 256) {
        const int q = idx / NRHS, c = idx % NRHS;
        s_X[q][c] = X[(int64_t)(k + q) * NRHS_MAX + c];
      }
      __syncthreads();
      if (wave == 0) diag_unit_lower<NRHS>(s_T, s_X, lane);
      __syncthreads();
      for (int idx = t; idx < NB * NRHS; idx += 256) {
        const int q = idx / NRHS, c = idx % NRHS;
        X[(int64_t)(k + q) * NRHS_MAX + c] = s_X[q][c];
      }
      const int rows = npad - k - NB;
      for (int idx = t; idx < rows * NRHS; idx += 256) {
        const int r = k + NB + idx / NRHS, c = idx % NRHS;
        double2 acc = X[(int64_t)r * NRHS_MAX + c];
        const T* lrow = A + r * ld + k;
#pragma unroll 8
        for (int q = 0; q < NB; ++q) acc = cfms(acc, ld2(lrow + q), s_X[q][c]);
        X[(int64_t)r * NRHS_MAX + c] = acc;
      }
      __syncthreads();
    }
    // U phase
    for (int k = npad - NB; k >= 0; k -= NB) {
      for (int idx = t; idx < NB * NRHS; idx += 256) {
        const int q = idx / NRHS, c = idx % NRHS;
        double2 acc = X[(int64_t)(k + q) * NRHS_MAX + c];
        const T* urow = A + (k + q) * ld;
        for (int col = k + NB; col < npad; ++col) acc = cfms(acc, ld2(urow + col), X[(int64_t)col * NRHS_MAX + c]);
        s_X[q][c] = acc;
      }
      for (int idx = t; idx < NB * NB; idx += 256) {
        const int q = idx / NB, pp = idx % NB;
        s_T[q][pp] = pp >= q ? ld2(A + (k + q) * ld + k + pp) : make_double2(0.0, 0.0);
      }
      __syncthreads();
      if (wave == 0) diag_upper<NRHS>(s_T, s_X, lane);
      __syncthreads();
      for (int idx = t; idx < NB * NRHS; idx += 256) {
        const int q = idx / NRHS, c = idx % NRHS;
        X[(int64_t)(k + q) * NRHS_MAX + c] = s_X[q][c];
      }
      __syncthreads();
    }
  } else {
    // U^T phase (forward)
    for (int k = 0; k < npad; k += NB) {
      for (int idx = t; idx < NB * NB; idx += 256) {
        const int q = idx / NB, pp = idx % NB;
        s_T[q][pp] = pp >= q ? ld2(A + (k + q) * ld + k + pp) : make_double2(0.0, 0.0);
      }
      for (int idx = t; idx < NB * NRHS; idx += 256) {
        const int q = idx / NRHS, c = idx % NRHS;
        s_X[q][c] = X[(int64_t)(k + q) * NRHS_MAX + c];
      }
      __syncthreads();
      if (wave == 0) diag_upper_trans<NRHS>(s_T, s_X, lane);
      __syncthreads();
      for (int idx = t; idx < NB * NRHS; idx += 256) {
        const int q = idx / NRHS, c = idx % NRHS;
        X[(int64_t)(k + q) * NRHS_MAX + c] = s_X[q][c];
      }
      const int rows = npad - k - NB;
      for (int idx = t; idx < rows * NRHS; idx += 256) {
        const int r = k + NB + idx / NRHS, c = idx % NRHS;
        double2 acc = X[(int64_t)r * NRHS_MAX + c];
#pragma unroll 8
        for (int q = 0; q < NB; ++q) acc = cfms(acc, ld2(A + (k + q) * ld + r), s_X[q][c]);
        X[(int64_t)r * NRHS_MAX + c] = acc;
      }
      __syncthreads();
    }
    // L^T phase (backward) with the panel interchanges undone in reverse order
    for (int k = npad - NB; k >= 0; k -= NB) {
      for (int idx = t; idx < NB * NRHS; idx += 256) {
        const int q = idx % NB, c = idx / NB;
        double2 acc = X[(int64_t)(k + q) * NRHS_MAX + c];
        for (int r = k + NB; r < npad; ++r) acc = cfms(acc, ld2(A + r * ld + k + q), X[(int64_t)r * NRHS_MAX + c]);
        s_X[q][c] = acc;
      }
      for (int idx = t; idx < NB * NB; idx += 256) {
        const int q = idx / NB, pp = idx % NB;
        s_T[q][pp] = pp < q ? ld2(A + (k + q) * ld + k + pp) : make_double2(0.0, 0.0);
      }
      __syncthreads();
      if (wave == 0) diag_unit_lower_trans<NRHS>(s_T, s_X, lane);
      __syncthreads();
      for (int idx = t; idx < NB * NRHS; idx += 256) {
        const int q = idx / NRHS, c = idx % NRHS;
        X[(int64_t)(k + q) * NRHS_MAX + c] = s_X[q][c];
      }
      __syncthreads();
      swap_rows(k, true);
      __syncthreads();
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
