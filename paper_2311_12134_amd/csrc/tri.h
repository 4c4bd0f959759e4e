// Wavefront-level triangular solves on NB x NB diagonal blocks held in LDS.
//
// One wavefront solves NC right-hand-side columns: lane = column + NC * group (G = 64/NC
// groups); row q belongs to group q % G, block q / G.  Each lane keeps the RPL = NB/G
// rows of its group in registers, and every finished row is broadcast to the other
// lanes of its column with a cross-lane shuffle, so the NB dependent steps need no
// workgroup barrier.  Blocks are processed by a runtime loop that keeps the current
// block at a fixed register slot and shifts the others, so every register index is a
// compile-time constant.  T is the triangle (row stride ldT), X the right-hand sides
// (row stride ldX, columns [c0, c0 + NC)); arithmetic is FP64.
#pragma once

#include "lsms_internal.h"

namespace lsms {

template <int NC>
struct TriShape {
  static constexpr int G = 64 / NC;   // row groups per wavefront
  static constexpr int RPL = NB / G;  // rows (blocks) per lane
};

__device__ inline double2 shfl2(double2 v, int src) {
  double2 r;
  r.x = __shfl(v.x, src);
  r.y = __shfl(v.y, src);
  return r;
}

// Forward: rows ascending.  UNIT: L unit lower, x_q -= L[q][r] x_r.  !UNIT && TRANS:
// U^T, x_r /= U[r][r] then x_q -= U[r][q] x_r.
template <int NC, bool UNIT, bool TRANS, typename TT, typename XT>
__device__ inline void tri_forward(const TT* T, int ldT, XT* X, int ldX, int c0, int lane) {
  constexpr int G = TriShape<NC>::G, RPL = TriShape<NC>::RPL;
  const int c = lane % NC, g = lane / NC;
  double2 xr[RPL];
#pragma unroll
  for (int s = 0; s < RPL; ++s) xr[s] = ld2(X + (g + G * s) * ldX + c0 + c);
  for (int b = 0; b < RPL; ++b) {  // xr[s] holds block b + s
#pragma unroll 1
    for (int gr = 0; gr < G; ++gr) {
      const int r = G * b + gr;
      if (!UNIT && g == gr) xr[0] = cmul(xr[0], cinv(ld2(T + r * ldT + r)));
      const double2 xv = shfl2(xr[0], c + NC * gr);
      if (g > gr) {
        const int q = g + G * b;
        xr[0] = cfms(xr[0], ld2(TRANS ? T + r * ldT + q : T + q * ldT + r), xv);
      }
#pragma unroll
      for (int s = 1; s < RPL; ++s) {
        if (b + s < RPL) {
          const int q = g + G * (b + s);
          xr[s] = cfms(xr[s], ld2(TRANS ? T + r * ldT + q : T + q * ldT + r), xv);
        }
      }
    }
    st2(X + (g + G * b) * ldX + c0 + c, xr[0]);
#pragma unroll
    for (int s = 0; s < RPL - 1; ++s) xr[s] = xr[s + 1];
  }
}

// Backward: rows descending.  !UNIT && !TRANS: U upper, x_r /= U[r][r] then
// x_q -= U[q][r] x_r.  UNIT && TRANS: L^T unit upper, x_q -= L[r][q] x_r.
template <int NC, bool UNIT, bool TRANS, typename TT, typename XT>
__device__ inline void tri_backward(const TT* T, int ldT, XT* X, int ldX, int c0, int lane) {
  constexpr int G = TriShape<NC>::G, RPL = TriShape<NC>::RPL;
  const int c = lane % NC, g = lane / NC;
  double2 xr[RPL];
#pragma unroll
  for (int s = 0; s < RPL; ++s) xr[s] = ld2(X + (g + G * s) * ldX + c0 + c);
  for (int b = RPL - 1; b >= 0; --b) {  // xr[s] holds block b - (RPL - 1 - s)
#pragma unroll 1
    for (int gr = G - 1; gr >= 0; --gr) {
      const int r = G * b + gr;
      if (!UNIT && g == gr) xr[RPL - 1] = cmul(xr[RPL - 1], cinv(ld2(T + r * ldT + r)));
      const double2 xv = shfl2(xr[RPL - 1], c + NC * gr);
      if (g < gr) {
        const int q = g + G * b;
        xr[RPL - 1] = cfms(xr[RPL - 1], ld2(TRANS ? T + r * ldT + q : T + q * ldT + r), xv);
      }
#pragma unroll
      for (int s = 0; s < RPL - 1; ++s) {
        const int blk = b - (RPL - 1 - s);
        if (blk >= 0) {
          const int q = g + G * blk;
          xr[s] = cfms(xr[s], ld2(TRANS ? T + r * ldT + q : T + q * ldT + r), xv);
        }
      }
    }
    st2(X + (g + G * b) * ldX + c0 + c, xr[RPL - 1]);
#pragma unroll
    for (int s = RPL - 1; s > 0; --s) xr[s] = xr[s - 1];
  }
}

// L unit lower (strictly lower part used), forward.
template <int NC, typename TT, typename XT>
__device__ inline void tri_unit_lower(const TT* T, int ldT, XT* X, int ldX, int c0, int lane) {
  tri_forward<NC, true, false>(T, ldT, X, ldX, c0, lane);
}
// U upper with diagonal, backward.
template <int NC, typename TT, typename XT>
__device__ inline void tri_upper(const TT* T, int ldT, XT* X, int ldX, int c0, int lane) {
  tri_backward<NC, false, false>(T, ldT, X, ldX, c0, lane);
}
// U^T (lower with diagonal), forward.
template <int NC, typename TT, typename XT>
__device__ inline void tri_upper_trans(const TT* T, int ldT, XT* X, int ldX, int c0, int lane) {
  tri_forward<NC, false, true>(T, ldT, X, ldX, c0, lane);
}
// L^T (unit upper), backward.
template <int NC, typename TT, typename XT>
__device__ inline void tri_unit_lower_trans(const TT* T, int ldT, XT* X, int ldX, int c0, int lane) {
  tri_backward<NC, true, true>(T, ldT, X, ldX, c0, lane);
}

}  // namespace lsms
