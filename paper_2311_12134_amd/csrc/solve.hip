// Solves with the blocked LU factors (forward substitution, back substitution, and the
// transposed pair used by the adjoint).
//
// The factorization is the product M = P_1^T L_1 P_2^T L_2 ... P_K^T L_K U of panel
// permutations P_p and unit-lower panel factors L_p (stored in the panel's columns,
// never re-permuted by later panels; the factorization leaves the inverses of the unit
// lower and the upper diagonal triangles in each diagonal block).  Hence
//   M X = B   :  X = U^-1 L_K^-1 P_K ... L_1^-1 P_1 B          (trans = 0)
//   M^T X = B :  X = P_1^T L_1^-T ... P_K^T L_K^-T U^-T B      (trans = 1)
// Panels come in groups of G (2 .. 4, as the factorization had them: the L rows of a
// panel are stored after the permutations of the later panels of its group) and every group
// costs two launches over the whole batch:
//   solve_group_diag_kernel    one workgroup per job: panel by panel, the permutation (a
//                              gather of at most 2 NB rows), the coupling blocks with the
//                              group's panels solved before it, and the NB x NB diagonal step
//                              as a product with the stored inverse (or its transpose);
//   solve_group_update_kernel  one workgroup per (64-row strip, job): the strip against the
//                              group's G NB solved rows (K = G NB) on the matrix cores,
//                              operands read straight from the factors (FP32 factors widened in
//                              registers for FP64 solves) and the solution, so the factors
//                              stream from HBM once per solve and the solution rows are read
//                              and written once per group.
// The update is column-oriented (rows below for L and U^T, rows above for U) except for
// L^T, whose group rows need a sum over all rows below: there every strip adds its partial
// product to the group rows with FP64 atomics.  Arithmetic is FP64 for both storage types of
// the factors, except in the split-mode refinement: its forward solves (L and U) with the
// FP32 factors run in FP32 (three-product FP32 MFMA) on an FP32 copy of the right-hand side,
// since a solve with FP32 factors is no more accurate than FP32 however it is summed; the
// residuals and the accumulation of the solution stay FP64.
#include <type_traits>

#include "lsms_internal.h"
#include "strip_mma.h"

namespace lsms {

typedef double d4 __attribute__((ext_vector_type(4)));

enum { MODE_L = 0, MODE_U = 1, MODE_UT = 2, MODE_LT = 3 };

// The solution block of a job: FP64 rows of NRHS_MAX columns, or the FP32 copy the split-mode
// refinement solves on, which lives in columns 16 .. 23 of the same rows (2 NRHS_MAX float2
// per row; the forward solves use columns 0 .. 15 only).
template <typename XT>
struct XView;
template <>
struct XView<double2> {
  static constexpr int LD = NRHS_MAX;
  __device__ static double2* base(double2* xbuf, const JobDesc& jd, int64_t col_off) {
    return xbuf + jd.x_off + col_off;
  }
};
template <>
struct XView<float2> {
  static constexpr int LD = 2 * NRHS_MAX;
  __device__ static float2* base(double2* xbuf, const JobDesc& jd, int64_t) {
    return (float2*)(xbuf + jd.x_off) + 2 * 16;
  }
};
// a factor element in the solve's precision
template <typename XT, typename T>
__device__ inline XT fac(const T* p);
template <>
__device__ inline double2 fac<double2, double2>(const double2* p) { return *p; }
template <>
__device__ inline double2 fac<double2, float2>(const float2* p) { return ld2(p); }
template <>
__device__ inline float2 fac<float2, float2>(const float2* p) { return *p; }
__device__ inline double2 xminus(double2 x, double2 v) { return csub(x, v); }
__device__ inline float2 xminus(float2 x, double2 v) { return make_float2(x.x - (float)v.x, x.y - (float)v.y); }
__device__ inline void xput(double2& d, double2 v) { d = v; }
__device__ inline void xput(float2& d, double2 v) { d = make_float2((float)v.x, (float)v.y); }

// One panel permutation of the solution rows (at most PERM_MAX (dst, src) pairs): every
// source row is read into registers before any destination row is written.
template <int NRHS, typename XT>
__device__ inline void apply_perm(const int32_t* lst, bool inverse, XT* X, int* s_dst, int* s_src, int t) {
  constexpr int HELD = PERM_MAX * NRHS / 256;
  const int cnt = lst[0];
  for (int i = t; i < cnt; i += 256) {
    s_dst[i] = lst[2 + i];
    s_src[i] = lst[2 + PERM_MAX + i];
  }
  __syncthreads();
  const int* from = inverse ? s_dst : s_src;
  const int* to = inverse ? s_src : s_dst;
  constexpr int LD = XView<XT>::LD;
  XT held[HELD];
#pragma unroll
  for (int u = 0; u < HELD; ++u) {
    const int idx = t + 256 * u, i = idx / NRHS, c = idx % NRHS;
    held[u] = i < cnt ? X[(int64_t)from[i] * LD + c] : XT{};
  }
  __syncthreads();
#pragma unroll
  for (int u = 0; u < HELD; ++u) {
    const int idx = t + 256 * u, i = idx / NRHS, c = idx % NRHS;
    if (i < cnt) X[(int64_t)to[i] * LD + c] = held[u];
  }
  __syncthreads();
}

// ------------------------------------------------------------------------------------
// group solves: the panels of the factorization come in groups (k, k + NB, ..), k a
// multiple of G NB (see lu_factor_any).  One launch per group solves its diagonal blocks and
// the coupling blocks between them; one launch per group updates every other 64-row strip
// with K = G NB (less when the job's matrix ends inside the group).  MFMA operands of the
// update are read straight from the factors and the solution rows (through the caches); no
// LDS stage, no barriers in the update.
// ------------------------------------------------------------------------------------

// Element (q, p) of an operator on a panel's rows at kp, from the stored diagonal block:
// the inverse of the unit lower triangle (unit diagonal implied) or of the upper one.
template <typename XT, typename T>
__device__ inline XT lower_inv(const T* A, int64_t ld, int kp, int q, int p) {
  return p < q ? fac<XT>(A + (int64_t)(kp + q) * ld + kp + p) : XT{p == q ? 1.0f : 0.0f, 0.0f};
}
template <typename XT, typename T>
__device__ inline XT upper_inv(const T* A, int64_t ld, int kp, int q, int p) {
  return p >= q ? fac<XT>(A + (int64_t)(kp + q) * ld + kp + p) : XT{};
}

// Y (64 x NRHS) = op (64 x 64) Xin (64 x NRHS in LDS): wave w forms rows 16w .. 16w+16 and
// hands each element to put(row, column, value).
template <int NRHS, typename XT, typename OP, typename PUT>
__device__ inline void panel_product(OP op, const XT (*xin)[NRHS], PUT put, int wave, int lane) {
  StripMma<XT, NRHS / 16> y;
  y.zero();
  y.run([&](int i, int kk) { return op(wave * 16 + i, kk); }, [&](int kk, int c) { return xin[kk][c]; }, lane);
  const int ii = lane & 15;
#pragma unroll
  for (int cb = 0; cb < NRHS / 16; ++cb)
#pragma unroll
    for (int r = 0; r < 4; ++r) put(wave * 16 + y.row(r, lane), cb * 16 + ii, y.value(cb, r));
}

template <typename T, typename XT, int NRHS, int MODE>
__global__ __launch_bounds__(256) void solve_group_diag_kernel(const JobDesc* jobs, int k, int group, const T* work,
                                                               const int32_t* piv, double2* xbuf, int64_t col_off,
                                                               const int32_t* skip) {
  const int job = blockIdx.x;
  if (skip && skip[job]) return;
  const JobDesc jd = jobs[job];
  if (k >= jd.npad) return;  // uniform
  const T* A = work + jd.a_off;
  const int64_t ld = jd.npad;
  const int32_t* pv = piv + jd.piv_off;
  XT* X = XView<XT>::base(xbuf, jd, col_off);
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int np = min(group, (jd.npad - k) / NB);  // panels of the group inside this job
  auto kp = [&](int j) { return k + j * NB; };
  __shared__ XT s_a[NB][NRHS];
  __shared__ XT s_b[NB][NRHS];
  __shared__ int s_dst[PERM_MAX], s_src[PERM_MAX];
  auto xrow = [&](int r) { return X + (int64_t)r * XView<XT>::LD; };
  auto load = [&](XT (*dst)[NRHS], int r0) {
    for (int idx = t; idx < NB * NRHS; idx += 256) dst[idx / NRHS][idx % NRHS] = xrow(r0 + idx / NRHS)[idx % NRHS];
  };
  auto to_x = [&](int r0) {  // result rows to the solution
    return [=](int row, int c, double2 v) { xput(xrow(r0 + row)[c], v); };
  };
  // rows of s_a minus a product: each wave updates only its own rows, after its product
  auto minus_into_a = [&](int row, int c, double2 v) { s_a[row][c] = xminus(s_a[row][c], v); };
  // s_a -= op (64 x 64) times the solved rows of panel i, staged through s_b
  auto couple = [&](int i, auto op) {
    __syncthreads();
    load(s_b, kp(i));
    __syncthreads();
    panel_product<NRHS, XT>(op, s_b, minus_into_a, wave, lane);
  };
  if (MODE == MODE_L) {
    // panel by panel: P_j (the earlier panels' L rows are stored after it), the couplings
    // L[j, i] with the earlier panels of the group, L_j^-1
    for (int j = 0; j < np; ++j) {
      if (j > 0) __syncthreads();
      apply_perm<NRHS, XT>(pv + perm_off(jd.npad, kp(j)), false, X, s_dst, s_src, t);
      load(s_a, kp(j));
      for (int i = 0; i < j; ++i)
        couple(i, [&](int q, int p) { return fac<XT>(A + (int64_t)(kp(j) + q) * ld + kp(i) + p); });
      __syncthreads();
      panel_product<NRHS, XT>([&](int q, int p) { return lower_inv<XT>(A, ld, kp(j), q, p); }, s_a, to_x(kp(j)),
                              wave, lane);
    }
  } else if (MODE == MODE_U) {
    // last panel first: the couplings U[j, i] with the later panels, U_j^-1
    for (int j = np - 1; j >= 0; --j) {
      __syncthreads();
      load(s_a, kp(j));
      for (int i = j + 1; i < np; ++i)
        couple(i, [&](int q, int p) { return fac<XT>(A + (int64_t)(kp(j) + q) * ld + kp(i) + p); });
      __syncthreads();
      panel_product<NRHS, XT>([&](int q, int p) { return upper_inv<XT>(A, ld, kp(j), q, p); }, s_a, to_x(kp(j)),
                              wave, lane);
    }
  } else if (MODE == MODE_UT) {
    // first panel first: the couplings U[i, j]^T with the earlier panels, U_j^-T
    for (int j = 0; j < np; ++j) {
      __syncthreads();
      load(s_a, kp(j));
      for (int i = 0; i < j; ++i)
        couple(i, [&](int q, int p) { return fac<XT>(A + (int64_t)(kp(i) + p) * ld + kp(j) + q); });
      __syncthreads();
      panel_product<NRHS, XT>([&](int q, int p) { return upper_inv<XT>(A, ld, kp(j), p, q); }, s_a, to_x(kp(j)),
                              wave, lane);
    }
  } else {
    // MODE_LT, last panel first: the couplings L[i, j]^T with the later panels, L_j^-T; then
    // the group's permutations inverted, last panel's first
    for (int j = np - 1; j >= 0; --j) {
      __syncthreads();
      load(s_a, kp(j));
      for (int i = j + 1; i < np; ++i)
        couple(i, [&](int q, int p) { return fac<XT>(A + (int64_t)(kp(i) + p) * ld + kp(j) + q); });
      __syncthreads();
      panel_product<NRHS, XT>([&](int q, int p) { return lower_inv<XT>(A, ld, kp(j), p, q); }, s_a, to_x(kp(j)),
                              wave, lane);
    }
    __syncthreads();
    for (int j = np - 1; j >= 0; --j) apply_perm<NRHS, XT>(pv + perm_off(jd.npad, kp(j)), true, X, s_dst, s_src, t);
  }
}

// One 64-row strip s against the group's K = KD rows (KD = G NB, or fewer where the job's
// matrix ends inside the group):
//          MODE_L   X[s] -= L[s, group] X[group]      (s below the group)
//          MODE_U   X[s] -= U[s, group] X[group]      (s above)
//          MODE_UT  X[s] -= U[group, s]^T X[group]    (s below)
//          MODE_LT  X[group] -= L[s, group]^T X[s]    (s below; FP64 atomics into the group rows)
template <typename T, typename XT, int NRHS, int MODE, int KD>
__device__ inline void group_update(const T* A, int64_t ld, XT* X, int k, int s0, int wave, int lane) {
  auto xrow = [&](int r) { return X + (int64_t)r * XView<XT>::LD; };
  const int ii = lane & 15;
  if constexpr (MODE == MODE_LT) {
    // out rows = the group's KD rows (KD / 16 blocks, dealt to the four waves), K = 64 strip rows
    for (int rb = wave; rb < KD / 16; rb += 4) {
      StripMma<double2, NRHS / 16> y;
      y.zero();
      y.run([&](int i, int kk) { return ld2(A + (int64_t)(s0 + kk) * ld + k + rb * 16 + i); },
            [&](int kk, int c) { return xrow(s0 + kk)[c]; }, lane);
#pragma unroll
      for (int cb = 0; cb < NRHS / 16; ++cb)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          double2* xp = xrow(k + rb * 16 + y.row(r, lane)) + cb * 16 + ii;
          const double2 v = y.value(cb, r);
          atomicAdd(&xp->x, -v.x);
          atomicAdd(&xp->y, -v.y);
        }
    }
    return;
  }
  StripMma<XT, NRHS / 16, KD> y;
  y.zero();
  const int r0 = s0 + wave * 16;
  y.run(
      [&](int i, int kk) {
        return MODE == MODE_UT ? fac<XT>(A + (int64_t)(k + kk) * ld + r0 + i)
                               : fac<XT>(A + (int64_t)(r0 + i) * ld + k + kk);
      },
      [&](int kk, int c) { return xrow(k + kk)[c]; }, lane);
#pragma unroll
  for (int cb = 0; cb < NRHS / 16; ++cb)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      XT* xp = xrow(r0 + y.row(r, lane)) + cb * 16 + ii;
      *xp = xminus(*xp, y.value(cb, r));
    }
}

// MODE_L and MODE_U with the strip's factor rows staged through LDS: the 64 x KD block
// A[s0 .., k ..] streams from HBM in chunks of 256 bytes per row (32 FP32 or 16 FP64
// complex columns), each thread moving 16-byte pieces of whole rows (coalesced), through two
// buffers (35 KB, four workgroups per compute unit) with the next chunk's loads issued before
// the current chunk's products; each wave then takes its 16 rows' operands from LDS.  Same
// products, same order as group_update.
template <typename T, typename XT, int NRHS, int KD>
__device__ inline void group_update_staged(const T* A, int64_t ld, XT* X, int k, int s0, int t, int wave, int lane,
                                           float4 (*sL)[64][17]) {
  constexpr int KCH = 256 / (int)sizeof(T);  // complex columns per chunk
  constexpr int NCH = KD / KCH;
  constexpr int Q = 64 * 16 / 256;            // 16-byte pieces per thread and chunk
  auto xrow = [&](int r) { return X + (int64_t)r * XView<XT>::LD; };
  float4 held[Q];
  auto load = [&](int c) {
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const int idx = t + 256 * q, row = idx >> 4, p4 = idx & 15;
      held[q] = ((const float4*)(A + (int64_t)(s0 + row) * ld + k + c * KCH))[p4];
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const int idx = t + 256 * q;
      sL[buf][idx >> 4][idx & 15] = held[q];
    }
  };
  StripMma<XT, NRHS / 16, KCH> y;
  y.zero();
  load(0);
  store(0);
  __syncthreads();
  for (int c = 0; c < NCH; ++c) {
    const int cur = c & 1;
    if (c + 1 < NCH) load(c + 1);
    const T* rows = (const T*)&sL[cur][wave * 16][0];
    y.run([&](int i, int kk) { return fac<XT>(rows + (int64_t)i * (17 * 16 / sizeof(T)) + kk); },
          [&](int kk, int cc) { return xrow(k + c * KCH + kk)[cc]; }, lane);
    if (c + 1 < NCH) store(cur ^ 1);
    __syncthreads();
  }
  const int ii = lane & 15;
  const int r0 = s0 + wave * 16;
#pragma unroll
  for (int cb = 0; cb < NRHS / 16; ++cb)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      XT* xp = xrow(r0 + y.row(r, lane)) + cb * 16 + ii;
      *xp = xminus(*xp, y.value(cb, r));
    }
}

template <typename T, typename XT, int NRHS, int MODE>
__global__ __launch_bounds__(256) void solve_group_update_kernel(const JobDesc* jobs, int k, int group, const T* work,
                                                                 double2* xbuf, int64_t col_off, const int32_t* skip) {
  const int job = blockIdx.y;
  if (skip && skip[job]) return;
  const JobDesc jd = jobs[job];
  if (k >= jd.npad) return;
  const int s0 = (MODE == MODE_U) ? blockIdx.x * 64 : k + group * NB + blockIdx.x * 64;
  if (MODE == MODE_U ? (s0 >= k) : (s0 >= jd.npad)) return;  // uniform
  const T* A = work + jd.a_off;
  const int64_t ld = jd.npad;
  XT* X = XView<XT>::base(xbuf, jd, col_off);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  // strips below the group exist only when the whole group lies inside the job
  const int kd = min(group * NB, jd.npad - k);
  if constexpr (MODE == MODE_L || MODE == MODE_U) {
    __shared__ float4 sL[2][64][17];
    const int t = threadIdx.x;
    switch (kd / NB) {
      case 1: group_update_staged<T, XT, NRHS, NB>(A, ld, X, k, s0, t, wave, lane, sL); break;
      case 2: group_update_staged<T, XT, NRHS, 2 * NB>(A, ld, X, k, s0, t, wave, lane, sL); break;
      case 3: group_update_staged<T, XT, NRHS, 3 * NB>(A, ld, X, k, s0, t, wave, lane, sL); break;
      default: group_update_staged<T, XT, NRHS, 4 * NB>(A, ld, X, k, s0, t, wave, lane, sL); break;
    }
    return;
  }
  switch (kd / NB) {
    case 1: group_update<T, XT, NRHS, MODE, NB>(A, ld, X, k, s0, wave, lane); break;
    case 2: group_update<T, XT, NRHS, MODE, 2 * NB>(A, ld, X, k, s0, wave, lane); break;
    case 3: group_update<T, XT, NRHS, MODE, 3 * NB>(A, ld, X, k, s0, wave, lane); break;
    default: group_update<T, XT, NRHS, MODE, 4 * NB>(A, ld, X, k, s0, wave, lane); break;
  }
}

template <typename T, typename XT, int NRHS>
static void solve_all(const JobDesc* jobs, int njobs, int npad_max, const T* work, const int32_t* piv, double2* x,
                      int64_t col_off, int trans, int group, const int32_t* skip, hipStream_t s) {
  const int GW = group * NB;
  const int last = ((npad_max - 1) / GW) * GW;  // start of the last group
  auto diag = [&](auto mode_tag, int k) {
    constexpr int MODE = decltype(mode_tag)::value;
    solve_group_diag_kernel<T, XT, NRHS, MODE><<<njobs, 256, 0, s>>>(jobs, k, group, work, piv, x, col_off, skip);
  };
  auto update = [&](auto mode_tag, int k, int strips) {
    constexpr int MODE = decltype(mode_tag)::value;
    if (strips <= 0) return;
    solve_group_update_kernel<T, XT, NRHS, MODE>
        <<<dim3(strips, njobs), 256, 0, s>>>(jobs, k, group, work, x, col_off, skip);
  };
  using L = std::integral_constant<int, MODE_L>;
  using U = std::integral_constant<int, MODE_U>;
  using UT = std::integral_constant<int, MODE_UT>;
  using LT = std::integral_constant<int, MODE_LT>;
  if (!trans) {
    for (int k = 0; k < npad_max; k += GW) {
      diag(L{}, k);
      update(L{}, k, (npad_max - k - GW) / 64);
    }
    for (int k = last; k >= 0; k -= GW) {
      diag(U{}, k);
      update(U{}, k, k / 64);
    }
  } else if constexpr (std::is_same<XT, double2>::value) {  // transposed solves: FP64 only
    for (int k = 0; k < npad_max; k += GW) {
      diag(UT{}, k);
      update(UT{}, k, (npad_max - k - GW) / 64);
    }
    for (int k = last; k >= 0; k -= GW) {
      update(LT{}, k, (npad_max - k - GW) / 64);
      diag(LT{}, k);
    }
  }
}

template <typename T>
static void solve_dispatch(const JobDesc* jobs, int njobs, int npad_max, const T* work, const int32_t* piv,
                           double2* x, int64_t col_off, int nrhs, int trans, int group, const int32_t* skip,
                           hipStream_t s) {
  if (nrhs == 16)
    solve_all<T, double2, 16>(jobs, njobs, npad_max, work, piv, x, col_off, trans, group, skip, s);
  else
    solve_all<T, double2, 32>(jobs, njobs, npad_max, work, piv, x, col_off, trans, group, skip, s);
}

void lu_solve_f64(const JobDesc* jobs, int njobs, int npad_max, const double2* work, const int32_t* piv,
                  double2* x, int64_t x_col_off, int nrhs, int trans, int group, hipStream_t s) {
  solve_dispatch<double2>(jobs, njobs, npad_max, work, piv, x, x_col_off, nrhs, trans, group, nullptr, s);
}

void lu_solve_f32(const JobDesc* jobs, int njobs, int npad_max, const float2* work, const int32_t* piv,
                  double2* x, int64_t x_col_off, int nrhs, int trans, int group, hipStream_t s) {
  solve_dispatch<float2>(jobs, njobs, npad_max, work, piv, x, x_col_off, nrhs, trans, group, nullptr, s);
}

void lu_solve_f32_single(const JobDesc* jobs, int njobs, int npad_max, const float2* work, const int32_t* piv,
                         double2* x, const int32_t* skip, int group, hipStream_t s) {
  solve_all<float2, float2, 16>(jobs, njobs, npad_max, work, piv, x, 0, 0, group, skip, s);
}

}  // namespace lsms
