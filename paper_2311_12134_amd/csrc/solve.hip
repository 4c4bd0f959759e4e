// Solves with the blocked LU factors (forward substitution, back substitution, and the
// transposed pair used by the adjoint).
//
// The factorization is the product M = P_1^T L_1 P_2^T L_2 ... P_K^T L_K U of panel
// permutations P_p and unit-lower panel factors L_p (stored in the panel's columns,
// never re-permuted by later panels; the factorization leaves the inverses of the unit
// lower and the upper diagonal triangles in each diagonal block).  Hence
//   M X = B   :  X = U^-1 L_K^-1 P_K ... L_1^-1 P_1 B          (trans = 0)
//   M^T X = B :  X = P_1^T L_1^-T ... P_K^T L_K^-T U^-T B      (trans = 1)
// Every panel costs two launches over the whole batch:
//   solve_diag_kernel    one workgroup per job: the panel's permutation as one gather of
//                        at most 2 NB rows, then the NB x NB diagonal block as a product
//                        with the stored inverse (L11^-1, U11^-1 or their transposes) on
//                        FP64 MFMA;
//   solve_update_kernel  one workgroup per (64-row strip, job): the off-diagonal block
//                        times the panel's NB solved rows, on FP64 MFMA 16x16x4 (four real
//                        products per complex product) from LDS-staged tiles, so the
//                        factors stream from HBM once per solve.
// The update is column-oriented (rows below for L and U^T, rows above for U) except for
// L^T, whose panel rows need a sum over all rows below: there every strip adds its
// partial product to the panel rows with FP64 atomics.  Arithmetic is FP64 for both
// storage types of the factors.
#include "lsms_internal.h"
#include "strip_mma.h"

namespace lsms {

typedef double d4 __attribute__((ext_vector_type(4)));

enum { MODE_L = 0, MODE_U = 1, MODE_UT = 2, MODE_LT = 3 };

// One panel permutation of the solution rows (at most PERM_MAX (dst, src) pairs): every
// source row is read into registers before any destination row is written.
template <int NRHS>
__device__ inline void apply_perm(const int32_t* lst, bool inverse, double2* X, int* s_dst, int* s_src, int t) {
  constexpr int HELD = PERM_MAX * NRHS / 256;
  const int cnt = lst[0];
  for (int i = t; i < cnt; i += 256) {
    s_dst[i] = lst[2 + i];
    s_src[i] = lst[2 + PERM_MAX + i];
  }
  __syncthreads();
  const int* from = inverse ? s_dst : s_src;
  const int* to = inverse ? s_src : s_dst;
  double2 held[HELD];
#pragma unroll
  for (int u = 0; u < HELD; ++u) {
    const int idx = t + 256 * u, i = idx / NRHS, c = idx % NRHS;
    held[u] = i < cnt ? X[(int64_t)from[i] * NRHS_MAX + c] : make_double2(0.0, 0.0);
  }
  __syncthreads();
#pragma unroll
  for (int u = 0; u < HELD; ++u) {
    const int idx = t + 256 * u, i = idx / NRHS, c = idx % NRHS;
    if (i < cnt) X[(int64_t)to[i] * NRHS_MAX + c] = held[u];
  }
  __syncthreads();
}

template <typename T, int NRHS, int MODE>
__global__ __launch_bounds__(256) void solve_diag_kernel(const JobDesc* jobs, int k, const T* work,
                                                         const int32_t* piv, double2* xbuf, int64_t col_off,
                                                         const int32_t* skip) {
  const int job = blockIdx.x;
  if (skip && skip[job]) return;
  const JobDesc jd = jobs[job];
  if (k >= jd.npad) return;  // uniform
  const T* A = work + jd.a_off;
  const int64_t ld = jd.npad;
  const int32_t* pv = piv + jd.piv_off;
  double2* X = xbuf + jd.x_off + col_off;
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  constexpr int HELD = PERM_MAX * NRHS / 256;
  typedef typename LdsOf<T>::type S;
  __shared__ S s_T[NB][NB + 1];
  __shared__ double2 s_X[NB][NRHS];
  __shared__ int s_dst[PERM_MAX], s_src[PERM_MAX];
  auto xrow = [&](int r) { return X + (int64_t)r * NRHS_MAX; };
  auto permute = [&](int kp, bool inverse) {
    apply_perm<NRHS>(pv + perm_off(jd.npad, kp), inverse, X, s_dst, s_src, t);
  };
  // Panels come in pairs (first at multiples of 2 NB, see lu_factor): the first panel's
  // L rows are stored after the second panel's permutation, so the forward solve applies
  // that permutation right after the first triangle, and the transposed solve undoes both
  // permutations after the first triangle.
  const bool first = (k % (2 * NB)) == 0;
  const bool has_second = first && (k + NB < jd.npad);
  if (MODE == MODE_L && first) permute(k, false);
  // the diagonal block holds L11^-1 below the diagonal (unit diagonal implied) and U11^-1 on
  // and above it; the step is a product with the needed inverse (transposed for U^T, L^T)
  const bool upper = (MODE == MODE_U || MODE == MODE_UT);
  for (int idx = t; idx < NB * NB; idx += 256) {
    const int q = idx / NB, pp = idx % NB;
    if (upper)
      s_T[q][pp] = pp >= q ? A[(k + q) * ld + k + pp] : S{0, 0};
    else
      st2(&s_T[q][pp], pp < q ? ld2(A + (k + q) * ld + k + pp) : make_double2(pp == q ? 1.0 : 0.0, 0.0));
  }
  for (int idx = t; idx < NB * NRHS; idx += 256) s_X[idx / NRHS][idx % NRHS] = xrow(k + idx / NRHS)[idx % NRHS];
  __syncthreads();
  {
    // wave w writes rows 16w .. 16w+16 of the panel
    constexpr bool TRANS = (MODE == MODE_UT || MODE == MODE_LT);
    StripMma<double2, NRHS / 16> y;
    y.zero();
    y.run([&](int i, int kk) { return TRANS ? ld2(&s_T[kk][wave * 16 + i]) : ld2(&s_T[wave * 16 + i][kk]); },
          [&](int kk, int c) { return s_X[kk][c]; }, lane);
    const int ii = lane & 15;
#pragma unroll
    for (int cb = 0; cb < NRHS / 16; ++cb)
#pragma unroll
      for (int r = 0; r < 4; ++r) xrow(k + wave * 16 + y.row(r, lane))[cb * 16 + ii] = y.value(cb, r);
  }
  if (MODE == MODE_L && has_second) {
    __syncthreads();
    permute(k + NB, false);
  }
  if (MODE == MODE_LT && first) {
    __syncthreads();
    if (has_second) permute(k + NB, true);
    permute(k, true);
  }
}

// One 64-row strip:  MODE_L   X[s] -= L[s, P] X[P]      (s below the panel P)
//                    MODE_U   X[s] -= U[s, P] X[P]      (s above the panel)
//                    MODE_UT  X[s] -= U[P, s]^T X[P]    (s below)
//                    MODE_LT  X[P] -= L[s, P]^T X[s]    (s below; atomics into the panel rows)
// out (64 x NRHS) = A (64 x NB) B (NB x NRHS) with K chunks of 32 staged in LDS.
template <typename T, int NRHS, int MODE>
__global__ __launch_bounds__(256) void solve_update_kernel(const JobDesc* jobs, int k, const T* work,
                                                           double2* xbuf, int64_t col_off, const int32_t* skip) {
  const int job = blockIdx.y;
  if (skip && skip[job]) return;
  const JobDesc jd = jobs[job];
  const int s0 = (MODE == MODE_U) ? blockIdx.x * 64 : k + NB + blockIdx.x * 64;  // strip rows
  if (k >= jd.npad) return;
  if (MODE == MODE_U ? (s0 >= k) : (s0 >= jd.npad)) return;  // uniform
  const T* A = work + jd.a_off;
  const int64_t ld = jd.npad;
  double2* X = xbuf + jd.x_off + col_off;
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  constexpr int KC = 32;
  constexpr int CB = NRHS / 16;  // 16-column output blocks per wave
  typedef typename LdsOf<T>::type S;
  __shared__ S sA[KC][64 + 1];            // sA[kk][o]: A[o][k0 + kk] for output row o
  __shared__ double2 sB[NB][NRHS + 1];    // right-hand operand, NB x NRHS
  // right-hand operand: the panel rows (L, U, UT) or the strip rows (LT)
  const int brow = (MODE == MODE_LT) ? s0 : k;
  for (int idx = t; idx < NB * NRHS; idx += 256)
    sB[idx / NRHS][idx % NRHS] = X[(int64_t)(brow + idx / NRHS) * NRHS_MAX + idx % NRHS];
  d4 are[CB], aim[CB];
#pragma unroll
  for (int cb = 0; cb < CB; ++cb) {
    are[cb] = d4{0, 0, 0, 0};
    aim[cb] = d4{0, 0, 0, 0};
  }
  const int ii = lane & 15, kq = lane >> 4;
  for (int k0 = 0; k0 < NB; k0 += KC) {
    __syncthreads();
    // stage A[o][k0 .. k0+KC) for the 64 output rows o into sA[kk][o]
    for (int idx = t; idx < KC * 64; idx += 256) {
      if (MODE == MODE_L || MODE == MODE_U) {
        const int o = idx / KC, kk = idx % KC;  // consecutive threads walk a row
        sA[kk][o] = A[(int64_t)(s0 + o) * ld + k + k0 + kk];
      } else if (MODE == MODE_UT) {
        const int kk = idx / 64, o = idx % 64;  // U[k + k0 + kk][s0 + o]
        sA[kk][o] = A[(int64_t)(k + k0 + kk) * ld + s0 + o];
      } else {
        const int kk = idx / 64, o = idx % 64;  // L[s0 + k0 + kk][k + o]: sum over strip rows
        sA[kk][o] = A[(int64_t)(s0 + k0 + kk) * ld + k + o];
      }
    }
    __syncthreads();
#pragma unroll
    for (int k4 = 0; k4 < KC; k4 += 4) {
      const double2 a = ld2(&sA[k4 + kq][wave * 16 + ii]);
#pragma unroll
      for (int cb = 0; cb < CB; ++cb) {
        const double2 b = sB[k0 + k4 + kq][cb * 16 + ii];
        are[cb] = __builtin_amdgcn_mfma_f64_16x16x4f64(a.x, b.x, are[cb], 0, 0, 0);
        are[cb] = __builtin_amdgcn_mfma_f64_16x16x4f64(-a.y, b.y, are[cb], 0, 0, 0);
        aim[cb] = __builtin_amdgcn_mfma_f64_16x16x4f64(a.x, b.y, aim[cb], 0, 0, 0);
        aim[cb] = __builtin_amdgcn_mfma_f64_16x16x4f64(a.y, b.x, aim[cb], 0, 0, 0);
      }
    }
  }
  // D lane l, register r -> output row 16 wave + l/16 + 4r, column 16 cb + l%16
  const int orow0 = (MODE == MODE_LT) ? k : s0;
#pragma unroll
  for (int cb = 0; cb < CB; ++cb)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int o = wave * 16 + kq + 4 * r, c = cb * 16 + ii;
      double2* xp = X + (int64_t)(orow0 + o) * NRHS_MAX + c;
      if (MODE == MODE_LT) {
        atomicAdd(&xp->x, -are[cb][r]);
        atomicAdd(&xp->y, -aim[cb][r]);
      } else {
        double2 v = *xp;
        v.x -= are[cb][r];
        v.y -= aim[cb][r];
        *xp = v;
      }
    }
}

template <typename T, int NRHS, int MODE>
static void diag(const JobDesc* jobs, int njobs, int k, const T* work, const int32_t* piv, double2* x,
                 int64_t col_off, const int32_t* skip, hipStream_t s) {
  solve_diag_kernel<T, NRHS, MODE><<<njobs, 256, 0, s>>>(jobs, k, work, piv, x, col_off, skip);
}

template <typename T, int NRHS, int MODE>
static void update(const JobDesc* jobs, int njobs, int k, int strips, const T* work, double2* x, int64_t col_off,
                   const int32_t* skip, hipStream_t s) {
  if (strips <= 0) return;
  solve_update_kernel<T, NRHS, MODE><<<dim3(strips, njobs), 256, 0, s>>>(jobs, k, work, x, col_off, skip);
}

template <typename T, int NRHS>
static void solve_all(const JobDesc* jobs, int njobs, int npad_max, const T* work, const int32_t* piv, double2* x,
                      int64_t col_off, int trans, const int32_t* skip, hipStream_t s) {
  if (!trans) {
    for (int k = 0; k < npad_max; k += NB) {
      diag<T, NRHS, MODE_L>(jobs, njobs, k, work, piv, x, col_off, skip, s);
      update<T, NRHS, MODE_L>(jobs, njobs, k, (npad_max - k - NB) / 64, work, x, col_off, skip, s);
    }
    for (int k = npad_max - NB; k >= 0; k -= NB) {
      diag<T, NRHS, MODE_U>(jobs, njobs, k, work, piv, x, col_off, skip, s);
      update<T, NRHS, MODE_U>(jobs, njobs, k, k / 64, work, x, col_off, skip, s);
    }
  } else {
    for (int k = 0; k < npad_max; k += NB) {
      diag<T, NRHS, MODE_UT>(jobs, njobs, k, work, piv, x, col_off, skip, s);
      update<T, NRHS, MODE_UT>(jobs, njobs, k, (npad_max - k - NB) / 64, work, x, col_off, skip, s);
    }
    for (int k = npad_max - NB; k >= 0; k -= NB) {
      update<T, NRHS, MODE_LT>(jobs, njobs, k, (npad_max - k - NB) / 64, work, x, col_off, skip, s);
      diag<T, NRHS, MODE_LT>(jobs, njobs, k, work, piv, x, col_off, skip, s);
    }
  }
}

template <typename T>
static void solve_dispatch(const JobDesc* jobs, int njobs, int npad_max, const T* work, const int32_t* piv,
                           double2* x, int64_t col_off, int nrhs, int trans, const int32_t* skip, hipStream_t s) {
  if (nrhs == 16)
    solve_all<T, 16>(jobs, njobs, npad_max, work, piv, x, col_off, trans, skip, s);
  else
    solve_all<T, 32>(jobs, njobs, npad_max, work, piv, x, col_off, trans, skip, s);
}

void lu_solve_f64(const JobDesc* jobs, int njobs, int npad_max, const double2* work, const int32_t* piv,
                  double2* x, int64_t x_col_off, int nrhs, int trans, hipStream_t s) {
  solve_dispatch<double2>(jobs, njobs, npad_max, work, piv, x, x_col_off, nrhs, trans, nullptr, s);
}

void lu_solve_f32(const JobDesc* jobs, int njobs, int npad_max, const float2* work, const int32_t* piv,
                  double2* x, int64_t x_col_off, int nrhs, int trans, hipStream_t s) {
  solve_dispatch<float2>(jobs, njobs, npad_max, work, piv, x, x_col_off, nrhs, trans, nullptr, s);
}

void lu_solve_f32_skip(const JobDesc* jobs, int njobs, int npad_max, const float2* work, const int32_t* piv,
                       double2* x, const int32_t* skip, hipStream_t s) {
  solve_dispatch<float2>(jobs, njobs, npad_max, work, piv, x, 0, 16, 0, skip, s);
}

}  // namespace lsms
