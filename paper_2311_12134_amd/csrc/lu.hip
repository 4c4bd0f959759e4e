// Batched complex LU with partial pivoting (the tau inverse of Eq. (3) is the dominant
// cost of the method, Sec. II.A), blocked with panel width NB: right-looking over groups of
// 2 to 4 panels, left-looking within a group (see lu_factor_any).
//
// All jobs of a wave advance through the same panel steps; every panel is a few
// launches over the whole batch:
//   panel_kernel      one workgroup per job factors rows [k, n) x cols [k, k+NB) with
//                     partial pivoting (pivot = largest |re|+|im|, first on ties, keys
//                     compared in FP64): IB-wide leaves live in registers (rows distributed
//                     cyclically over the workgroup) and are updated in the storage
//                     precision, every pivot swaps the whole panel row, and the rest of the
//                     panel is updated by the leaf (triangular solve + rank-IB).
//   swap_trsm_kernel  applies the panel's row interchanges to the trailing columns and
//                     forms U12 = L11^-1 A12 (one workgroup per 64-column tile).
//   gemm_*_kernel     (gemm.hip) trailing update A22 -= L21 U12 on the matrix cores:
//                     FP64 MFMA 16x16x4 with the four real products of a complex product,
//                     or (split mode) FP32 MFMA 16x16x4 with three real products
//                     (Ar Br, Ai Bi, (Ar+Ai)(Br+Bi)).
// Interchanges are applied only to the right of each panel (and to the L columns of the
// earlier panels of its group); the solves apply them panel by panel in the same order,
// so the columns of earlier groups never need swapping.
// Matrices are row-major with leading dimension npad (a multiple of 64); the padding
// is an identity block that no pivot ever selects.
#include <algorithm>

#include "lsms_internal.h"
#include "strip_mma.h"
#include "tri.h"

namespace lsms {

typedef double d4 __attribute__((ext_vector_type(4)));

// ------------------------------------------------------------------------------------
// panel factorization
// ------------------------------------------------------------------------------------
// Pivot keys: a non-negative double orders like its bit pattern, so the magnitude with
// its 13 lowest mantissa bits replaced by (8191 - local row) is one 64-bit integer whose
// maximum is the largest magnitude, the lowest row on ties (relative resolution 2^-39).
// NaN magnitudes get key 0 and never win; key 0 overall means "keep the diagonal row".
__device__ inline unsigned long long pivot_key(double mag, int row_local) {
  if (!(mag == mag)) return 0ull;
  return ((unsigned long long)__double_as_longlong(mag) & ~0x1FFFull) | (unsigned long long)(0x1FFF - row_local);
}
__device__ inline int pivot_row(unsigned long long key) { return 0x1FFF - (int)(key & 0x1FFFull); }

// One lane's 64-bit key moved within its 16-lane row by the DPP pattern CTRL.
template <int CTRL>
__device__ inline unsigned long long dpp_key(unsigned long long x) {
  const int lo = (int)(unsigned)x, hi = (int)(unsigned)(x >> 32);
  const unsigned rlo = (unsigned)__builtin_amdgcn_update_dpp(lo, lo, CTRL, 0xF, 0xF, false);
  const unsigned rhi = (unsigned)__builtin_amdgcn_update_dpp(hi, hi, CTRL, 0xF, 0xF, false);
  return ((unsigned long long)rhi << 32) | rlo;
}
__device__ inline unsigned long long umax64(unsigned long long a, unsigned long long b) { return a > b ? a : b; }
__device__ inline unsigned long long lane_key(unsigned long long x, int l) {
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)x, l);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(x >> 32), l);
  return ((unsigned long long)hi << 32) | lo;
}
// Largest key of the wavefront, the same in every lane: the maximum within each 16-lane
// row by DPP (quad exchanges 1 and 2, half-row mirror, row mirror; each step combines
// groups that already agree), then the four rows' maxima read as scalars.
__device__ inline unsigned long long wave_max_key(unsigned long long key) {
  key = umax64(key, dpp_key<0xB1>(key));   // quad_perm [1, 0, 3, 2]
  key = umax64(key, dpp_key<0x4E>(key));   // quad_perm [2, 3, 0, 1]
  key = umax64(key, dpp_key<0x141>(key));  // row_half_mirror
  key = umax64(key, dpp_key<0x140>(key));  // row_mirror
  return umax64(umax64(lane_key(key, 0), lane_key(key, 16)), umax64(lane_key(key, 32), lane_key(key, 48)));
}

// Inverse of a pivot in FP64.  Values stored in FP32 have squared magnitudes well inside
// the FP64 range, so conj(a) / |a|^2 needs one division; FP64 storage keeps the scaled
// (Smith) form.
__device__ inline double2 pivot_inverse(double2 a, float2) {
  const double rn = 1.0 / (a.x * a.x + a.y * a.y);
  return make_double2(a.x * rn, -a.y * rn);
}
__device__ inline double2 pivot_inverse(double2 a, double2) { return cinv(a); }

// a - b c for the leaf's rank-1 updates: each component as two fused multiply-adds (two
// roundings, where the product-then-difference form takes three operations and three roundings)
__device__ inline float2 leaf_fms(float2 a, float2 b, float2 c) {
  return make_float2(__builtin_fmaf(-b.x, c.x, __builtin_fmaf(b.y, c.y, a.x)),
                     __builtin_fmaf(-b.x, c.y, __builtin_fmaf(-b.y, c.x, a.y)));
}
__device__ inline double2 leaf_fms(double2 a, double2 b, double2 c) {
  return make_double2(__builtin_fma(-b.x, c.x, __builtin_fma(b.y, c.y, a.x)),
                      __builtin_fma(-b.x, c.y, __builtin_fma(-b.y, c.x, a.y)));
}

__device__ inline double2 wide(double2 a) { return a; }
__device__ inline double2 wide(float2 a) { return make_double2((double)a.x, (double)a.y); }
__device__ inline void narrow_to(double2& d, double2 a) { d = a; }
__device__ inline void narrow_to(float2& d, double2 a) { d = make_float2((float)a.x, (float)a.y); }

// IB consecutive elements of one row, moved 16 bytes at a time (rows start 16-byte aligned)
template <int IB>
__device__ inline void load_row(const float2* p, float2 (&d)[IB]) {
#pragma unroll
  for (int u = 0; u < IB / 2; ++u) {
    const float4 x = ((const float4*)p)[u];
    d[2 * u] = make_float2(x.x, x.y);
    d[2 * u + 1] = make_float2(x.z, x.w);
  }
}
template <int IB>
__device__ inline void load_row(const double2* p, double2 (&d)[IB]) {
#pragma unroll
  for (int u = 0; u < IB; ++u) d[u] = p[u];
}
template <int IB>
__device__ inline void store_row(float2* p, const float2 (&d)[IB]) {
#pragma unroll
  for (int u = 0; u < IB / 2; ++u) ((float4*)p)[u] = make_float4(d[2 * u].x, d[2 * u].y, d[2 * u + 1].x, d[2 * u + 1].y);
}
template <int IB>
__device__ inline void store_row(double2* p, const double2 (&d)[IB]) {
#pragma unroll
  for (int u = 0; u < IB; ++u) p[u] = d[u];
}
// Orders LDS traffic between the lanes of one wavefront (its LDS operations run in order).
__device__ inline void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// The NB interchanges of a panel starting at row k (pivall[q]: the row exchanged with
// k + q at step q) as one permutation of at most 2 NB rows, written to lst: entries
// 0..NB-1 are the positions k..k+NB-1, further entries the pivot rows below the panel;
// org[e] is the original row that ends up at position pos[e].  Executed by one wavefront;
// returns the number of entries (the same in every lane).
__device__ inline int write_perm_list(int k, const int* pivall, int* s_pos, int* s_org, int32_t* lst, int lane) {
  for (int i = lane; i < NB; i += 64) {
    s_pos[i] = k + i;
    s_org[i] = k + i;
  }
  int cnt = NB;
  for (int q = 0; q < NB; ++q) {
    const int d = k + q, p = pivall[q];
    if (p == d) continue;
    int e;
    if (p < k + NB) {
      e = p - k;
    } else {
      const unsigned long long m = __ballot(NB + lane < cnt && s_pos[NB + lane] == p);
      if (m) {
        e = NB + __ffsll((long long)m) - 1;
      } else {
        e = cnt;
        if (lane == 0) {
          s_pos[cnt] = p;
          s_org[cnt] = p;
        }
        ++cnt;
      }
    }
    if (lane == 0) {
      const int tmp = s_org[q];
      s_org[q] = s_org[e];
      s_org[e] = tmp;
    }
  }
  if (lane == 0) lst[0] = cnt;
  for (int i = lane; i < cnt; i += 64) {
    lst[2 + i] = s_pos[i];
    lst[2 + PERM_MAX + i] = s_org[i];
  }
  return cnt;
}

// nopiv: keep the diagonal row at every step (the symmetric factorization below); the
// permutation list is then the identity.
template <typename T, int PT, int S, int IB>
__global__ __launch_bounds__(PT) void panel_kernel(const JobDesc* jobs, int k, int left, T* work, int32_t* piv,
                                                   int32_t* info, int nopiv) {
  const JobDesc jd = jobs[blockIdx.x];
  if (k >= jd.npad) return;  // uniform over the workgroup
  T* A = work + jd.a_off;
  const int64_t ld = jd.ld > 0 ? jd.ld : jd.npad;
  const int nrows = jd.npad;
  int32_t* ip = piv + jd.piv_off;
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  constexpr int NW = PT / 64;

  // Per pivot column one barrier: before it every wave posts its best key (LDS atomic
  // max into one of three rotating slots) and its candidate row, and the owner of the
  // diagonal row posts that row (two rotating buffers); after it every thread knows the
  // pivot row and both rows to exchange.  Column j clears slot (j + 1) % 3: its last
  // readers (column j - 2) passed barrier j - 1 before anyone reaches column j, and its
  // next writers (column j + 1) start after barrier j.  A row buffer written before
  // barrier j is rewritten only before barrier j + 2, after every read of column j.
  __shared__ unsigned long long s_key[3];
  __shared__ T s_cand[2][NW][IB];
  __shared__ T s_drow[2][IB];
  __shared__ int s_piv[IB];
  __shared__ double2 s_L11[IB][IB];
  __shared__ double2 s_U[IB][NB];
  __shared__ int s_pivall[NB];
  __shared__ int s_pos[PERM_MAX], s_org[PERM_MAX];
  __shared__ int s_lpos[2 * IB], s_lorg[2 * IB], s_lcnt;
  __shared__ T s_held[2 * IB][2 * NB - IB];
  // The next leaf stays on chip for 16-wide FP32 leaves of at most half of the registers and
  // for the 256-thread kernels' 8-wide FP32 leaves of one or two row slots (the other shapes
  // run out of registers or occupancy with it).
  constexpr bool KEEP_NEXT = sizeof(T) == sizeof(float2) && (IB == 16 || (PT == 256 && S <= 2)) && S * IB * 2 <= 128;
  // FP32 leaves move between memory and the row-per-thread registers through the wave's own
  // rows of s_X: a row of IB FP32 complex values is IB / 2 16-byte chunks, so a wavefront's
  // 16-byte access covers 64 / (IB / 2) whole rows (full 128- or 64-byte lines) instead of one
  // chunk of 64 different rows, which costs one L2 request per lane and is the slow part of
  // storing a leaf.  The same rows carry the next leaf out of the rank update.
  constexpr bool STAGE = sizeof(T) == sizeof(float2);
  constexpr int CPR = IB / 2, RPI = 64 / CPR;  // chunks per leaf row, rows per staged access
  __shared__ T s_X[STAGE ? PT : 1][IB + 1];  // one row per thread (wave-private rows)

  // the leaf in registers in the storage precision (its updates too; pivot keys in FP64)
  T v[S][IB];
  int first_zero = 0;
  if (t < 3) s_key[t] = 0ull;
  __syncthreads();
  int col = 0;  // pivot columns done so far (selects the rotating slots)

  for (int c = 0; c < NB / IB; ++c) {
    const int cl = k + c * IB;
    if (c == 0 || !KEEP_NEXT) {  // otherwise the leaf came from the previous leaf's rank update
      if constexpr (STAGE) {
        const int ch = lane % CPR, rsub = lane / CPR;
        int kb = k;
        asm volatile("" : "+s"(kb));  // row addresses are formed here, not held across the leaves
#pragma unroll
        for (int s = 0; s < S; ++s) {
          const int rw = kb + s * PT + wave * 64;  // the wave's first row in this slot
          if (rw >= nrows) {                      // uniform per wave
#pragma unroll
            for (int q = 0; q < IB; ++q) v[s][q] = T{0, 0};
            continue;
          }
          float4 x[CPR];
#pragma unroll
          for (int u = 0; u < CPR; ++u) {
            const int r = rw + u * RPI + rsub;
            x[u] = (r >= cl && r < nrows) ? *(const float4*)(A + r * ld + cl + 2 * ch) : make_float4(0.f, 0.f, 0.f, 0.f);
          }
#pragma unroll
          for (int u = 0; u < CPR; ++u) {
            T* d = s_X[wave * 64 + u * RPI + rsub] + 2 * ch;
            d[0] = T{x[u].x, x[u].y};
            d[1] = T{x[u].z, x[u].w};
          }
          wave_sync();
#pragma unroll
          for (int q = 0; q < IB; ++q) v[s][q] = s_X[t][q];
          wave_sync();  // every lane has its row before the next slot rewrites them
        }
      } else {
#pragma unroll
        for (int s = 0; s < S; ++s) {
          const int r = k + t + s * PT;
          if (r >= cl && r < nrows) {
            load_row<IB>(A + r * ld + cl, v[s]);
          } else {
#pragma unroll
            for (int q = 0; q < IB; ++q) v[s][q] = T{0, 0};
          }
        }
      }
    }
#pragma clang loop unroll(full)
    for (int j = 0; j < IB; ++j, ++col) {
      const int d = cl + j;
      const int buf = col & 1;
      unsigned long long key = 0ull;
#pragma unroll
      for (int s = 0; s < S; ++s) {
        const int r = k + t + s * PT;
        if (!nopiv && r >= d && r < nrows) {
          const double2 e = wide(v[s][j]);
          const unsigned long long kk = pivot_key(fabs(e.x) + fabs(e.y), r - k);
          key = kk > key ? kk : key;
        }
      }
      key = wave_max_key(key);
      if (key != 0ull) {  // the lane holding the wave's best row posts it (never with nopiv)
        const int rl = pivot_row(key);
        if (rl % PT == t) {
#pragma unroll
          for (int s = 0; s < S; ++s)
            if (s == rl / PT) {
#pragma unroll
              for (int q = 0; q < IB; ++q) s_cand[buf][wave][q] = v[s][q];
            }
        }
      }
      if (lane == 0) atomicMax(&s_key[col % 3], key);
      const int od = (d - k) % PT, sd = (d - k) / PT;
      if (t == od) {
#pragma unroll
        for (int s = 0; s < S; ++s)
          if (s == sd) {
#pragma unroll
            for (int q = 0; q < IB; ++q) s_drow[buf][q] = v[s][q];
          }
      }
      if (t == 0) s_key[(col + 1) % 3] = 0ull;
      __syncthreads();
      // every lane reads the same key: taking it as a scalar makes the pivot row, its slot and
      // the row buffers uniform, so the interchange below branches per wavefront
      const unsigned long long bk = s_key[col % 3];
      const unsigned long long best =
          ((unsigned long long)(unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)(bk >> 32)) << 32) |
          (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)bk);
      int p = best != 0ull ? k + pivot_row(best) : d;
      const bool from_cand = best != 0ull && p >= d && p < nrows;
      if (!from_cand) p = d;
      const T* prow = from_cand ? s_cand[buf][((p - k) % PT) / 64] : s_drow[buf];
      const int op = (p - k) % PT, sp = (p - k) / PT;
      if (t == 0) {
        s_piv[j] = p;
        s_pivall[c * IB + j] = p;
        ip[d] = p;
      }
      if (t == od) {
#pragma unroll
        for (int s = 0; s < S; ++s)
          if (s == sd) {
#pragma unroll
            for (int q = 0; q < IB; ++q) v[s][q] = prow[q];
          }
      }
      if (t == op && p != d) {
#pragma unroll
        for (int s = 0; s < S; ++s)
          if (s == sp) {
#pragma unroll
            for (int q = 0; q < IB; ++q) v[s][q] = s_drow[buf][q];
          }
      }
      const double2 pv = wide(prow[j]);
      const bool zero = (pv.x == 0.0 && pv.y == 0.0);
      if (zero && first_zero == 0) first_zero = d + 1;
      T inv;  // the pivot's inverse in FP64, rounded once to the storage precision
      narrow_to(inv, zero ? make_double2(0.0, 0.0) : pivot_inverse(pv, T{}));
      // the leaf's rank-1 update in the storage precision (FP32 in split mode, like the
      // trailing updates; the pivot keys above compare these values in FP64).  While the
      // leaf takes at most half of the registers, rows on or above the pivot take a zero
      // multiplier (which leaves them as they are) so the update has no branches, and each
      // pivot-row entry is read from LDS once for all S row slots; wider leaves (and eight
      // row slots) update the slots one by one under a branch, which keeps fewer values live.
      if constexpr (S * IB * (int)sizeof(T) / 4 <= 128 && S < 8) {
        T l[S];
#pragma unroll
        for (int s = 0; s < S; ++s) {
          const int r = k + t + s * PT;
          const bool below = r > d && r < nrows;
          l[s] = below ? cmul(v[s][j], inv) : T{0, 0};
          if (below) v[s][j] = l[s];
        }
#pragma unroll
        for (int q = 0; q < IB; ++q) {  // full range: j is a constant once unrolled
          if (q > j) {
            const T pq = prow[q];
#pragma unroll
            for (int s = 0; s < S; ++s) v[s][q] = leaf_fms(v[s][q], l[s], pq);
          }
        }
      } else {
#pragma unroll
        for (int s = 0; s < S; ++s) {
          const int r = k + t + s * PT;
          if (r > d && r < nrows) {
            const T l = cmul(v[s][j], inv);
            v[s][j] = l;
#pragma unroll
            for (int q = 0; q < IB; ++q)
              if (q > j) v[s][q] = leaf_fms(v[s][q], l, prow[q]);
          }
        }
      }
    }
    // the leaf's diagonal block to LDS, then the leaf back to memory (the registers of a row
    // slot are free once it is staged)
#pragma unroll
    for (int s = 0; s < S; ++s) {
      const int r = k + t + s * PT;
      if (r >= cl && r < cl + IB) {
#pragma unroll
        for (int q = 0; q < IB; ++q) s_L11[r - cl][q] = wide(v[s][q]);
      }
    }
    if constexpr (STAGE) {
      const int ch = lane % CPR, rsub = lane / CPR;
      int kb = k;
      asm volatile("" : "+s"(kb));  // row addresses are formed here, not held across the leaves
#pragma unroll
      for (int s = 0; s < S; ++s) {
        const int rw = kb + s * PT + wave * 64;
        if (rw + 64 <= cl || rw >= nrows) continue;  // uniform per wave
#pragma unroll
        for (int q = 0; q < IB; ++q) s_X[t][q] = v[s][q];
        wave_sync();
#pragma unroll
        for (int u = 0; u < CPR; ++u) {
          const int r = rw + u * RPI + rsub;
          const T* e = s_X[wave * 64 + u * RPI + rsub] + 2 * ch;
          const T e0 = e[0], e1 = e[1];
          if (r >= cl && r < nrows) *(float4*)(A + r * ld + cl + 2 * ch) = make_float4(e0.x, e0.y, e1.x, e1.y);
        }
        wave_sync();  // read before the next slot rewrites the rows
      }
    } else {
#pragma unroll
      for (int s = 0; s < S; ++s) {
        const int r = k + t + s * PT;
        if (r >= cl && r < nrows) store_row<IB>(A + r * ld + cl, v[s]);
      }
    }
    __syncthreads();
    // the leaf's interchanges on the other columns of the panel (whole panel rows), and on
    // the `left` columns before it (the earlier panels of its group, see lu_factor_any),
    // applied as one gather: at most 2 IB rows change, listed as (position, original row)
    // pairs, moved through LDS in chunks of 2 NB - IB columns
    if (t == 0) {
      int cnt = IB;
      for (int i = 0; i < IB; ++i) {
        s_lpos[i] = cl + i;
        s_lorg[i] = cl + i;
      }
      for (int q = 0; q < IB; ++q) {
        const int d = cl + q, p = s_piv[q];
        if (p == d || p <= d || p >= nrows) continue;
        int e = -1;
        if (p < cl + IB) {
          e = p - cl;
        } else {
          for (int i = IB; i < cnt; ++i)
            if (s_lpos[i] == p) e = i;
          if (e < 0) {
            e = cnt++;
            s_lpos[e] = p;
            s_lorg[e] = p;
          }
        }
        const int tmp = s_lorg[q];
        s_lorg[q] = s_lorg[e];
        s_lorg[e] = tmp;
      }
      s_lcnt = cnt;
    }
    __syncthreads();
    {
      constexpr int CH = 2 * NB - IB;
      const int ncols = left + NB - IB, cnt = s_lcnt;
      for (int c0 = 0; c0 < ncols; c0 += CH) {
        const int nc = min(CH, ncols - c0);
        if (c0 > 0) __syncthreads();  // the previous chunk is written back
        for (int idx = t; idx < cnt * nc; idx += PT) {
          const int e = idx / nc, ch = idx - e * nc, cc = c0 + ch, cr = cc - left;
          const int colx = cc < left ? k - left + cc : k + (cr < c * IB ? cr : cr + IB);
          s_held[e][ch] = A[s_lorg[e] * ld + colx];
        }
        __syncthreads();
        for (int idx = t; idx < cnt * nc; idx += PT) {
          const int e = idx / nc, ch = idx - e * nc, cc = c0 + ch, cr = cc - left;
          const int colx = cc < left ? k - left + cc : k + (cr < c * IB ? cr : cr + IB);
          A[s_lpos[e] * ld + colx] = s_held[e][ch];
        }
      }
    }
    __syncthreads();
    const int w = k + NB - cl - IB;  // panel columns right of the leaf
    if (w > 0) {
      // U rows of the leaf, U = L11^-1 A[cl .. cl+IB, right of the leaf], by forward
      // substitution in FP64: one thread per column (w < 64, one wavefront), the column's IB
      // values in registers, the entries of the leaf's unit lower triangle read alike by all
      if (t < w) {
        double2 u[IB];
#pragma unroll
        for (int q = 0; q < IB; ++q) u[q] = ld2(A + (cl + q) * ld + cl + IB + t);
#pragma unroll
        for (int q = 1; q < IB; ++q)
#pragma unroll
          for (int pp = 0; pp < q; ++pp) u[q] = leaf_fms(u[q], s_L11[q][pp], u[pp]);
#pragma unroll
        for (int q = 0; q < IB; ++q) {
          st2(A + (cl + q) * ld + cl + IB + t, u[q]);
          s_U[q][t] = u[q];
        }
      }
      __syncthreads();
      // rank-IB update of the panel right of the leaf on the matrix cores: each wave updates
      // its own 64 rows of every PT-row slab, RBP 16-row blocks at a time.  The leaf's L rows
      // are read back from memory (stored before the barrier above), and all old values and
      // L operands of a group are loaded before its first product, so a group waits for
      // memory once instead of once per 16 x 16 tile.  The first IB columns right of the leaf
      // are the next leaf: their results go through the wave's own rows of s_X straight into
      // the leaf registers (the slab's old leaf values are dead by then), so the next leaf is
      // neither stored here nor loaded again; the other columns are written back.  Rows above
      // the leaf's last row and columns past w are masked at the load and store.
      constexpr int CBM = (NB - IB + 15) / 16;          // 16-column blocks, at most
      constexpr int VRB = CBM * 4 * (int)sizeof(T) / 4;  // registers per block's old values
      // with the next leaf kept on chip its registers stay live through the update, so the
      // groups are two blocks (one with four row slots or 256 threads)
      constexpr int RBP = KEEP_NEXT ? (S >= 4 || PT == 256 ? 1 : 2) : (VRB * 4 <= 96 ? 4 : (VRB * 2 <= 96 ? 2 : 1));
      // The 16-wide kept leaves take their L operand from LDS, which shortens their rank
      // updates; the leaves not kept on chip would pay for its registers in occupancy or
      // spills, and the 256-thread kernels ran their rank updates slower with it.
      constexpr bool LOP_LDS = KEEP_NEXT && IB == 16;
      typedef StripMma<T, 1, IB> Mma;
      const int ii = lane & 15, kq = lane >> 4;
#pragma unroll 1
      for (int s = 0; s < S; ++s) {
        const int r0 = k + s * PT;
        if constexpr (LOP_LDS) {
          // the slab's leaf rows, the L operand of its products, into the wave's rows of s_X
          // (read there instead of from memory; rows past the matrix hold zeros); a group's
          // rows take the next leaf only after the group's own products have read them
          wave_sync();
#pragma unroll
          for (int ss = 0; ss < S; ++ss)
            if (ss == s) {
#pragma unroll
              for (int q = 0; q < IB; ++q) s_X[t][q] = v[ss][q];
            }
          wave_sync();
        }
#pragma unroll 1
        for (int g = 0; g < 4; g += RBP) {
          const int gbase = r0 + wave * 64 + g * 16;
          if (gbase >= nrows || gbase + RBP * 16 <= cl + IB) continue;  // uniform per wave
          T lop[RBP][IB / 4];
          T old[RBP][CBM][4];
#pragma unroll
          for (int b = 0; b < RBP; ++b) {
            const int rl = gbase + b * 16 + ii;
            if constexpr (LOP_LDS) {
#pragma unroll
              for (int q = 0; q < IB / 4; ++q) lop[b][q] = s_X[wave * 64 + (g + b) * 16 + ii][4 * q + kq];
            } else {
#pragma unroll
              for (int q = 0; q < IB / 4; ++q) lop[b][q] = rl < nrows ? A[rl * ld + cl + 4 * q + kq] : T{0, 0};
            }
#pragma unroll
            for (int cb = 0; cb < CBM; ++cb)
#pragma unroll
              for (int r = 0; r < 4; ++r) {
                const int row = gbase + b * 16 + Mma::row(r, lane), cc = cb * 16 + ii;
                old[b][cb][r] = (row >= cl + IB && row < nrows && cc < w) ? A[row * ld + cl + IB + cc] : T{0, 0};
              }
          }
#pragma unroll
          for (int b = 0; b < RBP; ++b) {
            const int rbase = gbase + b * 16;
            if (rbase + 16 <= cl + IB || rbase >= nrows) continue;  // uniform per wave
#pragma unroll
            for (int cb = 0; cb < CBM; ++cb) {
              if (cb * 16 >= w) continue;  // uniform
              Mma acc;
              acc.zero();
              acc.run_regs(lop[b],
                           [&](int kk, int cc) {
                             T u;
                             narrow_to(u, s_U[kk][cb * 16 + cc]);
                             return u;
                           },
                           lane);
#pragma unroll
              for (int r = 0; r < 4; ++r) {
                const int row = rbase + Mma::row(r, lane), cc = cb * 16 + ii;
                if (row >= cl + IB && row < nrows && cc < w) {
                  T nv;
                  narrow_to(nv, csub(wide(old[b][cb][r]), acc.value(0, r)));
                  if (KEEP_NEXT && cc < IB)
                    s_X[row - r0][cc] = nv;
                  else
                    A[row * ld + cl + IB + cc] = nv;
                }
              }
            }
          }
        }
        if constexpr (KEEP_NEXT) {
          wave_sync();
          // the next leaf's rows of this slab (rows above it or past the matrix are zero);
          // register slots are indexed by constants only
          const int r = r0 + t;
          const bool in = r >= cl + IB && r < nrows;
#pragma unroll
          for (int ss = 0; ss < S; ++ss)
            if (ss == s) {
#pragma unroll
              for (int q = 0; q < IB; ++q) v[ss][q] = in ? s_X[t][q] : T{0, 0};
            }
          wave_sync();  // every lane has its row before the next slab writes s_X
        }
      }
    }
    // the next leaf reads columns written above by other threads, and s_U / s_L11 /
    // s_piv are rewritten by it
    __syncthreads();
  }
  // The panel's NB interchanges as one permutation of at most 2 NB rows.
  __syncthreads();
  if (wave == 0) write_perm_list(k, s_pivall, s_pos, s_org, ip + perm_off(nrows, k), lane);
  if (t == 0 && first_zero != 0) {
    if (info[blockIdx.x] == 0) info[blockIdx.x] = first_zero;
  }
}

// ------------------------------------------------------------------------------------
// inverses of the panel's diagonal triangles, in place
// ------------------------------------------------------------------------------------
// After panel(k) the diagonal block holds L11 (strictly lower, unit diagonal implied) and
// U11 (upper with diagonal).  One workgroup per job solves L11 X = I and U11 Y = I (four
// wavefronts of 16 columns each per triangle, FP64 shuffle substitution, tri.h) and overwrites the block with
// X = L11^-1 below the diagonal and Y = U11^-1 on and above it.  Every later use of the
// block wants an inverse: U12 = L11^-1 A12 in swap_trsm_kernel and the four diagonal steps
// of the solves, which thereby become products on the matrix cores.  No later interchange
// touches the block (pivots of later panels lie below it), and nothing else reads U11.
// This form serves FP64 storage; FP32 storage takes the blocked kernel below.
template <typename T>
__global__ __launch_bounds__(512) void linv_kernel(const JobDesc* jobs, int k, T* work) {
  const JobDesc jd = jobs[blockIdx.x];
  if (k >= jd.npad) return;  // uniform
  T* A = work + jd.a_off;
  const int64_t ld = jd.npad;
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  typedef typename LdsOf<T>::type S;
  // FP32 storage: both inverses at once (waves 0-3 L11, 4-7 U11, 100 KB of LDS); FP64
  // storage: one after the other in two arrays (133 KB), waves 4-7 idle
  constexpr bool BOTH = sizeof(S) == sizeof(float2);
  __shared__ S s_T[NB][NB + 1];
  __shared__ S s_X[NB][NB + 1];
  __shared__ S s_Y[BOTH ? NB : 1][NB + 1];
  for (int idx = t; idx < NB * NB; idx += 512) {
    const int q = idx / NB, pp = idx % NB;
    s_T[q][pp] = A[(k + q) * ld + k + pp];
    st2(&s_X[q][pp], make_double2(q == pp ? 1.0 : 0.0, 0.0));
    if (BOTH) st2(&s_Y[BOTH ? q : 0][pp], make_double2(q == pp ? 1.0 : 0.0, 0.0));
  }
  __syncthreads();
  // the substitutions read only the triangle they need (tri.h)
  if (wave < 4) tri_unit_lower<16>(&s_T[0][0], NB + 1, &s_X[0][0], NB + 1, wave * 16, lane);
  if (BOTH && wave >= 4) tri_upper<16>(&s_T[0][0], NB + 1, &s_Y[0][0], NB + 1, (wave - 4) * 16, lane);
  __syncthreads();
  if (BOTH) {
    for (int idx = t; idx < NB * NB; idx += 512) {
      const int q = idx / NB, pp = idx % NB;
      A[(k + q) * ld + k + pp] = pp < q ? s_X[q][pp] : s_Y[BOTH ? q : 0][pp];
    }
    return;
  }
  for (int idx = t; idx < NB * NB; idx += 512) {
    const int q = idx / NB, pp = idx % NB;
    if (pp < q) A[(k + q) * ld + k + pp] = s_X[q][pp];
    st2(&s_X[q][pp], make_double2(q == pp ? 1.0 : 0.0, 0.0));
  }
  __syncthreads();
  if (wave < 4) tri_upper<16>(&s_T[0][0], NB + 1, &s_X[0][0], NB + 1, wave * 16, lane);
  __syncthreads();
  for (int idx = t; idx < NB * NB; idx += 512) {
    const int q = idx / NB, pp = idx % NB;
    if (pp >= q) A[(k + q) * ld + k + pp] = s_X[q][pp];
  }
}

// FP32 storage: the same inverses blocked in 16 x 16 blocks (indices i, m in 0..3).  One
// wavefront per diagonal block forms X_ii = L_ii^-1 or Y_ii = U_ii^-1 (16-step FP64
// substitutions), then the off-diagonal blocks follow from FP64 matrix-core products:
//   X_ij = -sum_{j <= m < i} (X_ii L_im) X_mj,   Y_ij = -sum_{i < m <= j} (Y_ii U_im) Y_mj,
// first the six products W = X_ii L_im and the six Y_ii U_im, then the blocks one, two and
// three steps off the diagonal (waves 0-3 the lower triangle, 4-7 the upper one).  Results
// are kept in FP64 and rounded once to FP32 at the store.
__device__ inline void lower_pair(int task, int& i, int& m) {  // (1,0) (2,0) (2,1) (3,0) (3,1) (3,2)
  i = 1 + (task >= 1) + (task >= 3);
  m = task - i * (i - 1) / 2;
}
__global__ __launch_bounds__(512) void linv_blocked_kernel(const JobDesc* jobs, int k, float2* work) {
  constexpr int B = 16;
  const JobDesc jd = jobs[blockIdx.x];
  if (k >= jd.npad) return;  // uniform
  float2* A = work + jd.a_off;
  const int64_t ld = jd.npad;
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  __shared__ float2 s_T[NB][NB + 1];           // L11 \ U11 as factored
  __shared__ double2 s_V[NB][NB + 1];          // X = L11^-1 below the diagonal, Y = U11^-1 on and above
  __shared__ double2 s_W[2][6][B][B + 1];      // X_ii L_im (index i (i - 1) / 2 + m) and Y_mm U_mi
  for (int idx = t; idx < NB * NB; idx += 512) {
    const int q = idx / NB, pp = idx % NB;
    s_T[q][pp] = A[(k + q) * ld + k + pp];
  }
  __syncthreads();
  const int c = lane & 15, g = lane >> 4;  // a lane's column and row group (rows g + 4 j)
  const bool lower = wave < 4;
  // diagonal blocks
  {
    const int o = (wave & 3) * B;
    double2 x[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) x[j] = make_double2(g + 4 * j == c ? 1.0 : 0.0, 0.0);
    if (lower) {
#pragma unroll
      for (int q = 0; q < B; ++q) {  // x_q is final: broadcast it down its column
        const double2 xq = shfl2(x[q / 4], (q & 3) * 16 + c);
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int r = g + 4 * j;
          if (r > q) x[j] = cfms(x[j], ld2(&s_T[o + r][o + q]), xq);
        }
      }
#pragma unroll
      for (int j = 0; j < 4; ++j)
        if (g + 4 * j > c) s_V[o + g + 4 * j][o + c] = x[j];
    } else {
#pragma unroll
      for (int q = B - 1; q >= 0; --q) {  // y_q /= U_qq, then broadcast it up its column
        if (g == (q & 3)) x[q / 4] = cmul(x[q / 4], cinv(ld2(&s_T[o + q][o + q])));
        const double2 yq = shfl2(x[q / 4], (q & 3) * 16 + c);
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int r = g + 4 * j;
          if (r < q) x[j] = cfms(x[j], ld2(&s_T[o + r][o + q]), yq);
        }
      }
#pragma unroll
      for (int j = 0; j < 4; ++j)
        if (g + 4 * j <= c) s_V[o + g + 4 * j][o + c] = x[j];
    }
  }
  __syncthreads();
  typedef StripMma<double2, 1, B> Mma;
  // the inverted diagonal block d as an operand (unit diagonal of X implied, zeros outside)
  auto diag_at = [&](int d, int r, int cc) -> double2 {
    const int o = d * B;
    if (lower) return r > cc ? s_V[o + r][o + cc] : make_double2(r == cc ? 1.0 : 0.0, 0.0);
    return r <= cc ? s_V[o + r][o + cc] : make_double2(0.0, 0.0);
  };
  // W products: lower X_ii L_im (i > m), upper Y_mm U_mi (m < i), six each over four waves
  for (int task = wave & 3; task < 6; task += 4) {
    int i, m;
    lower_pair(task, i, m);
    Mma acc;
    acc.zero();
    if (lower)
      acc.run([&](int r, int kk) { return diag_at(i, r, kk); },
              [&](int kk, int cc) { return ld2(&s_T[i * B + kk][m * B + cc]); }, lane);
    else
      acc.run([&](int r, int kk) { return diag_at(m, r, kk); },
              [&](int kk, int cc) { return ld2(&s_T[m * B + kk][i * B + cc]); }, lane);
#pragma unroll
    for (int r = 0; r < 4; ++r) s_W[lower ? 0 : 1][task][Mma::row(r, lane)][c] = acc.value(0, r);
  }
  __syncthreads();
  // blocks dd steps off the diagonal: lower X_{i, i-dd}, upper Y_{i-dd, i}, i = dd .. 3
#pragma unroll 1
  for (int dd = 1; dd < 4; ++dd) {
    const int i = dd + (wave & 3);
    if (i < 4) {
      const int j = i - dd;
      Mma acc;
      acc.zero();
      for (int m = j; m < i; ++m) {  // lower: W_im X_mj; upper: (Y_jj U_jm... ) as W(j, m) Y_mi
        if (lower)
          acc.run([&](int r, int kk) { return s_W[0][i * (i - 1) / 2 + m][r][kk]; },
                  [&](int kk, int cc) { return m == j ? diag_at(j, kk, cc) : s_V[m * B + kk][j * B + cc]; }, lane);
        else {
          const int mm = m + 1;  // Y_{j, i} = -sum_{j < mm <= i} (Y_jj U_{j mm}) Y_{mm, i}
          acc.run([&](int r, int kk) { return s_W[1][mm * (mm - 1) / 2 + j][r][kk]; },
                  [&](int kk, int cc) { return mm == i ? diag_at(i, kk, cc) : s_V[mm * B + kk][i * B + cc]; }, lane);
        }
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const double2 v = acc.value(0, r);
        const int rr = Mma::row(r, lane);
        if (lower)
          s_V[i * B + rr][j * B + c] = make_double2(-v.x, -v.y);
        else
          s_V[j * B + rr][i * B + c] = make_double2(-v.x, -v.y);
      }
    }
    __syncthreads();
  }
  for (int idx = t; idx < NB * NB; idx += 512) {
    const int q = idx / NB, pp = idx % NB;
    st2(A + (k + q) * ld + k + pp, s_V[q][pp]);
  }
}

template <typename T>
static void launch_linv(const JobDesc* jobs, int njobs, int k, T* work, hipStream_t s) {
  if constexpr (sizeof(T) == sizeof(float2))
    linv_blocked_kernel<<<njobs, 512, 0, s>>>(jobs, k, work);
  else
    linv_kernel<T><<<njobs, 512, 0, s>>>(jobs, k, work);
}

// ------------------------------------------------------------------------------------
// interchanges + U12 = L11^-1 A12 on one 64-column tile of the trailing matrix
// ------------------------------------------------------------------------------------
// The tile's panel rows are gathered through LDS with the panel's permutation (the other
// permuted rows are written back directly), then U12 = L11^-1 A12 is one 64 x 64 x 64
// product on the matrix cores with the inverse stored by the inverse kernel (FP32 three-product
// MFMA for FP32 storage, FP64 MFMA otherwise).
// SECOND: k is panel nprev >= 1 of a group whose first panel starts at k - nprev NB.  Its
// trailing columns have not yet received the updates of the group's earlier panels, so
// after the gather the panel rows get  A12 -= L[k.., k - nprev NB .. k) U12_earlier  (the
// same 64 x 64 products, one per earlier panel, in panel order) before U12.
template <typename T, bool SECOND>
__global__ __launch_bounds__(256, sizeof(T) == sizeof(float2) ? 4 : 2) void swap_trsm_kernel(const JobDesc* jobs, int k, int nprev, T* work,
                                                        const int32_t* piv) {
  const JobDesc jd = jobs[blockIdx.y];
  const int col0 = k + NB + blockIdx.x * 64;
  if (k >= jd.npad || col0 >= jd.npad) return;  // uniform
  T* A = work + jd.a_off;
  const int64_t ld = jd.npad;
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  typedef typename LdsOf<T>::type S;
  // Only the gathered tile lives in LDS; the 64 x 64 left operands (the inverse of the
  // panel's unit lower triangle, and for SECOND the first panel's facing L rows) are the
  // same for every tile of a job and are read through the cache by the MFMA operand loads.
  __shared__ S s_X[NB][64 + 4];
  __shared__ int s_dst[PERM_MAX], s_src[PERM_MAX];
  const int32_t* lst = piv + jd.piv_off + perm_off(jd.npad, k);
  const int cnt = lst[0];
  for (int i = t; i < cnt; i += 256) {
    s_dst[i] = lst[2 + i];
    s_src[i] = lst[2 + PERM_MAX + i];
  }
  __syncthreads();
  // the panel's permutation as a gather on this tile: entry i = wave + 4 s, column = lane
  T held[PERM_MAX / 4];
#pragma unroll
  for (int u = 0; u < PERM_MAX / 4; ++u) {
    const int i = wave + 4 * u;
    if (i < cnt) {
      const int dst = s_dst[i];
      const T v = A[s_src[i] * ld + col0 + lane];
      if (dst < k + NB)
        s_X[dst - k][lane] = v;
      else
        held[u] = v;
    }
  }
  __syncthreads();  // every source row is read before any destination row is written
#pragma unroll
  for (int u = 0; u < PERM_MAX / 4; ++u) {
    const int i = wave + 4 * u;
    if (i < cnt) {
      const int dst = s_dst[i];
      if (dst >= k + NB) A[dst * ld + col0 + lane] = held[u];
    }
  }
  const int ii = lane & 15;
  const int row0 = k + wave * 16;  // this wavefront's 16 panel rows
  if (SECOND) {
    // s_X -= L[k.., kl..k) U[kl.., col0..], kl = k - nprev NB: wave w owns rows 16w .. 16w+16.
    StripMma<T, 4, sizeof(T) == sizeof(float2) ? NB / 2 : NB> d;
    d.zero();
    if constexpr (sizeof(T) == sizeof(float2)) {
      // FP32 storage: the wave's gathered rows move to registers (accumulator layout), so that
      // s_X can stage each earlier panel's 64 x 64 block of U rows, loaded once per workgroup
      // 16 bytes of a row per access instead of once per wave through the cache
      S xs[4][4];
#pragma unroll
      for (int cb = 0; cb < 4; ++cb)
#pragma unroll
        for (int r = 0; r < 4; ++r) xs[cb][r] = s_X[wave * 16 + d.row(r, lane)][cb * 16 + ii];
      constexpr int P4 = 64 * (int)sizeof(T) / 16;  // 16-byte pieces per row of the block
#pragma unroll 1
      for (int q = 0; q < nprev; ++q) {
        const int kq = k - (nprev - q) * NB;  // the earlier panel's first column
        __syncthreads();                      // s_X is free (copied out, or the last products done)
        for (int idx = t; idx < NB * P4; idx += 256) {
          const int row = idx / P4, p4 = idx - row * P4;
          ((float4*)&s_X[row][0])[p4] = ((const float4*)(A + (int64_t)(kq + row) * ld + col0))[p4];
        }
        // the left operand in two halves of K (the same products in the same order), so that
        // its registers fit beside the held rows and the accumulators
        T la[NB / 8];
#pragma unroll
        for (int s4 = 0; s4 < NB / 8; ++s4) la[s4] = A[(int64_t)(row0 + ii) * ld + kq + 4 * s4 + (lane >> 4)];
        __syncthreads();
        d.run_regs(la, [&](int kk, int c) { return s_X[kk][c]; }, lane);
#pragma unroll
        for (int s4 = 0; s4 < NB / 8; ++s4)
          la[s4] = A[(int64_t)(row0 + ii) * ld + kq + NB / 2 + 4 * s4 + (lane >> 4)];
        d.run_regs(la, [&](int kk, int c) { return s_X[NB / 2 + kk][c]; }, lane);
      }
      __syncthreads();  // every wave's products read s_X before it takes the updated rows
#pragma unroll
      for (int cb = 0; cb < 4; ++cb)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          S* xp = &s_X[wave * 16 + d.row(r, lane)][cb * 16 + ii];
          st2(xp, csub(wide(xs[cb][r]), d.value(cb, r)));
        }
    } else {
      // FP64 storage (half the occupancy already): operands through the cache
#pragma unroll 1
      for (int q = 0; q < nprev; ++q) {
        const int kq = k - (nprev - q) * NB;
        T la[NB / 4];
#pragma unroll
        for (int s4 = 0; s4 < NB / 4; ++s4) la[s4] = A[(int64_t)(row0 + ii) * ld + kq + 4 * s4 + (lane >> 4)];
        d.run_regs(la, [&](int kk, int c) { return A[(int64_t)(kq + kk) * ld + col0 + c]; }, lane);
      }
#pragma unroll
      for (int cb = 0; cb < 4; ++cb)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          S* xp = &s_X[wave * 16 + d.row(r, lane)][cb * 16 + ii];
          st2(xp, csub(ld2(xp), d.value(cb, r)));
        }
    }
  }
  // U12 = L11^-1 A12 straight from the accumulators to the panel rows (the inverse is
  // stored below the diagonal; its unit diagonal and zero upper part are implied).  The
  // lane's sixteen inverse entries are loaded before the barrier, in one batch.
  T li[NB / 4];
  {
    const int q = wave * 16 + ii;
#pragma unroll
    for (int s4 = 0; s4 < NB / 4; ++s4) {
      const int kk = 4 * s4 + (lane >> 4);
      li[s4] = kk < q ? A[(int64_t)(k + q) * ld + k + kk] : T{kk == q ? 1.0f : 0.0f, 0.0f};
    }
  }
  __syncthreads();
  StripMma<T, 4> u;
  u.zero();
  u.run_regs(li, [&](int kk, int c) { return s_X[kk][c]; }, lane);
#pragma unroll
  for (int cb = 0; cb < 4; ++cb)
#pragma unroll
    for (int r = 0; r < 4; ++r)
      st2(A + (int64_t)(row0 + u.row(r, lane)) * ld + col0 + cb * 16 + ii, u.value(cb, r));
}

// ------------------------------------------------------------------------------------
// tall panels: tournament pivoting
// ------------------------------------------------------------------------------------
// A panel of R rows keeps R / PT rows per thread in registers, which bounds the
// one-workgroup panel kernel to 4096 rows.  Taller panels (LIZ of several hundred to
// ~1000 sites) choose their NB pivot rows by a tournament over many workgroups instead
// (communication-avoiding LU, Grigori, Demmel and Xiang 2011):
//   1. the panel is cut into chunks of C rows, copied to scratch, and every chunk is
//      factored with partial pivoting by the panel kernel (one workgroup each); the NB
//      rows its pivots bring to the top are the chunk's candidates;
//   2. the original values of all candidates are gathered into one block and factored
//      with partial pivoting once more; the NB rows chosen there, in that order, are the
//      panel's pivot rows, and that block's top NB x NB factors are the panel's L11, U11;
//   3. the interchanges that bring those rows to the top (same permutation-list format
//      as the panel kernel's) are applied to the panel (and the `left` columns), L11\U11
//      is written over the diagonal block, and after the inverses the rows below are
//      L21 = A21 U11^-1, one 64 x 64 x 64 product per 16-row strip on the matrix cores.
// Every step is an ordinary launch over the batch: no workgroup waits for another.

struct TallLayout {
  int nc_max;
  int64_t w1, w2, p1, p2, g2, sub1, sub2, si1, si2, total;  // byte offsets
};

static TallLayout tall_layout(int njobs, int npad_max, int chunk) {
  TallLayout L{};
  L.nc_max = (npad_max + chunk - 1) / chunk;
  auto al = [](int64_t b) { return (b + 255) / 256 * 256; };
  int64_t off = 0;
  L.w1 = off;  // [job][npad_max][NB] elements of at most 16 bytes
  off += al((int64_t)njobs * npad_max * NB * 16);
  L.w2 = off;  // [job][nc_max * NB][NB]
  off += al((int64_t)njobs * L.nc_max * NB * NB * 16);
  L.p1 = off;  // [job][nc_max][piv_ints(chunk)]
  off += al((int64_t)njobs * L.nc_max * piv_ints(chunk) * 4);
  L.p2 = off;  // [job][piv_ints(nc_max * NB)]
  off += al((int64_t)njobs * piv_ints(L.nc_max * NB) * 4);
  L.g2 = off;  // [job][nc_max * NB] global row of each candidate
  off += al((int64_t)njobs * L.nc_max * NB * 4);
  L.sub1 = off;
  off += al((int64_t)njobs * L.nc_max * sizeof(JobDesc));
  L.sub2 = off;
  off += al((int64_t)njobs * sizeof(JobDesc));
  L.si1 = off;
  off += al((int64_t)njobs * L.nc_max * 4);
  L.si2 = off;
  off += al((int64_t)njobs * 4);
  L.total = off;
  return L;
}

size_t tall_scratch_bytes(int njobs, int npad_max, int chunk) {
  if (chunk <= 0 || npad_max <= 2 * chunk) return 0;
  return (size_t)tall_layout(njobs, npad_max, chunk).total;
}

// Sub-problem descriptors for this panel: chunk c of job j is rows [c C, ...) of the
// job's panel copy (leading dimension NB); chunks past a job's rows are empty (npad 0).
__global__ void tslu_setup_kernel(const JobDesc* jobs, int njobs, int k, int chunk, int nc_max, int npad_max,
                                  JobDesc* sub1, JobDesc* sub2, int32_t* si1, int32_t* si2) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= njobs * nc_max) return;
  const int j = idx / nc_max, c = idx - j * nc_max;
  const int rows = jobs[j].npad - k;
  const int nc = rows > 0 ? (rows + chunk - 1) / chunk : 0;
  JobDesc d{};
  if (c < nc) {
    const int r = min(chunk, rows - c * chunk);  // a multiple of NB, at least NB
    d.a_off = ((int64_t)j * npad_max + (int64_t)c * chunk) * NB;
    d.piv_off = ((int64_t)j * nc_max + c) * piv_ints(chunk);
    d.n = r;
    d.npad = r;
    d.ld = NB;
  }
  sub1[idx] = d;
  si1[idx] = 0;
  if (c == 0) {
    JobDesc e{};
    if (nc > 0) {
      e.a_off = (int64_t)j * nc_max * NB * NB;
      e.piv_off = (int64_t)j * piv_ints(nc_max * NB);
      e.n = nc * NB;
      e.npad = nc * NB;
      e.ld = NB;
    }
    sub2[j] = e;
    si2[j] = 0;
  }
}

// rows [k, npad) x cols [k, k + NB) of each job into its panel copy
template <typename T>
__global__ void tslu_copy_kernel(const JobDesc* jobs, int k, int npad_max, const T* work, T* w1) {
  const JobDesc jd = jobs[blockIdx.y];
  const int rows = jd.npad - k;
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (rows <= 0 || idx >= (int64_t)rows * NB) return;
  const int r = (int)(idx / NB), q = (int)(idx - (int64_t)r * NB);
  w1[((int64_t)blockIdx.y * npad_max + r) * NB + q] = work[jd.a_off + (int64_t)(k + r) * jd.npad + k + q];
}

// Candidates of chunk (blockIdx.x) of job (blockIdx.y): the original rows that the chunk's
// interchanges moved to its first NB positions, gathered from the (unmodified) panel.
template <typename T>
__global__ __launch_bounds__(256) void tslu_gather_kernel(const JobDesc* jobs, int k, int chunk, int nc_max,
                                                          const JobDesc* sub1, const int32_t* p1, const T* work,
                                                          T* w2, int32_t* g2) {
  const int j = blockIdx.y, c = blockIdx.x;
  const JobDesc sd = sub1[j * nc_max + c];
  if (sd.npad == 0) return;
  const JobDesc jd = jobs[j];
  const int32_t* lst = p1 + sd.piv_off + perm_off(sd.npad, 0);
  const int64_t base = (int64_t)j * nc_max * NB + (int64_t)c * NB;
  for (int idx = threadIdx.x; idx < NB * NB; idx += 256) {
    const int e = idx / NB, q = idx - e * NB;
    const int gid = k + c * chunk + lst[2 + PERM_MAX + e];
    w2[(base + e) * NB + q] = work[jd.a_off + (int64_t)gid * jd.npad + k + q];
    if (q == 0) g2[base + e] = gid;
  }
}

// Position (index into pos/row lists of cnt <= PERM_MAX entries) of value v, or -1.
__device__ inline int find_entry(const int* arr, int cnt, int v, int lane) {
  const unsigned long long m0 = __ballot(lane < cnt && arr[lane] == v);
  if (m0) return __ffsll((long long)m0) - 1;
  const unsigned long long m1 = __ballot(lane + 64 < cnt && arr[lane + 64] == v);
  return m1 ? 64 + __ffsll((long long)m1) - 1 : -1;
}

// The tournament's winners become the panel's pivot rows: interchanges, permutation list,
// L11\U11 from the final factorization, zero-pivot report.  One workgroup per job.
template <typename T>
__global__ __launch_bounds__(256) void tslu_apply_kernel(const JobDesc* jobs, int k, int left, int nc_max,
                                                         const JobDesc* sub2, const int32_t* p2, const T* w2,
                                                         const int32_t* g2, const int32_t* si2, T* work,
                                                         int32_t* piv, int32_t* info) {
  const int j = blockIdx.x;
  const JobDesc jd = jobs[j];
  if (k >= jd.npad) return;  // uniform
  const JobDesc rd = sub2[j];
  T* A = work + jd.a_off;
  const int64_t ld = jd.npad;
  int32_t* ip = piv + jd.piv_off;
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  __shared__ int s_sel[NB], s_pivall[NB];
  __shared__ int s_mpos[PERM_MAX], s_mrow[PERM_MAX];
  __shared__ int s_pos[PERM_MAX], s_org[PERM_MAX], s_cnt;
  __shared__ T s_held[PERM_MAX][33];
  const int32_t* lst2 = p2 + rd.piv_off + perm_off(rd.npad, 0);
  if (t < NB) s_sel[t] = g2[(int64_t)j * nc_max * NB + lst2[2 + PERM_MAX + t]];
  __syncthreads();
  if (wave == 0) {
    // Interchanges that bring s_sel[q] to position k + q for q = 0, 1, ... in turn, as
    // partial pivoting records them: (s_mpos[e], s_mrow[e]) lists the positions whose row
    // has changed and the row each now holds (at most 2 NB entries).
    int cnt = 0;
    for (int q = 0; q < NB; ++q) {
      const int row = s_sel[q], d = k + q;
      const int er = find_entry(s_mrow, cnt, row, lane);
      const int p = er >= 0 ? s_mpos[er] : row;  // where that row is now
      if (lane == 0) s_pivall[q] = p;
      if (p != d) {
        const int ed = find_entry(s_mpos, cnt, d, lane);
        const int at_d = ed >= 0 ? s_mrow[ed] : d;
        if (lane == 0) {
          if (ed >= 0) {
            s_mrow[ed] = row;
          } else {
            s_mpos[cnt] = d;
            s_mrow[cnt] = row;
          }
          const int e2 = ed >= 0 ? cnt : cnt + 1;
          if (er >= 0) {
            s_mrow[er] = at_d;
          } else {
            s_mpos[e2] = p;
            s_mrow[e2] = at_d;
          }
        }
        cnt += (ed >= 0 ? 0 : 1) + (er >= 0 ? 0 : 1);
      }
    }
    for (int q = lane; q < NB; q += 64) ip[k + q] = s_pivall[q];
    const int c = write_perm_list(k, s_pivall, s_pos, s_org, ip + perm_off(jd.npad, k), lane);
    if (lane == 0) s_cnt = c;  // (pos, org) stay in LDS for the other wavefronts
  }
  __syncthreads();
  // the permutation on the panel's columns and the `left` columns before them
  const int cnt = s_cnt;
  const int ncols = left + NB;
  for (int c0 = 0; c0 < ncols; c0 += 32) {
    for (int idx = t; idx < cnt * 32; idx += 256) {
      const int e = idx >> 5, cc = idx & 31;
      if (c0 + cc < ncols) s_held[e][cc] = A[(int64_t)s_org[e] * ld + (k - left) + c0 + cc];
    }
    __syncthreads();
    for (int idx = t; idx < cnt * 32; idx += 256) {
      const int e = idx >> 5, cc = idx & 31;
      if (c0 + cc < ncols) A[(int64_t)s_pos[e] * ld + (k - left) + c0 + cc] = s_held[e][cc];
    }
    __syncthreads();
  }
  // L11\U11 of the chosen rows, as the final factorization left them
  const T* top = w2 + (int64_t)j * nc_max * NB * NB;
  for (int idx = t; idx < NB * NB; idx += 256) {
    const int q = idx / NB, pp = idx - q * NB;
    A[(int64_t)(k + q) * ld + k + pp] = top[(int64_t)q * NB + pp];
  }
  if (t == 0 && si2[j] != 0 && info[j] == 0) info[j] = k + si2[j];
}

// L21 = A21 U11^-1 below the diagonal block (U11^-1 on and above the block's diagonal,
// written by the inverse kernel): wave w of workgroup (x, job) takes rows k + NB + 64 x + 16 w.
template <typename T>
__global__ __launch_bounds__(256) void tslu_l21_kernel(const JobDesc* jobs, int k, T* work) {
  const JobDesc jd = jobs[blockIdx.y];
  const int lane = threadIdx.x & 63, ii = lane & 15;
  const int r0 = k + NB + blockIdx.x * 64 + (threadIdx.x >> 6) * 16;
  if (k >= jd.npad || r0 >= jd.npad) return;  // uniform per wavefront; no barrier below
  T* A = work + jd.a_off;
  const int64_t ld = jd.npad;
  StripMma<T, 4> d;
  d.zero();
  d.run([&](int i, int kk) { return A[(int64_t)(r0 + i) * ld + k + kk]; },
        [&](int kk, int c) {
          T u = A[(int64_t)(k + kk) * ld + k + c];
          if (kk > c) u = T{0, 0};
          return u;
        },
        lane);
#pragma unroll
  for (int cb = 0; cb < 4; ++cb)
#pragma unroll
    for (int r = 0; r < 4; ++r) st2(A + (int64_t)(r0 + d.row(r, lane)) * ld + k + cb * 16 + ii, d.value(cb, r));
}

// ------------------------------------------------------------------------------------
// drivers
// ------------------------------------------------------------------------------------
// Leaf width: FP32 storage keeps the leaf in FP32 registers, so 16 columns fit where FP64
// storage holds 8; wider leaves halve the passes over the rest of the panel (the
// panel's memory traffic).  Past 2560 rows the leaf is halved to stay in registers.
template <typename T>
static void launch_panel(const JobDesc* jobs, int njobs, int k, int left, int rows, T* work, int32_t* piv,
                         int32_t* info, hipStream_t s, int nopiv = 0, int small_rows = PANEL_SMALL_ROWS) {
  constexpr int PT = 512;
  constexpr int IBW = sizeof(T) == sizeof(float2) ? 16 : 8;
  if constexpr (sizeof(T) == sizeof(float2)) {
    if (rows <= std::min(small_rows, PANEL_SMALL_MAX)) {
      // FP32 storage up to small_rows (at most PANEL_SMALL_MAX = 768) rows: 256-thread
      // workgroups with 8-wide leaves fit three jobs per CU, which hides more of the short
      // panels' barrier and shuffle latency behind another job's work (where the wider leaves
      // of the 512-thread kernel, one job per CU, win instead is found by the autotuner; up
      // to 2304 rows the small form was measured 1.1-1.6x slower than the large one from
      // 1024 rows on, as more row slots per thread drop it to two and one job per CU)
      const int S2 = (rows + 255) / 256;
      switch (S2) {
        case 1: panel_kernel<T, 256, 1, 8><<<njobs, 256, 0, s>>>(jobs, k, left, work, piv, info, nopiv); return;
        case 2: panel_kernel<T, 256, 2, 8><<<njobs, 256, 0, s>>>(jobs, k, left, work, piv, info, nopiv); return;
        default: panel_kernel<T, 256, 3, 8><<<njobs, 256, 0, s>>>(jobs, k, left, work, piv, info, nopiv); return;
      }
    }
  }
  const int S = (rows + PT - 1) / PT;
  switch (S) {
    case 1: panel_kernel<T, PT, 1, IBW><<<njobs, PT, 0, s>>>(jobs, k, left, work, piv, info, nopiv); break;
    case 2: panel_kernel<T, PT, 2, IBW><<<njobs, PT, 0, s>>>(jobs, k, left, work, piv, info, nopiv); break;
    case 3: panel_kernel<T, PT, 3, IBW><<<njobs, PT, 0, s>>>(jobs, k, left, work, piv, info, nopiv); break;
    case 4: panel_kernel<T, PT, 4, IBW><<<njobs, PT, 0, s>>>(jobs, k, left, work, piv, info, nopiv); break;
    case 5: panel_kernel<T, PT, 5, IBW><<<njobs, PT, 0, s>>>(jobs, k, left, work, piv, info, nopiv); break;
    case 6: panel_kernel<T, PT, 6, IBW / 2><<<njobs, PT, 0, s>>>(jobs, k, left, work, piv, info, nopiv); break;
    case 7: panel_kernel<T, PT, 7, IBW / 2><<<njobs, PT, 0, s>>>(jobs, k, left, work, piv, info, nopiv); break;
    default: panel_kernel<T, PT, 8, IBW / 2><<<njobs, PT, 0, s>>>(jobs, k, left, work, piv, info, nopiv); break;
  }
}

// The split-mode panel at k = 0 of systems of `rows` rows, for the autotuner: variant 0 the
// 256-thread workgroups with 8-wide leaves (rows <= PANEL_SMALL_MAX), 1 the 512-thread ones.
void launch_panel_f32_variant(int variant, const JobDesc* jobs, int njobs, int rows, float2* work, int32_t* piv,
                              int32_t* info, hipStream_t s) {
  launch_panel<float2>(jobs, njobs, 0, 0, rows, work, piv, info, s, 0, variant == 0 ? PANEL_SMALL_MAX : 0);
}

// One panel (and the inverses of its diagonal triangles): the register-resident panel
// kernel, or the tournament for panels taller than 2 chunk rows.
template <typename T>
static void panel_step(const JobDesc* jobs, int njobs, int npad_max, int k, int left, T* work, int32_t* piv,
                       int32_t* info, const TallScratch& ts, hipStream_t s, int small_rows) {
  const int rows = npad_max - k;
  if (ts.chunk > 0 && rows > 2 * ts.chunk && ts.base) {
    const TallLayout L = tall_layout(ts.njobs, ts.npad_max, ts.chunk);
    char* b = (char*)ts.base;
    T* w1 = (T*)(b + L.w1);
    T* w2 = (T*)(b + L.w2);
    int32_t* p1 = (int32_t*)(b + L.p1);
    int32_t* p2 = (int32_t*)(b + L.p2);
    int32_t* g2 = (int32_t*)(b + L.g2);
    JobDesc* sub1 = (JobDesc*)(b + L.sub1);
    JobDesc* sub2 = (JobDesc*)(b + L.sub2);
    int32_t* si1 = (int32_t*)(b + L.si1);
    int32_t* si2 = (int32_t*)(b + L.si2);
    const int nc_max = L.nc_max;
    tslu_setup_kernel<<<(njobs * nc_max + 255) / 256, 256, 0, s>>>(jobs, njobs, k, ts.chunk, nc_max, ts.npad_max,
                                                                 sub1, sub2, si1, si2);
    tslu_copy_kernel<T><<<dim3((unsigned)(((int64_t)rows * NB + 255) / 256), njobs), 256, 0, s>>>(
        jobs, k, ts.npad_max, work, w1);
    launch_panel<T>(sub1, njobs * nc_max, 0, 0, ts.chunk, w1, p1, si1, s);
    tslu_gather_kernel<T><<<dim3(nc_max, njobs), 256, 0, s>>>(jobs, k, ts.chunk, nc_max, sub1, p1, work, w2, g2);
    launch_panel<T>(sub2, njobs, 0, 0, ((rows + ts.chunk - 1) / ts.chunk) * NB, w2, p2, si2, s);
    tslu_apply_kernel<T><<<njobs, 256, 0, s>>>(jobs, k, left, nc_max, sub2, p2, w2, g2, si2, work, piv, info);
    launch_linv<T>(jobs, njobs, k, work, s);
    if (rows > NB) tslu_l21_kernel<T><<<dim3((rows - NB + 63) / 64, njobs), 256, 0, s>>>(jobs, k, work);
    return;
  }
  launch_panel<T>(jobs, njobs, k, left, rows, work, piv, info, s, 0, small_rows);
  launch_linv<T>(jobs, njobs, k, work, s);
}

// Algorithmic flops and bytes of one trailing-update launch over the unpadded rows m and
// columns c of each job's updated block: 8 m c kd flops (complex multiply-add count) and
// es (m kd + kd c + 2 m c) bytes (L21 and U12 read once, A22 read and written once).
static void update_cost(const GemmProfiler* prof, int njobs, int kd, int r_begin, int c_begin, int c_end, int es,
                        double* flops, double* bytes) {
  double f = 0.0, b = 0.0;
  for (int j = 0; j < njobs; ++j) {
    const int n = prof->n_true[j];
    const double m = (double)(n - r_begin);
    const double c = (double)((c_end > 0 ? std::min(c_end, n) : n) - c_begin);
    if (m > 0 && c > 0) {
      f += 8.0 * m * c * kd;
      b += (double)es * (m * kd + kd * c + 2.0 * m * c);
    }
  }
  *flops = f;
  *bytes = b;
}

// Blocked LU over groups of G panels (G = group, 2 .. GROUP_MAX): groups start at every
// multiple of G NB, and the big trailing update runs once per group with K = G NB, so the
// trailing matrix is streamed once per G NB columns.  Within a group the panels are
// left-looking: for panel j of the group (first column kj = k + j NB)
//   update of panel j's columns by the group's earlier panels (K = j NB, rows from kj) ->
//   panel(kj), whose interchanges also permute the earlier panels' L columns (j NB of them)
//   -> interchanges + delayed update by the earlier panels + U12 on every column past the
//   panel (swap_trsm_kernel).
// Then one trailing update A22 -= L21 U12 with K = G NB over the rows and columns past the
// group.  Every element thus receives the same updates as in the right-looking order, in
// a different association.  The solves apply each panel's permutation right after the
// earlier panels of its group (see solve.hip).
// With a side stream, the trailing update is split at the next group's first panel: its
// NB columns are updated first, then that panel (and its inverses) is factored on the
// side stream while the rest of the update runs on the main one.  The two touch disjoint
// data (the panel reads and writes only its own columns and the diagonal block; the
// update reads the L and U12 rows of this group and writes columns past the panel), and
// the next group's interchanges wait for both.
template <typename T, typename Gemm>
static void lu_factor_any(const JobDesc* jobs, int njobs, int npad_max, T* work, int32_t* piv, int32_t* info,
                          hipStream_t s, GemmProfiler* prof, const TallScratch& tall, const SideStream* side,
                          int small_rows, int group, Gemm gemm) {
  auto timed_gemm = [&](int k, int kd, int r_begin, int c_begin, int c_end) {
    const int rows = npad_max - r_begin;
    const int cols = (c_end > 0 ? std::min(c_end, npad_max) : npad_max) - c_begin;
    if (rows <= 0 || cols <= 0) return;
    if (prof) prof->before(s);
    gemm(rows, cols, k, kd, r_begin, c_begin, c_end);
    if (prof) {
      double f, b;
      update_cost(prof, njobs, kd, r_begin, c_begin, c_end, (int)sizeof(T), &f, &b);
      prof->after(s, f, b, c_end > 0 ? 0 : 1);
    }
  };
  const int GW = group * NB;
  bool ahead = false;  // this group's first panel was factored on the side stream
  for (int k = 0; k < npad_max; k += GW) {
    for (int j = 0; j < group; ++j) {
      const int kj = k + j * NB;
      if (j > 0) timed_gemm(k, j * NB, kj, kj, kj + NB);  // panel j's columns, K = j NB
      if (j == 0 && ahead)
        (void)hipStreamWaitEvent(s, side->panel_done, 0);
      else
        panel_step<T>(jobs, njobs, npad_max, kj, j * NB, work, piv, info, tall, s, small_rows);
      const int rest = npad_max - kj - NB;
      if (rest <= 0) return;
      if (j == 0)
        swap_trsm_kernel<T, false><<<dim3(rest / 64, njobs), 256, 0, s>>>(jobs, kj, 0, work, piv);
      else
        swap_trsm_kernel<T, true><<<dim3(rest / 64, njobs), 256, 0, s>>>(jobs, kj, j, work, piv);
    }
    ahead = false;
    const int rest = npad_max - k - GW;  // > 0: the group's last panel had columns past it
    if (side && rest > NB) {
      timed_gemm(k, GW, k + GW, k + GW, k + GW + NB);  // the next first panel's columns
      (void)hipEventRecord(side->update_done, s);
      (void)hipStreamWaitEvent(side->stream, side->update_done, 0);
      panel_step<T>(jobs, njobs, npad_max, k + GW, 0, work, piv, info, tall, side->stream, small_rows);
      (void)hipEventRecord(side->panel_done, side->stream);
      ahead = true;
      timed_gemm(k, GW, k + GW, k + GW + NB, 0);
    } else {
      timed_gemm(k, GW, k + GW, k + GW, 0);
    }
  }
}

// ------------------------------------------------------------------------------------
// symmetric factorization (complex-symmetric S, no pivoting)
// ------------------------------------------------------------------------------------
// For S = S^T the unpivoted LU has U = D L^T (D = diag U).  So after each panel the U12 rows
// are the transpose of the panel's L21 scaled by D (no triangular solve, no interchanges),
// the trailing matrix is kept only on and below the diagonal, and every trailing update is
// the lower-triangle half of A22 -= L21 U12: (4/3) n^3 instead of (8/3) n^3.  The factors
// are stored exactly as the LU's (L below, U above the diagonal, identity permutations), so
// the LU solves and the diagonal-block inverses apply unchanged.

// U[k + q][c] = D[q] L[c][k + q] for c in [k + NB, npad): one 64-column tile per workgroup,
// transposed through LDS.  Runs before the inverse kernel (D is read off the diagonal block).
// from_inverse: the diagonal block already holds the inverses (tall panels), D = 1 / diag.
template <typename T>
__global__ __launch_bounds__(256) void sym_u12_kernel(const JobDesc* jobs, int k, T* work, int from_inverse) {
  const JobDesc jd = jobs[blockIdx.y];
  const int c0 = k + NB + blockIdx.x * 64;
  if (k >= jd.npad || c0 >= jd.npad) return;  // uniform
  T* A = work + jd.a_off;
  const int64_t ld = jd.npad;
  __shared__ T s_t[64][NB + 1];
  __shared__ T s_d[NB];
  const int t = threadIdx.x;
  if (t < NB) {
    const T dd = A[(int64_t)(k + t) * ld + k + t];
    if (from_inverse)
      narrow_to(s_d[t], cinv(wide(dd)));
    else
      s_d[t] = dd;
  }
  for (int idx = t; idx < 64 * NB; idx += 256) {
    const int i = idx / NB, q = idx - i * NB;
    s_t[i][q] = A[(int64_t)(c0 + i) * ld + k + q];
  }
  __syncthreads();
  for (int idx = t; idx < NB * 64; idx += 256) {
    const int q = idx >> 6, i = idx & 63;
    A[(int64_t)(k + q) * ld + c0 + i] = cmul(s_d[q], s_t[i][q]);
  }
}

// Panels of the symmetric factorization: without pivoting a panel is its diagonal block
// (factored in place by the panel kernel as a 64-row sub-problem with the job's leading
// dimension) and L21 = A21 U11^-1 below it (tslu_l21_kernel), so no pass over the panel's
// whole height is needed; panels of at most tall_rows rows may instead use the panel kernel.  Sub-problem j of a
// step covers job j's block at (k, k); its pivots and list go to scratch, and the job's own
// list for the panel is the identity.
__global__ void sym_tall_setup_kernel(const JobDesc* jobs, int njobs, int k, JobDesc* sub, int32_t* sinfo,
                                      int32_t* piv) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= njobs) return;
  const JobDesc jd = jobs[j];
  JobDesc d{};
  if (k < jd.npad) {
    d.a_off = jd.a_off + (int64_t)k * jd.npad + k;
    d.ld = jd.npad;
    d.n = NB;
    d.npad = NB;
    d.piv_off = (int64_t)j * piv_ints(NB);
    // the job's permutation list for this panel: the identity
    int32_t* ip = piv + jd.piv_off;
    int32_t* lst = ip + perm_off(jd.npad, k);
    lst[0] = NB;
    for (int i = 0; i < NB; ++i) {
      ip[k + i] = k + i;
      lst[2 + i] = k + i;
      lst[2 + PERM_MAX + i] = k + i;
    }
  }
  sub[j] = d;
  sinfo[j] = 0;
}

__global__ void sym_tall_info_kernel(int njobs, int k, const int32_t* sinfo, int32_t* info) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j < njobs && sinfo[j] != 0 && info[j] == 0) info[j] = k + sinfo[j];
}

size_t ldlt_scratch_bytes(int njobs) {
  return (size_t)njobs * (sizeof(JobDesc) + 4 * (size_t)piv_ints(NB) + 4) + 3 * 256;
}

void ldlt_factor_f32(const JobDesc* jobs, int njobs, int npad_max, float2* work, int32_t* piv, int32_t* info,
                     hipStream_t s, GemmProfiler* prof, int gemm_variant, int tall_rows, void* scratch) {
  JobDesc* sub = (JobDesc*)scratch;
  int32_t* spiv = (int32_t*)((char*)scratch + (njobs * sizeof(JobDesc) + 255) / 256 * 256);
  int32_t* sinfo = spiv + (int64_t)njobs * piv_ints(NB);
  // one panel with its U12 rows and inverses; tall panels as above
  auto panel = [&](int k) {
    const int rows = npad_max - k, rest = rows - NB;
    if (rows > tall_rows && scratch) {
      sym_tall_setup_kernel<<<(njobs + 255) / 256, 256, 0, s>>>(jobs, njobs, k, sub, sinfo, piv);
      launch_panel<float2>(sub, njobs, 0, 0, NB, work, spiv, sinfo, s, 1);
      sym_tall_info_kernel<<<(njobs + 255) / 256, 256, 0, s>>>(njobs, k, sinfo, info);
      launch_linv<float2>(jobs, njobs, k, work, s);
      if (rest > 0) {
        tslu_l21_kernel<float2><<<dim3((rest + 63) / 64, njobs), 256, 0, s>>>(jobs, k, work);
        sym_u12_kernel<float2><<<dim3(rest / 64, njobs), 256, 0, s>>>(jobs, k, work, 1);
      }
      return;
    }
    launch_panel<float2>(jobs, njobs, k, 0, rows, work, piv, info, s, 1);
    if (rest > 0) sym_u12_kernel<float2><<<dim3(rest / 64, njobs), 256, 0, s>>>(jobs, k, work, 0);
    launch_linv<float2>(jobs, njobs, k, work, s);
  };
  auto timed = [&](int k, int kd, int rb, bool lower, int c_end) {
    const int rows = npad_max - rb;
    if (rows <= 0) return;
    if (prof) prof->before(s);
    if (lower)
      launch_gemm_f32_lower(jobs, njobs, rows, k, kd, rb, work, s);
    else
      launch_gemm_f32(0, jobs, njobs, rows, std::min(c_end, npad_max) - rb, k, kd, rb, rb, c_end, work, s);
    if (prof) {
      // algorithmic work: the lower triangle (with diagonal) of each job's unpadded block
      double f = 0.0, b = 0.0;
      for (int j = 0; j < njobs; ++j) {
        const double m = (double)(prof->n_true[j] - rb);
        if (m <= 0) continue;
        const double c = lower ? m : std::min((double)(c_end - rb), m);
        const double e = lower ? m * (m + 1) / 2 : m * c;
        f += 8.0 * e * kd;
        b += 8.0 * (m * kd + kd * c + 2.0 * e);
      }
      prof->after(s, f, b, lower ? 1 : 0);
    }
  };
  (void)gemm_variant;
  for (int k = 0; k < npad_max; k += 2 * NB) {
    panel(k);
    const int rest = npad_max - k - NB;
    if (rest <= 0) break;
    timed(k, NB, k + NB, false, k + 2 * NB);  // the second panel's columns
    panel(k + NB);
    const int rest2 = npad_max - k - 2 * NB;
    if (rest2 <= 0) break;
    timed(k, 2 * NB, k + 2 * NB, true, 0);
  }
}

// The updates of a panel's columns within its group (64 columns, K < G NB) take the narrow
// tiling; the K = G NB updates (split or not at the look-ahead panel) take the wide one, so
// every element sums in the same order with and without the look-ahead stream.
void lu_factor_f64(const JobDesc* jobs, int njobs, int npad_max, double2* work, int32_t* piv, int32_t* info,
                   hipStream_t s, GemmProfiler* prof, Tiling tiling, const TallScratch& tall, const SideStream* side) {
  lu_factor_any<double2>(jobs, njobs, npad_max, work, piv, info, s, prof, tall, side, tiling.panel_small_rows,
                         tiling.group, [&](int rows, int cols, int k, int kd, int rb, int cb, int ce) {
                           launch_gemm_f64_variant(kd < tiling.group * NB ? tiling.narrow : tiling.wide, jobs, njobs,
                                                   rows, cols, k, kd, rb, cb, ce, work, s);
                         });
}

void lu_factor_f32(const JobDesc* jobs, int njobs, int npad_max, float2* work, int32_t* piv, int32_t* info,
                   hipStream_t s, GemmProfiler* prof, Tiling tiling, const TallScratch& tall, const SideStream* side) {
  lu_factor_any<float2>(jobs, njobs, npad_max, work, piv, info, s, prof, tall, side, tiling.panel_small_rows,
                        tiling.group, [&](int rows, int cols, int k, int kd, int rb, int cb, int ce) {
                          launch_gemm_f32_any(kd < tiling.group * NB ? tiling.narrow : tiling.wide, jobs, njobs,
                                              rows, cols, k, kd, rb, cb, ce, work, s);
                        });
}

}  // namespace lsms
