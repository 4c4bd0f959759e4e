// FP64 iterative refinement for the split-precision solve, and the copy kernels of
// the diagnostic batched-solve entry point.
//
// Classical mixed-precision iterative refinement (Wilkinson; Moler 1967): with FP32
// factors of M, repeat  r = B - M X (FP64),  d = U^-1 L^-1 P r (an FP32 solve with the FP32
// factors on a rounded copy of r),  X += d (FP64),  until the normwise backward error
//   berr = ||r||_inf / (||M||_inf ||X||_inf + ||B||_inf)
// reaches the requested tolerance.  B = E0 t_centre is regenerated from the t-matrix.
// Per-job norms live in norms[job][8]: 0 ||M||, 1 ||r||, 2 ||X||, 3 berr, 4 ||B||.
#include "lsms_internal.h"

namespace lsms {

typedef double d4 __attribute__((ext_vector_type(4)));

__device__ inline void atomic_max_nonneg(double* addr, double v) {
  // non-negative doubles order like their bit patterns
  atomicMax((unsigned long long*)addr, (unsigned long long)__double_as_longlong(v));
}

__device__ inline double cabs_(double2 v) { return sqrt(v.x * v.x + v.y * v.y); }
__device__ inline int lch(int L) { return L < 1 ? 0 : L < 4 ? 1 : L < 9 ? 2 : 3; }  // l of channel L

// z i^e
__device__ inline double2 ipow_mul(double2 z, int e) {
  e &= 3;
  return e == 0 ? z : e == 1 ? make_double2(-z.y, z.x) : e == 2 ? make_double2(-z.x, -z.y) : make_double2(z.y, -z.x);
}

// The residual uses M = 1 - D G E (G the structure constants, zero diagonal blocks and
// padding; D = T, E = 1, or D = E = T^{1/2} in the symmetric form) through the packed
// contractions v (g^{ab} = I v^{ab} I^{-1}, I = diag(i^l)):
//   r_a = B_a - X_a + D_a I sum_{b != a} v^{ab} X'_b,   X'_b = I^{-1} E_b X_b.
// rotate_x_kernel forms X' once per pass, in columns 16 .. 31 of the residual rows (their
// columns 0 .. 15 receive the residual); zero on padding members.
__global__ void rotate_x_kernel(const JobDesc* jobs, const int32_t* liz_atom, const double2* spm, const double2* x,
                                double2* r, const int32_t* done) {
  const int job = blockIdx.y;
  if (done[job]) return;
  const JobDesc jd = jobs[job];
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= jd.npad * NL) return;
  const int row = idx / NL, c = idx % NL, site = row / NL, L = row % NL;
  double2 v = make_double2(0.0, 0.0);
  if (site < jd.nl) {
    v = x[jd.x_off + (int64_t)row * NRHS_MAX + c];
    if (spm) v = cmul(spm[liz_atom[jd.liz_off + site] * 8 + jd.energy * 4 + lch(L)], v);
    v = ipow_mul(v, -lch(L));
  }
  r[jd.x_off + (int64_t)row * NRHS_MAX + NL + c] = v;
}

// r = B - M X for the 16 rows of one member per wavefront (four per workgroup): per member
// b != a the 16 x 16 block v^{ab} is read from the packed table straight into the FP64 MFMA
// operand layout (lane l, step s: entry (l % 16, 4 s + l / 16), the table's upper triangle by
// symmetry; reversed pairs take the sign (-1)^{l + l'}), X'_b from the rotated rows, and
// v X' accumulates with three real products per complex product (Ar Br, Ai Bi,
// (Ar + Ai)(Br + Bi)); table blocks load RDEPTH members ahead, X' one member ahead, while
// the current products run.  Reads 2176 bytes of table per block instead of the 4 KB of a
// stored FP64 block of M; these reads do not bound the kernel (loading further ahead, or
// keeping the loads ahead of the products, leaves its time unchanged).
// Each pair's block has two readers (rows a and b): the members are visited in the cyclic
// order a + 1, a - 1, a + 2, a - 2, ... (mod nl), so both readers of pair (a, a + t) reach it
// within one block of each other, and a job's workgroups are dealt to one XCD (workgroups
// go to the eight XCDs round-robin), so that the second read may find the block in that
// XCD's L2 (the fetch counters show it mostly does not; the order costs nothing).
// MNORM: also ||M||_inf (first pass of a refinement): per row 1 + |d_l| sum |v e|, the moduli
// in FP32 (a relative error of about 1e-7 in a norm that only scales the backward error),
// summed in FP64.
constexpr int RDEPTH = 2;
static_assert(RDEPTH % 2 == 0, "the X' register sets alternate by block parity across the unrolled steps");

template <bool MNORM, bool SYM>
__global__ __launch_bounds__(256, MNORM && SYM ? 2 : 3) void residual_kernel(const JobDesc* jobs, const double2* vtab,
                                                       const int32_t* liz_atom, const double2* dtab,
                                                       const double2* x, double2* r, double* norms,
                                                       const int32_t* done, int tiles) {
  int T = blockIdx.x;
  {
    const int N = gridDim.x, q = N >> 3, r = N & 7, x = T & 7;
    T = x * q + min(x, r) + (T >> 3);
  }
  const int job = T / tiles;
  if (done[job]) return;
  const JobDesc jd = jobs[job];
  const int row0 = (T - job * tiles) * 64;
  if (row0 >= jd.npad) return;
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int a = row0 / NL + wave;  // this wavefront's member (16 rows)
  const int nl = jd.nl, nb = jd.npad / NL;
  __shared__ double s_max[3][4];
  const double2* X = x + jd.x_off;
  double2* R = r + jd.x_off;
  const double2* Xr = R + NL;  // X'
  const double2* V = vtab + jd.v_off;
  const int eoff = jd.energy * 4;
  d4 t1 = {0, 0, 0, 0}, t2 = {0, 0, 0, 0}, t3 = {0, 0, 0, 0};
  double rowabs = 0.0;
  if (a < nl) {  // uniform per wavefront
    const int i = lane & 15;
    int toff[4];
    double sg[4];
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const int k = 4 * s + (lane >> 4);
      toff[s] = i <= k ? vblock_index(i, k) : vblock_index(k, i);
      sg[s] = ((lch(i) + lch(k)) & 1) ? -1.0 : 1.0;
    }
    const int xo = (lane >> 4) * NRHS_MAX + i;  // X' entry (row b NL + lane / 16 + 4 s)
    // block k of the cyclic order: member a + (k / 2 + 1) for even k, a - (k / 2 + 1) for odd k
    auto member = [&](int k) {
      const int d = (k >> 1) + 1;
      return (k & 1) ? (a - d + nl) % nl : (a + d) % nl;
    };
    const int nblk = nl - 1;
    auto load_v = [&](int k, double2* av) {
      if (k < nblk) {  // uniform
        const int b = member(k);
        const double2* blk = V + pair_index(min(a, b), max(a, b), nb) * VBLOCK;
#pragma unroll
        for (int s = 0; s < 4; ++s) av[s] = blk[toff[s]];
      }
    };
    auto load_x = [&](int k, double2* xv) {
      if (k < nblk) {  // uniform
        const int b = member(k);
#pragma unroll
        for (int s = 0; s < 4; ++s) xv[s] = Xr[(int64_t)b * NL * NRHS_MAX + xo + 4 * s * NRHS_MAX];
      }
    };
    auto mul = [&](int k, const double2* av, const double2* xv) {
      const int b = member(k);
      double2 A[4];
#pragma unroll
      for (int s = 0; s < 4; ++s) A[s] = b < a ? make_double2(sg[s] * av[s].x, sg[s] * av[s].y) : av[s];
      if (MNORM) {
        double2 eb[4];
        if (SYM) {
          const double2* e = dtab + liz_atom[jd.liz_off + b] * 8 + eoff;
#pragma unroll
          for (int s = 0; s < 4; ++s) eb[s] = e[lch(4 * s + (lane >> 4))];
        }
#pragma unroll
        for (int s = 0; s < 4; ++s) {
          double m = (double)__builtin_sqrtf((float)(A[s].x * A[s].x + A[s].y * A[s].y));
          if (SYM) m *= cabs_(eb[s]);
          rowabs += m;
        }
      }
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        t1 = __builtin_amdgcn_mfma_f64_16x16x4f64(A[s].x, xv[s].x, t1, 0, 0, 0);
        t2 = __builtin_amdgcn_mfma_f64_16x16x4f64(A[s].y, xv[s].y, t2, 0, 0, 0);
        t3 = __builtin_amdgcn_mfma_f64_16x16x4f64(A[s].x + A[s].y, xv[s].x + xv[s].y, t3, 0, 0, 0);
      }
    };
    // table blocks load RDEPTH blocks ahead (they come from HBM), X' one block ahead (it stays
    // in L2); static register sets through unrolling
    double2 av[RDEPTH][4], xv[2][4];
#pragma unroll
    for (int u = 0; u < RDEPTH; ++u) load_v(u, av[u]);
    load_x(0, xv[0]);
    for (int k = 0; k < nblk; k += RDEPTH) {
#pragma unroll
      for (int u = 0; u < RDEPTH; ++u) {
        if (k + u < nblk) {  // uniform
          load_x(k + u + 1, xv[(u + 1) & 1]);
          mul(k + u, av[u], xv[u & 1]);
          load_v(k + u + RDEPTH, av[u]);
        }
      }
    }
  }
  // ||M||_inf over the member's rows: lanes l, l + 16, l + 32, l + 48 hold parts of row l % 16
  double mmax = 1.0;
  if (MNORM) {
    rowabs += __shfl_xor(rowabs, 16);
    rowabs += __shfl_xor(rowabs, 32);
    if (a < nl) mmax = 1.0 + cabs_(dtab[liz_atom[jd.liz_off + a] * 8 + eoff + lch(lane & 15)]) * rowabs;
  }
  // residual entries: lane l, register q -> row 16 a + l / 16 + 4 q, column l % 16
  const int col = lane & 15;
  const double2 tc = dtab[liz_atom[jd.liz_off] * 8 + eoff + lch(col)];  // B = E0 t_centre (or s_centre)
  const double2* da = a < nl ? dtab + liz_atom[jd.liz_off + a] * 8 + eoff : nullptr;
  double rmax = 0.0;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int i = (lane >> 4) + 4 * q, row = a * NL + i;
    const double2 xv = X[(int64_t)row * NRHS_MAX + col];
    double2 rv = (row == col) ? tc : make_double2(0.0, 0.0);
    rv.x -= xv.x;
    rv.y -= xv.y;
    if (da) {  // + d_l i^l (v X')
      const double2 dg = cmul(ipow_mul(da[lch(i)], lch(i)), make_double2(t1[q] - t2[q], t3[q] - t1[q] - t2[q]));
      rv.x += dg.x;
      rv.y += dg.y;
    }
    R[(int64_t)row * NRHS_MAX + col] = rv;
    double v = cabs_(rv);
#pragma unroll
    for (int o = 1; o < 16; o <<= 1) v += __shfl_xor(v, o);
    rmax = fmax(rmax, v);
  }
  // ||X||_inf over the workgroup's rows
  double xmax = 0.0;
  if (t < 64) {
    double v = 0.0;
    for (int c = 0; c < 16; ++c) v += cabs_(X[(int64_t)(row0 + t) * NRHS_MAX + c]);
    xmax = v;
  }
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) {
    mmax = fmax(mmax, __shfl_xor(mmax, o));
    rmax = fmax(rmax, __shfl_xor(rmax, o));
    xmax = fmax(xmax, __shfl_xor(xmax, o));
  }
  if (lane == 0) {
    s_max[0][wave] = mmax;
    s_max[1][wave] = rmax;
    s_max[2][wave] = xmax;
  }
  __syncthreads();
  if (t < 3 && (MNORM || t > 0)) {
    const double v = fmax(fmax(s_max[t][0], s_max[t][1]), fmax(s_max[t][2], s_max[t][3]));
    atomic_max_nonneg(norms + job * 8 + t, v);
  }
  if (t == 3 && row0 == 0) {
    double b = 0.0;
    for (int l = 0; l < 4; ++l) b = fmax(b, cabs_(dtab[liz_atom[jd.liz_off] * 8 + eoff + l]));
    norms[job * 8 + 4] = b;
  }
}

void launch_residual(const JobDesc* jobs, int njobs, int npad_max, const double2* vtab, const int32_t* liz_atom,
                     const double2* tpm, const double2* spm, const double2* x, double2* r, double* norms,
                     const int32_t* done, int first, hipStream_t s) {
  rotate_x_kernel<<<dim3((npad_max * NL + 255) / 256, njobs), 256, 0, s>>>(jobs, liz_atom, spm, x, r, done);
  const int tiles = npad_max / 64;
  const dim3 grid(tiles * njobs);
  const double2* d = spm ? spm : tpm;
  if (spm) {
    if (first)
      residual_kernel<true, true><<<grid, 256, 0, s>>>(jobs, vtab, liz_atom, d, x, r, norms, done, tiles);
    else
      residual_kernel<false, true><<<grid, 256, 0, s>>>(jobs, vtab, liz_atom, d, x, r, norms, done, tiles);
  } else {
    if (first)
      residual_kernel<true, false><<<grid, 256, 0, s>>>(jobs, vtab, liz_atom, d, x, r, norms, done, tiles);
    else
      residual_kernel<false, false><<<grid, 256, 0, s>>>(jobs, vtab, liz_atom, d, x, r, norms, done, tiles);
  }
}

// Backward error of every pending job; jobs that reach tol are marked done, the others
// are counted in *pending (one int, cleared by the caller before the launch).  Jobs that
// are flagged already (zero pivot, bad input) are not refined.
__global__ void refine_step_kernel(int njobs, double* norms, double tol, int32_t* done, int last,
                                   int32_t* job_info, int32_t* pending) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= njobs || done[j]) return;
  double* nm = norms + j * 8;
  const double berr = nm[1] / (nm[0] * nm[2] + nm[4]);
  nm[3] = berr;
  if (berr <= tol || job_info[j] != 0) {
    done[j] = 1;
  } else {
    atomicAdd(pending, 1);
    if (last) job_info[j] = -1;
  }
  nm[1] = 0.0;  // ||M|| (nm[0]) is kept for the next pass
  nm[2] = 0.0;
}

// Symmetric form (no pivoting): an exact zero pivot says nothing about S itself, so the
// system goes to the FP64 LU with partial pivoting like one whose refinement failed.
__global__ void zero_pivot_to_fallback_kernel(int njobs, int32_t* job_info) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j < njobs && job_info[j] > 0) job_info[j] = -1;
}

void launch_zero_pivot_to_fallback(int njobs, int32_t* job_info, hipStream_t s) {
  zero_pivot_to_fallback_kernel<<<(njobs + 255) / 256, 256, 0, s>>>(njobs, job_info);
}

// After the FP64 fallback: a zero pivot of the partial-pivoting LU marks the system singular,
// and the backward error of the discarded split-mode solution no longer describes the
// returned one, so it is replaced by the sentinel -1.
__global__ void fallback_status_kernel(int nf, const JobDesc* fjobs, const int32_t* finfo, int32_t* job_info,
                                       double* norms) {
  const int f = blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= nf) return;
  const int j = fjobs[f].info;
  if (finfo[f] > 0) job_info[j] = finfo[f];
  norms[j * 8 + 3] = -1.0;
}

void launch_fallback_status(int nf, const JobDesc* fjobs, const int32_t* finfo, int32_t* job_info, double* norms,
                            hipStream_t s) {
  fallback_status_kernel<<<(nf + 255) / 256, 256, 0, s>>>(nf, fjobs, finfo, job_info, norms);
}

void launch_refine_step(const JobDesc* jobs, int njobs, double* norms, double tol, int32_t* done, int last,
                        int32_t* job_info, int32_t* pending, hipStream_t s) {
  (void)jobs;
  refine_step_kernel<<<(njobs + 255) / 256, 256, 0, s>>>(njobs, norms, tol, done, last, job_info, pending);
}

// The split-mode refinement solves in FP32 in columns 16 .. 23 of each solution row (the
// forward solves use columns 0 .. 15 only): mode 0 rounds src columns 0 .. 15 into that copy,
// mode 1 widens the copy into x, mode 2 adds it to x (the correction of a refinement step).
__global__ void x32_kernel(const JobDesc* jobs, int mode, const double2* src, double2* x, const int32_t* done) {
  const int job = blockIdx.y;
  if (done && done[job]) return;
  const JobDesc jd = jobs[job];
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= jd.npad * NL) return;
  const int row = idx / NL, c = idx % NL;
  const int64_t o = jd.x_off + (int64_t)row * NRHS_MAX + c;
  float2* v = (float2*)(x + jd.x_off) + 2 * 16 + (int64_t)row * 2 * NRHS_MAX + c;
  if (mode == 0) {
    const double2 a = src[o];
    *v = make_float2((float)a.x, (float)a.y);
  } else {
    const double2 d = make_double2((double)v->x, (double)v->y);
    x[o] = mode == 1 ? d : cadd(x[o], d);
  }
}

void launch_x32(const JobDesc* jobs, int njobs, int npad_max, int mode, const double2* src, double2* x,
                const int32_t* done, hipStream_t s) {
  dim3 grid((npad_max * NL + 255) / 256, njobs);
  x32_kernel<<<grid, 256, 0, s>>>(jobs, mode, src, x, done);
}

__global__ void zero_i32_kernel(int32_t* p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}

void launch_zero_i32(int32_t* p, int n, hipStream_t s) {
  if (n <= 0) return;
  zero_i32_kernel<<<(n + 255) / 256, 256, 0, s>>>(p, n);
}

// diagnostic entry: caller matrices (row-major n x n, complex double) into padded work
template <typename T>
__global__ void load_user_kernel(const JobDesc* jobs, void* const* A_dev, void* const* B_dev, int nrhs, T* work,
                                 double2* x) {
  const JobDesc jd = jobs[blockIdx.y];
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t n2 = (int64_t)jd.npad * jd.npad;
  const double2* A = (const double2*)A_dev[jd.atom];
  const double2* B = (const double2*)B_dev[jd.atom];
  if (idx < n2) {
    const int row = (int)(idx / jd.npad), col = (int)(idx % jd.npad);
    double2 v;
    if (row < jd.n && col < jd.n)
      v = A[(int64_t)row * jd.n + col];
    else
      v = make_double2(row == col ? 1.0 : 0.0, 0.0);
    st2(work + jd.a_off + idx, v);
  }
  if (idx < (int64_t)jd.npad * NRHS_MAX) {
    const int row = (int)(idx / NRHS_MAX), col = (int)(idx % NRHS_MAX);
    x[jd.x_off + idx] = (row < jd.n && col < nrhs) ? B[(int64_t)row * nrhs + col] : make_double2(0.0, 0.0);
  }
}

void launch_load_user(const JobDesc* jobs, int njobs, int npad_max, void* const* A_dev, void* const* B_dev, int nrhs,
                      int precision, void* work, double2* x, hipStream_t s) {
  const int64_t n2 = (int64_t)npad_max * npad_max;
  dim3 grid((unsigned)((n2 + 255) / 256), njobs);
  if (precision == 1)
    load_user_kernel<float2><<<grid, 256, 0, s>>>(jobs, A_dev, B_dev, nrhs, (float2*)work, x);
  else
    load_user_kernel<double2><<<grid, 256, 0, s>>>(jobs, A_dev, B_dev, nrhs, (double2*)work, x);
}

__global__ void store_user_kernel(const JobDesc* jobs, void* const* B_dev, int nrhs, const double2* x) {
  const JobDesc jd = jobs[blockIdx.y];
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= jd.n * nrhs) return;
  const int row = idx / nrhs, col = idx % nrhs;
  ((double2*)B_dev[jd.atom])[idx] = x[jd.x_off + (int64_t)row * NRHS_MAX + col];
}

void launch_store_user(const JobDesc* jobs, int njobs, int npad_max, void* const* B_dev, int nrhs, const double2* x,
                       hipStream_t s) {
  dim3 grid((npad_max * nrhs + 255) / 256, njobs);
  store_user_kernel<<<grid, 256, 0, s>>>(jobs, B_dev, nrhs, x);
}

}  // namespace lsms
