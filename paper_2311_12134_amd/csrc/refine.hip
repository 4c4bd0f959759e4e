// FP64 iterative refinement for the split-precision solve, and the copy kernels of
// the diagnostic batched-solve entry point.
//
// Classical mixed-precision iterative refinement (Wilkinson; Moler 1967): with FP32
// factors of M, repeat  r = B - M X (FP64, M kept in FP64),  d = U^-1 L^-1 P r (an FP32 solve
// with the FP32 factors on a rounded copy of r),  X += d (FP64),  until the normwise backward error
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

__device__ inline double cabs2(double2 v) { return sqrt(v.x * v.x + v.y * v.y); }

// r = B - M X for 64 rows x 16 columns per workgroup; M X on FP64 MFMA with three real
// products per complex product (Ar Br, Ai Bi, (Ar + Ai)(Br + Bi)): the kernel streams the FP64
// copy of M once per pass, and three products keep the matrix cores under that stream.
// MNORM: also ||M||_inf (the first pass of a refinement; M does not change between passes,
// so the later passes skip the modulus of every element).  The moduli are taken in FP32 (a
// relative error of about 1e-7 in a norm that only scales the backward error) and summed
// in FP64; entries of M = 1 - t g are far below the FP32 range.
template <bool MNORM>
__global__ __launch_bounds__(256) void residual_kernel(const JobDesc* jobs, const double2* m64, const double2* x,
                                                       double2* r, const double2* tpm, const int32_t* liz_atom,
                                                       double* norms, const int32_t* done) {
  const int job = blockIdx.y;
  if (done[job]) return;
  const JobDesc jd = jobs[job];
  const int row0 = blockIdx.x * 64;
  if (row0 >= jd.npad) return;
  const double2* M = m64 + jd.m_off;
  const double2* X = x + jd.x_off;
  double2* R = r + jd.x_off;  // residual blocks mirror the solution blocks' offsets
  const int npad = jd.npad;
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  __shared__ double2 sM[64][16 + 1];
  __shared__ double2 sX[16][16 + 1];
  __shared__ double s_max[3][4];
  d4 t1 = {0, 0, 0, 0}, t2 = {0, 0, 0, 0}, t3 = {0, 0, 0, 0};
  double rowabs = 0.0;
  for (int kc = 0; kc < npad; kc += 16) {
    {
      const int i = t >> 2, k4 = (t & 3) * 4;
      const double2* src = M + (int64_t)(row0 + i) * npad + kc + k4;
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const double2 v = src[u];
        sM[i][k4 + u] = v;
        if (MNORM) rowabs += (double)__builtin_sqrtf((float)(v.x * v.x + v.y * v.y));
      }
      const int kk = t >> 4, c = t & 15;
      sX[kk][c] = X[(int64_t)(kc + kk) * NRHS_MAX + c];
    }
    __syncthreads();
#pragma unroll
    for (int k4 = 0; k4 < 16; k4 += 4) {
      const double2 a = sM[wave * 16 + (lane & 15)][k4 + (lane >> 4)];
      const double2 b = sX[k4 + (lane >> 4)][lane & 15];
      t1 = __builtin_amdgcn_mfma_f64_16x16x4f64(a.x, b.x, t1, 0, 0, 0);
      t2 = __builtin_amdgcn_mfma_f64_16x16x4f64(a.y, b.y, t2, 0, 0, 0);
      t3 = __builtin_amdgcn_mfma_f64_16x16x4f64(a.x + a.y, b.x + b.y, t3, 0, 0, 0);
    }
    __syncthreads();
  }
  // ||M||_inf over this tile's rows: four threads share a row
  rowabs += __shfl_xor(rowabs, 1);
  rowabs += __shfl_xor(rowabs, 2);
  double mmax = rowabs;
  // residual entries: lane l, register q -> row 16*wave + l/16 + 4q, column l%16
  const int col = lane & 15;
  const double2 tc = (col < NL) ? tpm[liz_atom[jd.liz_off] * 8 + jd.energy * 4 +
                                      (col == 0 ? 0 : (col < 4 ? 1 : (col < 9 ? 2 : 3)))]
                                : make_double2(0, 0);
  double rmax = 0.0;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int row = row0 + wave * 16 + (lane >> 4) + 4 * q;
    double2 b = (row == col) ? tc : make_double2(0.0, 0.0);
    double2 rv = make_double2(b.x - (t1[q] - t2[q]), b.y - (t3[q] - t1[q] - t2[q]));
    R[(int64_t)row * NRHS_MAX + col] = rv;
    double a = cabs2(rv);
#pragma unroll
    for (int o = 1; o < 16; o <<= 1) a += __shfl_xor(a, o);
    rmax = fmax(rmax, a);
  }
  // ||X||_inf over the tile's rows
  double xmax = 0.0;
  if (t < 64) {
    double s = 0.0;
    for (int c = 0; c < 16; ++c) s += cabs2(X[(int64_t)(row0 + t) * NRHS_MAX + c]);
    xmax = s;
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
    double v = fmax(fmax(s_max[t][0], s_max[t][1]), fmax(s_max[t][2], s_max[t][3]));
    atomic_max_nonneg(norms + job * 8 + t, v);
  }
  if (t == 3 && row0 == 0) {
    double b = 0.0;
    for (int l = 0; l < 4; ++l) b = fmax(b, cabs2(tpm[liz_atom[jd.liz_off] * 8 + jd.energy * 4 + l]));
    norms[job * 8 + 4] = b;
  }
}

void launch_residual_norms(const JobDesc* jobs, int njobs, int npad_max, const double2* m64, const double2* x,
                           double2* r, const double2* tpm, const int32_t* liz_atom, double* norms,
                           const int32_t* done, int first, hipStream_t s) {
  dim3 grid(npad_max / 64, njobs);
  if (first)
    residual_kernel<true><<<grid, 256, 0, s>>>(jobs, m64, x, r, tpm, liz_atom, norms, done);
  else
    residual_kernel<false><<<grid, 256, 0, s>>>(jobs, m64, x, r, tpm, liz_atom, norms, done);
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
