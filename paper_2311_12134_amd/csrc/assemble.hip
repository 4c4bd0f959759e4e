// Assembly of the KKR matrix M = 1 - T g of every LIZ (Eq. (3)-(4)), the single-site
// t-matrices, the right-hand side E0 t_centre, and small per-job bookkeeping kernels.
//
// Structure constants for LIZ members a != b, R = p_a - p_b:
//   g^{ab}_{LL'} = -4 pi i kappa  sum_{L''} i^{l - l' + l''} C_{L L' L''} h_{l''}(kappa |R|) Y_{L''}(R^)
// with C the Gaunt integrals of three real harmonics and h_l = j_l + i y_l.
// Each 16 x 16 block is produced by one wavefront: 49 lanes evaluate
// (-4 pi i kappa) i^{l''} h_{l''} Y_{L''} once, then every lane contracts four
// (L, L') entries against the sparse Gaunt table held in constant memory and writes
// -t_a * g (row-scaled by the t-matrix of the row's member), or the identity on the
// diagonal blocks and on the padding.
#include "lsms_internal.h"
#include "ylm.h"

namespace lsms {

__constant__ GauntTable c_gaunt;

hipError_t upload_gaunt(const GauntTable& g) { return hipMemcpyToSymbol(HIP_SYMBOL(c_gaunt), &g, sizeof(GauntTable)); }

// One real harmonic Y_{l m} of the unit vector (x, y, z) (see ylm.h for the convention).
__device__ inline double real_ylm_one(int l, int m, double x, double y, double z) {
  int am = m < 0 ? -m : m;
  double c = 1.0, s = 0.0;
  for (int q = 0; q < am; ++q) {
    double cn = c * x - s * y;
    s = c * y + s * x;
    c = cn;
  }
  double qmm = 1.0;
  for (int q = 1; q < 2 * am; q += 2) qmm *= q;
  double qa = qmm, qb = 0.0;  // Q_{l'}^{am} for l' = current, previous
  double qv = qmm;
  if (l > am) {
    double q1 = z * (2 * am + 1) * qmm;
    qb = qmm;
    qa = q1;
    for (int ll = am + 2; ll <= l; ++ll) {
      double qn = ((2 * ll - 1) * z * qa - (ll + am - 1) * qb) / (double)(ll - am);
      qb = qa;
      qa = qn;
    }
    qv = qa;
  }
  double nrm = ylm_norm<6>(l, am);
  if (m == 0) return nrm * qv;
  return M_SQRT2 * nrm * qv * (m > 0 ? c : s);
}

// t_l(z+) = -sin(d) e^{i d} / kappa+, t(z-) = conj(t(z+)).
__global__ void tmatrix_kernel(const double* phase, int n_atoms, double2 kp, double2* tpm) {
  int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= n_atoms * 4) return;
  int atom = idx / 4, l = idx % 4;
  double d = phase[idx];
  double sd, cd_;
  sincos(d, &sd, &cd_);
  double2 num = make_double2(-sd * cd_, -sd * sd);  // -sin d (cos d + i sin d)
  double2 t = cmul(num, cinv(kp));
  tpm[atom * 8 + l] = t;
  tpm[atom * 8 + 4 + l] = make_double2(t.x, -t.y);
}

void launch_tmatrix(const double* phase, int n_atoms, double2 kappa_plus, double2* tpm, hipStream_t s) {
  int n = n_atoms * 4;
  tmatrix_kernel<<<(n + 255) / 256, 256, 0, s>>>(phase, n_atoms, kappa_plus, tpm);
}

template <typename T>
__global__ __launch_bounds__(256) void assemble_kernel(const JobDesc* jobs, const double* liz_pos,
                                                       const int32_t* liz_atom, const double2* tpm, double2 kp,
                                                       double2 km, T* work, double2* m64) {
  __shared__ double2 s_hy[4][NL3];
  const JobDesc jd = jobs[blockIdx.y];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int nbp = jd.npad / NL;
  const int blk = blockIdx.x * 4 + wave;
  const bool valid = blk < nbp * nbp;
  const int a = valid ? blk / nbp : 0, b = valid ? blk % nbp : 0;
  const bool offdiag = valid && a != b && a < jd.nl && b < jd.nl;
  const double2 kappa = jd.energy == 0 ? kp : km;

  if (offdiag && lane < NL3) {
    const double* pa = liz_pos + (jd.liz_off + a) * 3;
    const double* pb = liz_pos + (jd.liz_off + b) * 3;
    double rx = pa[0] - pb[0], ry = pa[1] - pb[1], rz = pa[2] - pb[2];
    double dist = sqrt(rx * rx + ry * ry + rz * rz);
    double inv = 1.0 / dist;
    int l3 = 0;
    while ((l3 + 1) * (l3 + 1) <= lane) ++l3;
    int m3 = lane - l3 * l3 - l3;
    double y = real_ylm_one(l3, m3, rx * inv, ry * inv, rz * inv);
    // h_l(x), x = kappa * dist: h0 = -i e^{ix}/x, h1 = -e^{ix}(x + i)/x^2, upward recurrence
    double2 x = make_double2(kappa.x * dist, kappa.y * dist);
    double sx, cx;
    sincos(x.x, &sx, &cx);
    double ex = exp(-x.y);
    double2 eix = make_double2(ex * cx, ex * sx);
    double2 ix = cinv(x);
    double2 h0 = cmul(make_double2(eix.y, -eix.x), ix);  // -i e^{ix} / x
    double2 h = h0;
    if (l3 >= 1) {
      double2 t = cmul(eix, make_double2(x.x, x.y + 1.0));
      double2 h1 = cmul(make_double2(-t.x, -t.y), cmul(ix, ix));
      double2 hm = h0;
      h = h1;
      for (int l = 1; l < l3; ++l) {
        double2 hn = csub(cmul(make_double2((2 * l + 1) * ix.x, (2 * l + 1) * ix.y), h), hm);
        hm = h;
        h = hn;
      }
    }
    // (-4 pi i kappa) * i^{l''} * h * Y
    double2 pre = make_double2(4.0 * M_PI * kappa.y, -4.0 * M_PI * kappa.x);  // -4 pi i kappa
    double2 ph = (l3 & 3) == 0 ? make_double2(1, 0)
               : (l3 & 3) == 1 ? make_double2(0, 1)
               : (l3 & 3) == 2 ? make_double2(-1, 0)
                               : make_double2(0, -1);
    double2 v = cmul(cmul(pre, ph), h);
    s_hy[wave][lane] = make_double2(v.x * y, v.y * y);
  }
  __syncthreads();
  if (!valid) return;

  const int Lp = lane & 15;
  const int lp = Lp == 0 ? 0 : (Lp < 4 ? 1 : (Lp < 9 ? 2 : 3));
  double2 t_a = make_double2(0, 0);
  int atom_a = 0;
  if (offdiag) atom_a = liz_atom[jd.liz_off + a];
  const int64_t base = jd.a_off + (int64_t)(a * NL) * jd.npad + b * NL + Lp;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int L = (lane >> 4) + 4 * r;
    const int l = L == 0 ? 0 : (L < 4 ? 1 : (L < 9 ? 2 : 3));
    double2 val;
    if (offdiag) {
      t_a = tpm[atom_a * 8 + jd.energy * 4 + l];
      const int pair = L * NL + Lp;
      double2 g = make_double2(0, 0);
      for (int q = c_gaunt.start[pair]; q < c_gaunt.start[pair + 1]; ++q) {
        double2 hy = s_hy[wave][c_gaunt.l3[q]];
        double cf = c_gaunt.coef[q];
        g.x += cf * hy.x;
        g.y += cf * hy.y;
      }
      int e = ((l - lp) % 4 + 4) % 4;  // i^{l - l'}
      double2 gp = e == 0 ? g : e == 1 ? make_double2(-g.y, g.x) : e == 2 ? make_double2(-g.x, -g.y)
                                                                            : make_double2(g.y, -g.x);
      double2 tg = cmul(t_a, gp);
      val = make_double2(-tg.x, -tg.y);
    } else {
      val = make_double2((a == b && L == Lp) ? 1.0 : 0.0, 0.0);
    }
    const int64_t idx = base + (int64_t)L * jd.npad;
    st2(work + idx, val);
    if (m64) m64[jd.m_off + (int64_t)(a * NL + L) * jd.npad + b * NL + Lp] = val;
  }
}

void launch_assemble_f64(const JobDesc* jobs, int njobs, int npad_max, const double* liz_pos,
                         const int32_t* liz_atom, const double2* tpm, double2 kp, double2 km, double2* work,
                         hipStream_t s) {
  int nbp = npad_max / NL;
  dim3 grid((nbp * nbp + 3) / 4, njobs);
  assemble_kernel<double2><<<grid, 256, 0, s>>>(jobs, liz_pos, liz_atom, tpm, kp, km, work, nullptr);
}

void launch_assemble_split(const JobDesc* jobs, int njobs, int npad_max, const double* liz_pos,
                           const int32_t* liz_atom, const double2* tpm, double2 kp, double2 km, float2* work,
                           double2* m64, hipStream_t s) {
  int nbp = npad_max / NL;
  dim3 grid((nbp * nbp + 3) / 4, njobs);
  assemble_kernel<float2><<<grid, 256, 0, s>>>(jobs, liz_pos, liz_atom, tpm, kp, km, work, m64);
}

// B = E0 t_centre: rows (0, L) carry t_l of the centre on the diagonal.
__global__ void init_rhs_kernel(const JobDesc* jobs, const int32_t* liz_atom, const double2* tpm, double2* x) {
  const JobDesc jd = jobs[blockIdx.y];
  int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)jd.npad * NRHS_MAX) return;
  int row = (int)(idx / NRHS_MAX), col = (int)(idx % NRHS_MAX);
  double2 v = make_double2(0, 0);
  if (row < NL && col == row) {
    int l = row == 0 ? 0 : (row < 4 ? 1 : (row < 9 ? 2 : 3));
    v = tpm[liz_atom[jd.liz_off] * 8 + jd.energy * 4 + l];
  }
  x[jd.x_off + idx] = v;
}

void launch_init_rhs(const JobDesc* jobs, int njobs, int npad_max, const int32_t* liz_atom, const double2* tpm,
                     double2* x, hipStream_t s) {
  int64_t n = (int64_t)npad_max * NRHS_MAX;
  dim3 grid((unsigned)((n + 255) / 256), njobs);
  init_rhs_kernel<<<grid, 256, 0, s>>>(jobs, liz_atom, tpm, x);
}

// tau^{a0}_{LL'} = X[(a, L)][L'] for the first n rows.
__global__ void copy_tau_kernel(const JobDesc* jobs, const double2* x, double2* tau_plus, double2* tau_minus) {
  const JobDesc jd = jobs[blockIdx.y];
  int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= jd.n * NL) return;
  int row = idx / NL, col = idx % NL;
  double2* out = jd.energy == 0 ? tau_plus : tau_minus;
  out[jd.liz_off * NL * NL + idx] = x[jd.x_off + (int64_t)row * NRHS_MAX + col];
}

void launch_copy_tau(const JobDesc* jobs, int njobs, int npad_max, const double2* x, double2* tau_plus,
                     double2* tau_minus, hipStream_t s) {
  dim3 grid((npad_max * NL + 255) / 256, njobs);
  copy_tau_kernel<<<grid, 256, 0, s>>>(jobs, x, tau_plus, tau_minus);
}

__global__ void check_inputs_kernel(const JobDesc* jobs, const double* liz_pos, const int32_t* liz_atom,
                                    const double* phase, int32_t* job_info) {
  const JobDesc jd = jobs[blockIdx.x];
  int bad = 0;
  for (int a = threadIdx.x; a < jd.nl; a += blockDim.x) {
    const double* p = liz_pos + (jd.liz_off + a) * 3;
    const double* ph = phase + (int64_t)liz_atom[jd.liz_off + a] * 4;
    for (int q = 0; q < 3; ++q) bad |= !isfinite(p[q]);
    for (int q = 0; q < 4; ++q) bad |= !isfinite(ph[q]);
  }
  bad = __syncthreads_or(bad);
  if (threadIdx.x == 0) job_info[blockIdx.x] = bad ? -2 : 0;
}

void launch_check_inputs(const JobDesc* jobs, int njobs, const double* liz_pos, const int32_t* liz_atom,
                         const double* phase, int32_t* job_info, hipStream_t s) {
  check_inputs_kernel<<<njobs, 256, 0, s>>>(jobs, liz_pos, liz_atom, phase, job_info);
}

__global__ void write_status_kernel(const JobDesc* jobs, int njobs, const int32_t* job_info, const double* norms,
                                    int32_t* info, double* berr) {
  int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= njobs) return;
  const JobDesc jd = jobs[j];
  info[jd.atom * 2 + jd.energy] = job_info[j];
  berr[jd.atom * 2 + jd.energy] = norms ? norms[j * 8 + 3] : 0.0;
}

void launch_write_status(const JobDesc* jobs, int njobs, const int32_t* job_info, const double* norms,
                         int32_t* info, double* berr, hipStream_t s) {
  write_status_kernel<<<(njobs + 255) / 256, 256, 0, s>>>(jobs, njobs, job_info, norms, info, berr);
}

__global__ void zero_kernel(double* p, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0.0;
}

void launch_zero(double* p, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  zero_kernel<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(p, n);
}

}  // namespace lsms
