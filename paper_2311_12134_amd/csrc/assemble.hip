// Assembly of the KKR matrix M = 1 - T g of every LIZ (Eq. (3)-(4)), the single-site
// t-matrices, the right-hand side E0 t_centre, and small per-job bookkeeping kernels.
//
// Structure constants for LIZ members a != b, R = p_a - p_b:
//   g^{ab}_{LL'} = -4 pi i kappa  sum_{L''} i^{l - l' + l''} C_{L L' L''} h_{l''}(kappa |R|) Y_{L''}(R^)
// with C the Gaunt integrals of three real harmonics and h_l = j_l + i y_l.
// A workgroup produces 32 consecutive pairs of 16 x 16 blocks: the products of the harmonics
// and Hankel functions of each pair are evaluated once (eight lanes per pair), then each
// wavefront contracts its pairs against the Gaunt terms (dealt to lanes by term count, held
// in registers) and writes -t_a * g (row-scaled by the t-matrix of the row's member) and its
// transpose counterpart, or the identity on the diagonal blocks and on the padding; in split
// mode also the packed FP64 contraction of every pair, from which the refinement's residual
// forms M X.
#include <algorithm>
#include <cstring>

#include "lsms_internal.h"
#include "ylm.h"

namespace lsms {

// Gaunt terms dealt to lane slots: the 256 (L, L') pairs sorted by their number of terms and
// dealt to (group r, lane), so the 64 lanes of a group loop over nearly the same count
// (16 iterations over the four groups instead of 28 for the natural order).
constexpr int GT = 7;  // most terms of any (L, L') pair for l, l' <= 3
struct GauntSlots {
  double coef[4][64][GT];    // C_{L L' L''} (0 in padding terms)
  uint16_t l3[4][64][GT];    // L'' | l'' << 8
  uint16_t pair[4][64];      // L | L' << 4 | ((l - l') mod 4) << 8
  int32_t nterm[4];          // iterations of group r
  double ynorm[7][7];        // N_lm of the real harmonics, l, m <= 6
};
__constant__ GauntSlots c_slots;

// Terms per slot group of the lmax = 3 table (the upload checks them): the assembly keeps a
// lane's coefficients in registers, unrolled to these counts.
__host__ __device__ constexpr int slot_terms(int r) { return r == 0 ? 2 : r == 1 ? 3 : r == 2 ? 4 : 7; }
constexpr int SLOT_TERMS_ALL = 16;

static int lidx_h(int L) { return L == 0 ? 0 : (L < 4 ? 1 : (L < 9 ? 2 : 3)); }

hipError_t upload_gaunt(const GauntTable& g) {
  GauntSlots sl;
  std::memset(&sl, 0, sizeof(sl));
  int order[NL * NL];
  for (int p = 0; p < NL * NL; ++p) order[p] = p;
  std::stable_sort(order, order + NL * NL, [&](int x, int y) {
    return (g.start[x + 1] - g.start[x]) < (g.start[y + 1] - g.start[y]);
  });
  for (int i = 0; i < NL * NL; ++i) {
    const int p = order[i], r = i / 64, lane = i % 64;
    const int L = p / NL, Lp = p % NL;
    const int e = ((lidx_h(L) - lidx_h(Lp)) % 4 + 4) % 4;
    sl.pair[r][lane] = (uint16_t)(L | Lp << 4 | e << 8);
    const int n = g.start[p + 1] - g.start[p];
    if (n > GT) return hipErrorInvalidValue;
    sl.nterm[r] = std::max(sl.nterm[r], n);
    for (int j = 0; j < n; ++j) {
      const int l3 = g.l3[g.start[p] + j];
      int ll = 0;
      while ((ll + 1) * (ll + 1) <= l3) ++ll;
      sl.coef[r][lane][j] = g.coef[g.start[p] + j];
      sl.l3[r][lane][j] = (uint16_t)(l3 | ll << 8);
    }
  }
  for (int r = 0; r < 4; ++r)
    if (sl.nterm[r] > slot_terms(r)) return hipErrorInvalidValue;
  for (int l = 0; l <= 6; ++l)
    for (int m = 0; m <= l; ++m) sl.ynorm[l][m] = ylm_norm<6>(l, m);
  return hipMemcpyToSymbol(HIP_SYMBOL(c_slots), &sl, sizeof(GauntSlots));
}

// principal square root, formed without cancellation
__device__ inline double2 csqrt_p(double2 z) {
  const double r = hypot(z.x, z.y);
  if (r == 0.0) return make_double2(0.0, 0.0);
  if (z.x >= 0.0) {
    const double u = sqrt(0.5 * (r + z.x));
    return make_double2(u, z.y / (2.0 * u));
  }
  const double v = sqrt(0.5 * (r - z.x));
  return make_double2(fabs(z.y) / (2.0 * v), z.y >= 0.0 ? v : -v);
}

// t_l(z+) = -sin(d) e^{i d} / kappa+, t(z-) = conj(t(z+)); spm (optional): their principal
// square roots, the scaling of the symmetric form T^{1/2} (1 - g T) T^{-1/2} = 1 - T^{1/2} g T^{1/2}.
__global__ void tmatrix_kernel(const double* phase, int n_atoms, double2 kp, double2* tpm, double2* spm) {
  int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= n_atoms * 4) return;
  int atom = idx / 4, l = idx % 4;
  double d = phase[idx];
  double sd, cd_;
  sincos(d, &sd, &cd_);
  double2 num = make_double2(-sd * cd_, -sd * sd);  // -sin d (cos d + i sin d)
  double2 t = cmul(num, cinv(kp));
  const double2 tm = make_double2(t.x, -t.y);
  tpm[atom * 8 + l] = t;
  tpm[atom * 8 + 4 + l] = tm;
  if (spm) {
    spm[atom * 8 + l] = csqrt_p(t);
    spm[atom * 8 + 4 + l] = csqrt_p(tm);
  }
}

void launch_tmatrix(const double* phase, int n_atoms, double2 kappa_plus, double2* tpm, double2* spm,
                    hipStream_t s) {
  int n = n_atoms * 4;
  tmatrix_kernel<<<(n + 255) / 256, 256, 0, s>>>(phase, n_atoms, kappa_plus, tpm, spm);
}

__device__ inline int lidx(int L) { return L == 0 ? 0 : (L < 4 ? 1 : (L < 9 ? 2 : 3)); }

// P_{l, +-m} = H_l Y_{l, +-m} for one m and l = m .. 6: the real harmonics of the unit vector
// (x, y, z) (see ylm.h), (x + i y)^m and the associated Legendre recurrence in z, times the
// Hankel term of each l.  The l loop runs over every l with the entries below m skipped, so H
// is indexed statically.
__device__ inline void ylm_column_times(int m, double x, double y, double z, const double2* H, double2* P) {
  double c = 1.0, s = 0.0;  // (x + i y)^m
#pragma unroll
  for (int q = 0; q < 6; ++q)
    if (q < m) {
      const double cn = c * x - s * y;
      s = c * y + s * x;
      c = cn;
    }
  double qmm = 1.0;
#pragma unroll
  for (int q = 1; q < 12; q += 2)
    if (q < 2 * m) qmm *= q;  // (2m - 1)!!
  double q2 = 0.0, q1 = qmm;
#pragma unroll
  for (int l = 0; l <= 6; ++l) {
    if (l < m) continue;
    double q;
    if (l == m)
      q = qmm;
    else if (l == m + 1)
      q = z * (2 * m + 1) * qmm;
    else
      q = ((2 * l - 1) * z * q1 - (l + m - 1) * q2) / (double)(l - m);
    if (l > m) {
      q2 = q1;
      q1 = q;
    }
    const double nq = c_slots.ynorm[l][m] * q;
    if (m == 0) {
      P[l * l + l] = make_double2(nq * H[l].x, nq * H[l].y);
    } else {
      const double yc = M_SQRT2 * nq * c, ys = M_SQRT2 * nq * s;
      P[l * l + l + m] = make_double2(yc * H[l].x, yc * H[l].y);
      P[l * l + l - m] = make_double2(ys * H[l].x, ys * H[l].y);
    }
  }
}

// (-4 pi i kappa) i^l h_l(kappa d) for l = 0 .. 6 into H[0 .. 6]: h0 = -i e^{ix}/x,
// h1 = -e^{ix}(x + i)/x^2 (x = kappa d), then the upward recurrence
// h_{l+1} = (2l + 1)/x h_l - h_{l-1}.
__device__ inline void hankel_terms(double2 kappa, double dist, double2* H) {
  const double2 x = make_double2(kappa.x * dist, kappa.y * dist);
  double sx, cx;
  sincos(x.x, &sx, &cx);
  const double ex = exp(-x.y);
  const double2 eix = make_double2(ex * cx, ex * sx);
  const double2 ix = cinv(x);
  const double2 pre = make_double2(4.0 * M_PI * kappa.y, -4.0 * M_PI * kappa.x);  // -4 pi i kappa
  double2 hm = cmul(make_double2(eix.y, -eix.x), ix);                             // h0
  const double2 tq = cmul(eix, make_double2(x.x, x.y + 1.0));
  double2 h = cmul(make_double2(-tq.x, -tq.y), cmul(ix, ix));                      // h1
  H[0] = cmul(pre, hm);
  double2 ph = make_double2(0.0, 1.0);  // i^l
  H[1] = cmul(cmul(pre, ph), h);
  for (int l = 1; l < 6; ++l) {
    const double2 hn = csub(cmul(make_double2((2 * l + 1) * ix.x, (2 * l + 1) * ix.y), h), hm);
    hm = h;
    h = hn;
    ph = make_double2(-ph.y, ph.x);
    H[l + 1] = cmul(cmul(pre, ph), h);
  }
}

// Pair p of the upper triangle a <= b < n of an n x n grid, numbered row by row (row a
// starts at a n - a (a - 1) / 2); p past the end gives some a <= b, unused.
__device__ inline void pair_of(int p, int n, int& a, int& b) {
  const double w = 2.0 * n + 1.0;
  int r = (int)((w - sqrt(fmax(w * w - 8.0 * p, 0.0))) * 0.5);
  r = min(max(r, 0), n - 1);
  while (r > 0 && r * n - r * (r - 1) / 2 > p) --r;
  while (r < n - 1 && (r + 1) * n - (r + 1) * r / 2 <= p) ++r;
  a = r;
  b = r + (p - (r * n - r * (r - 1) / 2));
}

// M = 1 - T g for BPW consecutive pairs a <= b of 16 x 16 blocks of one job (the upper
// triangle of the padded block grid, row by row).  The structure constants are reciprocal,
// g^{ba}_{LL'} = g^{ab}_{L'L} (R -> -R flips Y_{L''} by (-1)^{l''} = (-1)^{l+l'} on the Gaunt
// terms, which cancels the i^{l-l'} phase change of the swap), so one evaluation per pair
// gives both blocks.  Phase 1: eight lanes per pair, lane m < 7 evaluates the Hankel terms
// (-4 pi i kappa) i^l h_l(kappa |R|) and the harmonics Y_{l, +-m} of R^ = (p_a - p_b)/|R| and
// writes P_{L''} = H_{l''} Y_{L''} for its channels to LDS.  Phase 2: each wavefront contracts
// its pairs, every lane over its Gaunt slots (coefficients and P offsets in registers,
// unrolled to the fixed term counts), applies i^{l - l'}, stages g^{ab} in LDS and writes the
// rows of -t_a g^{ab} and of -t_b (g^{ab})^T.  Diagonal and padding blocks are the identity / zero.
// spm != nullptr: the symmetric form, blocks -s_a g_ab s_b (s = t^{1/2}) instead of -t_a g_ab.
// vtab != nullptr (split mode): also the FP64 contraction v^{ab} = i^{-(l - l')} g^{ab} of each
// pair a < b, symmetric in (L, L') (the Gaunt coefficients are), packed as its upper triangle
// (vblock_index), for the refinement's residual: 2176 bytes per pair instead of the 8 KB of
// the two FP64 blocks of M.
constexpr int ASM_PAIRS = 32;  // pairs per workgroup

template <typename T>
__global__ __launch_bounds__(256, 3) void assemble_kernel(const JobDesc* jobs, const double* liz_pos,
                                                       const int32_t* liz_atom, const double2* tpm, double2 kp,
                                                       double2 km, T* work, double2* vtab, const double2* spm) {
  __shared__ double2 s_P[ASM_PAIRS][NL3];
  __shared__ double2 s_G[4][NL][NL + 1];
  const JobDesc jd = jobs[blockIdx.y];
  const int nbp = jd.npad / NL;
  const int npairs = nbp * (nbp + 1) / 2;
  const int p0 = blockIdx.x * ASM_PAIRS;
  if (p0 >= npairs) return;  // uniform
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const double2 kappa = jd.energy == 0 ? kp : km;
  {
    const int q = t >> 3, m = t & 7, pp = p0 + q;
    int a, b;
    pair_of(pp, nbp, a, b);
    if (m < 7 && pp < npairs && a != b && b < jd.nl) {  // a < b < nl
      const double* pa = liz_pos + (jd.liz_off + a) * 3;
      const double* pb = liz_pos + (jd.liz_off + b) * 3;
      const double rx = pa[0] - pb[0], ry = pa[1] - pb[1], rz = pa[2] - pb[2];
      const double dist = sqrt(rx * rx + ry * ry + rz * rz), inv = 1.0 / dist;
      double2 H[7];
      hankel_terms(kappa, dist, H);
      ylm_column_times(m, rx * inv, ry * inv, rz * inv, H, &s_P[q][0]);
    }
  }
  // this lane's Gaunt slots
  double coef[SLOT_TERMS_ALL];
  int pof[SLOT_TERMS_ALL];
  int Ls[4], Lps[4], es[4];
  {
    int k = 0;
#pragma unroll
    for (int g = 0; g < 4; ++g) {
      const int pr = c_slots.pair[g][lane];
      Ls[g] = pr & 15;
      Lps[g] = (pr >> 4) & 15;
      es[g] = pr >> 8;
#pragma unroll
      for (int j = 0; j < slot_terms(g); ++j, ++k) {
        coef[k] = c_slots.coef[g][lane][j];
        pof[k] = c_slots.l3[g][lane][j] & 0xff;
      }
    }
  }
  __syncthreads();
  const int Lr = lane >> 4, Lc = lane & 15;
  for (int q = wave; q < ASM_PAIRS; q += 4) {
    const int pp = p0 + q;
    if (pp >= npairs) break;  // uniform per wavefront
    int a, b;
    pair_of(pp, nbp, a, b);
    const int64_t base_ab = (int64_t)(a * NL) * jd.npad + b * NL;
    const int64_t base_ba = (int64_t)(b * NL) * jd.npad + a * NL;
    if (a != b && b < jd.nl) {
      const double2* P = &s_P[q][0];
      double2 p[SLOT_TERMS_ALL];
#pragma unroll
      for (int k = 0; k < SLOT_TERMS_ALL; ++k) p[k] = P[pof[k]];
      int k = 0;
#pragma unroll
      for (int g = 0; g < 4; ++g) {
        double2 v = make_double2(0.0, 0.0);
#pragma unroll
        for (int j = 0; j < slot_terms(g); ++j, ++k) {
          v.x += coef[k] * p[k].x;
          v.y += coef[k] * p[k].y;
        }
        if (vtab && Ls[g] <= Lps[g]) vtab[jd.v_off + (int64_t)pp * VBLOCK + vblock_index(Ls[g], Lps[g])] = v;
        // i^{l - l'}
        const int e = es[g];
        s_G[wave][Ls[g]][Lps[g]] = e == 0   ? v
                                   : e == 1 ? make_double2(-v.y, v.x)
                                   : e == 2 ? make_double2(-v.x, -v.y)
                                            : make_double2(v.y, -v.x);
      }
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
      const int atom_a = liz_atom[jd.liz_off + a], atom_b = liz_atom[jd.liz_off + b];
      const double2* ta = tpm + atom_a * 8 + jd.energy * 4;
      const double2* tb = tpm + atom_b * 8 + jd.energy * 4;
      const double2* sa = spm ? spm + atom_a * 8 + jd.energy * 4 : nullptr;
      const double2* sb = spm ? spm + atom_b * 8 + jd.energy * 4 : nullptr;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int L = Lr + 4 * r;
        // block (a, b): -t_a g^{ab} (rows scaled), or -s_a g^{ab} s_b
        const double2 gab = s_G[wave][L][Lc];
        const double2 vab = spm ? cmul(cmul(sa[lidx(L)], gab), sb[lidx(Lc)]) : cmul(ta[lidx(L)], gab);
        st2(work + jd.a_off + base_ab + (int64_t)L * jd.npad + Lc, make_double2(-vab.x, -vab.y));
        // block (b, a): g^{ba}_{L Lc} = g^{ab}_{Lc L}
        const double2 gba = s_G[wave][Lc][L];
        const double2 vba = spm ? cmul(cmul(sb[lidx(L)], gba), sa[lidx(Lc)]) : cmul(tb[lidx(L)], gba);
        st2(work + jd.a_off + base_ba + (int64_t)L * jd.npad + Lc, make_double2(-vba.x, -vba.y));
      }
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    } else {  // identity on the diagonal, zero off it (both blocks of an off-diagonal pair)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int L = Lr + 4 * r;
        const double2 v = make_double2((a == b && L == Lc) ? 1.0 : 0.0, 0.0);
        st2(work + jd.a_off + base_ab + (int64_t)L * jd.npad + Lc, v);
        if (a != b) st2(work + jd.a_off + base_ba + (int64_t)L * jd.npad + Lc, v);
      }
    }
  }
}

void launch_assemble_f64(const JobDesc* jobs, int njobs, int npad_max, const double* liz_pos,
                         const int32_t* liz_atom, const double2* tpm, double2 kp, double2 km, double2* work,
                         const double2* spm, hipStream_t s) {
  const int nbp = npad_max / NL;
  dim3 grid((nbp * (nbp + 1) / 2 + ASM_PAIRS - 1) / ASM_PAIRS, njobs);
  assemble_kernel<double2><<<grid, 256, 0, s>>>(jobs, liz_pos, liz_atom, tpm, kp, km, work, nullptr, spm);
}

void launch_assemble_split(const JobDesc* jobs, int njobs, int npad_max, const double* liz_pos,
                           const int32_t* liz_atom, const double2* tpm, double2 kp, double2 km, float2* work,
                           double2* vtab, const double2* spm, hipStream_t s) {
  const int nbp = npad_max / NL;
  dim3 grid((nbp * (nbp + 1) / 2 + ASM_PAIRS - 1) / ASM_PAIRS, njobs);
  assemble_kernel<float2><<<grid, 256, 0, s>>>(jobs, liz_pos, liz_atom, tpm, kp, km, work, vtab, spm);
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
__device__ inline int l_of(int L) { return L < 1 ? 0 : L < 4 ? 1 : L < 9 ? 2 : 3; }

// With mirror set, only z+ jobs exist and each also writes the z- block
// tau(z-)_{LL'} = (-1)^{l+l'} conj(tau(z+)_{LL'}): kappa- = -conj(kappa+) and
// t(z-) = conj t(z+) give g(z-) = P conj(g(z+)) P, P = diag((-1)^l), hence
// 1 - t g and its inverse times t transform the same way.
// With spm (symmetric form) the solution is Y = S^-1 T^{1/2} E0 and tau^{a0} = s_a Y_a.
__global__ void copy_tau_kernel(const JobDesc* jobs, const double2* x, double2* tau_plus, double2* tau_minus,
                                int mirror, const double2* spm, const int32_t* liz_atom) {
  const JobDesc jd = jobs[blockIdx.y];
  int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= jd.n * NL) return;
  int row = idx / NL, col = idx % NL;
  double2* out = jd.energy == 0 ? tau_plus : tau_minus;
  double2 v = x[jd.x_off + (int64_t)row * NRHS_MAX + col];
  if (spm) v = cmul(spm[liz_atom[jd.liz_off + row / NL] * 8 + jd.energy * 4 + l_of(row % NL)], v);
  out[jd.liz_off * NL * NL + idx] = v;
  if (mirror) {
    const double sg = ((l_of(row % NL) + l_of(col)) & 1) ? -1.0 : 1.0;
    tau_minus[jd.liz_off * NL * NL + idx] = make_double2(sg * v.x, -sg * v.y);
  }
}

void launch_copy_tau(const JobDesc* jobs, int njobs, int npad_max, const double2* x, double2* tau_plus,
                     double2* tau_minus, bool mirror, const double2* spm, const int32_t* liz_atom, hipStream_t s) {
  dim3 grid((npad_max * NL + 255) / 256, njobs);
  copy_tau_kernel<<<grid, 256, 0, s>>>(jobs, x, tau_plus, tau_minus, mirror ? 1 : 0, spm, liz_atom);
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
                                    int32_t* info, double* berr, int mirror) {
  int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= njobs) return;
  const JobDesc jd = jobs[j];
  const double b = norms ? norms[j * 8 + 3] : 0.0;
  info[jd.atom * 2 + jd.energy] = job_info[j];
  berr[jd.atom * 2 + jd.energy] = b;
  if (mirror) {  // the z- result is the z+ one transformed: same status
    info[jd.atom * 2 + 1] = job_info[j];
    berr[jd.atom * 2 + 1] = b;
  }
}

void launch_write_status(const JobDesc* jobs, int njobs, const int32_t* job_info, const double* norms,
                         int32_t* info, double* berr, bool mirror, hipStream_t s) {
  write_status_kernel<<<(njobs + 255) / 256, 256, 0, s>>>(jobs, njobs, job_info, norms, info, berr, mirror ? 1 : 0);
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
