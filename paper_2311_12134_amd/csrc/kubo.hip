// Kubo-Greenwood sums of Eq. (10) and the four-term combination of Eq. (7).
//
// For atom m (one workgroup) and every LIZ member a, with X_a(z) = tau^{a0}(z) and the
// row tau^{0a}(z) = X_a(z)^T (reciprocity of the complex-symmetric T^-1 - g):
//   s_m[c][mu][nu] += Tr[ J^{m mu}(z2,z1) X_a(z1)^T J^{a nu}(z1,z2) X_a(z2) ]
//                  = sum_{ij} (J0_mu X1^T)_{ij} (Ja_nu X2)_{ji}
// Thread (i, j) of the 16 x 16 workgroup forms one entry of each product for the four
// combos and three directions, then accumulates either the diagonal mu = nu (12 sums)
// or the full tensor (36 sums: the same six products per combo, nine pairings), and
// the workgroup reduces at the end.  The sum over atoms then runs in a fixed order in a
// single workgroup, so sigma is reproducible.
#include "lsms_internal.h"

namespace lsms {

__device__ inline int combo_z1(int c) { return c >> 1; }  // (+,+) (+,-) (-,+) (-,-)
__device__ inline int combo_z2(int c) { return c & 1; }

template <bool TENSOR>
__global__ __launch_bounds__(256) void kubo_trace_kernel(const int64_t* liz_ptr, const int32_t* liz_atom,
                                                         const double2* tau_plus, const double2* tau_minus,
                                                         const int32_t* species, int n_species,
                                                         const double2* J, double2* per_atom) {
  constexpr int NQ = TENSOR ? 36 : 12;  // accumulators per atom: [combo][mu] or [combo][mu][nu]
  const int atom = blockIdx.x;
  const int64_t off = liz_ptr[atom];
  const int nl = (int)(liz_ptr[atom + 1] - off);
  const int t = threadIdx.x, i = t >> 4, j = t & 15;
  __shared__ double2 sJ0[12][NL][NL + 1];
  __shared__ double2 sJa[12][NL][NL + 1];
  __shared__ double2 sX[2][NL][NL + 1];
  __shared__ double2 sred[4][NQ];
  const int s0 = species[atom];
  // an out-of-range species index poisons this atom's sums instead of reading past J
  bool bad = s0 < 0 || s0 >= n_species;
  for (int a = 0; a < nl; ++a) {
    const int sa = species[liz_atom[off + a]];
    bad |= sa < 0 || sa >= n_species;
  }
  if (bad) {
    if (t < NQ) per_atom[(int64_t)atom * NQ + t] = make_double2(NAN, NAN);
    return;
  }
  for (int idx = t; idx < 12 * NL * NL; idx += 256) {
    const int cm = idx / (NL * NL), e = idx % (NL * NL);
    sJ0[cm][e / NL][e % NL] = J[((int64_t)s0 * 12 + cm) * NL * NL + e];
  }
  double2 acc[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q) acc[q] = make_double2(0.0, 0.0);
  int cur = -1;
  for (int a = 0; a < nl; ++a) {
    __syncthreads();
    const int sa = species[liz_atom[off + a]];
    sX[0][i][j] = tau_plus[(off + a) * NL * NL + t];
    sX[1][i][j] = tau_minus[(off + a) * NL * NL + t];
    if (sa != cur) {
      for (int idx = t; idx < 12 * NL * NL; idx += 256) {
        const int cm = idx / (NL * NL), e = idx % (NL * NL);
        sJa[cm][e / NL][e % NL] = J[((int64_t)sa * 12 + cm) * NL * NL + e];
      }
      cur = sa;
    }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const int z1 = combo_z1(c), z2 = combo_z2(c);
      const int crev = z2 * 2 + z1;
      double2 p1[3], p2[3];
#pragma unroll
      for (int mu = 0; mu < 3; ++mu) {
        p1[mu] = make_double2(0.0, 0.0);
        p2[mu] = make_double2(0.0, 0.0);
#pragma unroll
        for (int k = 0; k < NL; ++k) {
          p1[mu] = cfma(p1[mu], sJ0[crev * 3 + mu][i][k], sX[z1][j][k]);  // (J0_mu X1^T)_{ij}
          p2[mu] = cfma(p2[mu], sJa[c * 3 + mu][j][k], sX[z2][k][i]);     // (Ja_mu X2)_{ji}
        }
      }
#pragma unroll
      for (int mu = 0; mu < 3; ++mu) {
        if (TENSOR) {
#pragma unroll
          for (int nu = 0; nu < 3; ++nu) acc[c * 9 + mu * 3 + nu] = cfma(acc[c * 9 + mu * 3 + nu], p1[mu], p2[nu]);
        } else {
          acc[c * 3 + mu] = cfma(acc[c * 3 + mu], p1[mu], p2[mu]);
        }
      }
    }
  }
  // workgroup reduction of the accumulators (fixed order)
  const int lane = t & 63, wave = t >> 6;
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    double2 v = acc[q];
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
      v.x += __shfl_xor(v.x, o);
      v.y += __shfl_xor(v.y, o);
    }
    if (lane == 0) sred[wave][q] = v;
  }
  __syncthreads();
  if (t < NQ) {
    double2 v = sred[0][t];
    for (int w = 1; w < 4; ++w) v = cadd(v, sred[w][t]);
    per_atom[(int64_t)atom * NQ + t] = v;
  }
}

void launch_kubo_trace(int n_atoms, const int64_t* liz_ptr_dev, const int32_t* liz_atom, const double2* tau_plus,
                       const double2* tau_minus, const int32_t* species, int n_species, const double2* J,
                       double2* per_atom, bool tensor, hipStream_t s) {
  if (tensor)
    kubo_trace_kernel<true><<<n_atoms, 256, 0, s>>>(liz_ptr_dev, liz_atom, tau_plus, tau_minus, species, n_species,
                                                    J, per_atom);
  else
    kubo_trace_kernel<false><<<n_atoms, 256, 0, s>>>(liz_ptr_dev, liz_atom, tau_plus, tau_minus, species, n_species,
                                                     J, per_atom);
}

// sigma~[c][q] = -(1/(pi V)) sum_m s_m[c][q];  sigma[q] = Re 1/4 (s~++ - s~+- - s~-+ + s~--)
// with q = mu (diagonal, NQ = 12) or q = 3 mu + nu (tensor, NQ = 36).  Thread t sums
// atoms t, t + 256, ...; the wavefronts then reduce in a fixed shuffle order.
template <int NQ>
__global__ __launch_bounds__(256) void kubo_reduce_kernel(int n_atoms, const double2* per_atom, double volume,
                                                          double* sigma, double2* sigma_tilde) {
  __shared__ double2 sred[4][NQ];
  __shared__ double2 stot[NQ];
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  double2 acc[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q) acc[q] = make_double2(0.0, 0.0);
  for (int a = t; a < n_atoms; a += 256) {
#pragma unroll
    for (int q = 0; q < NQ; ++q) acc[q] = cadd(acc[q], per_atom[(int64_t)a * NQ + q]);
  }
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    double2 v = acc[q];
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
      v.x += __shfl_xor(v.x, o);
      v.y += __shfl_xor(v.y, o);
    }
    if (lane == 0) sred[wave][q] = v;
  }
  __syncthreads();
  const double f = -1.0 / (M_PI * volume);
  if (t < NQ) {
    double2 v = sred[0][t];
    for (int w = 1; w < 4; ++w) v = cadd(v, sred[w][t]);
    stot[t] = v;
    sigma_tilde[t] = make_double2(f * v.x, f * v.y);
  }
  __syncthreads();
  constexpr int NS = NQ / 4;
  if (t < NS) {
    const double re = stot[0 * NS + t].x - stot[1 * NS + t].x - stot[2 * NS + t].x + stot[3 * NS + t].x;
    sigma[t] = 0.25 * f * re;
  }
}

void launch_kubo_reduce(int n_atoms, const double2* per_atom, double volume, double* sigma, double2* sigma_tilde,
                        bool tensor, hipStream_t s) {
  if (tensor)
    kubo_reduce_kernel<36><<<1, 256, 0, s>>>(n_atoms, per_atom, volume, sigma, sigma_tilde);
  else
    kubo_reduce_kernel<12><<<1, 256, 0, s>>>(n_atoms, per_atom, volume, sigma, sigma_tilde);
}

}  // namespace lsms
