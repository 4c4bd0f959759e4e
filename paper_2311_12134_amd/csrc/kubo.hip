// Kubo-Greenwood sums of Eq. (10) and the four-term combination of Eq. (7).
//
// For atom m (one workgroup) and every LIZ member a, with X_a(z) = tau^{a0}(z) and the
// row tau^{0a}(z) = X_a(z)^T (reciprocity of the complex-symmetric T^-1 - g):
//   s_m[c][mu] += Tr[ J^{m mu}(z2,z1) X_a(z1)^T J^{a mu}(z1,z2) X_a(z2) ]
//              = sum_{ij} (J0 X1^T)_{ij} (Ja X2)_{ji}
// Thread (i, j) of the 16 x 16 workgroup forms one entry of each product, for the
// twelve (combo, direction) pairs, and the workgroup reduces at the end.  The sum over
// atoms then runs in a fixed order in a single workgroup, so sigma is reproducible.
#include "lsms_internal.h"

namespace lsms {

__device__ inline int combo_z1(int c) { return c >> 1; }  // (+,+) (+,-) (-,+) (-,-)
__device__ inline int combo_z2(int c) { return c & 1; }

__global__ __launch_bounds__(256) void kubo_trace_kernel(const int64_t* liz_ptr, const int32_t* liz_atom,
                                                         const double2* tau_plus, const double2* tau_minus,
                                                         const int32_t* species, int n_species,
                                                         const double2* J, double2* per_atom) {
  const int atom = blockIdx.x;
  const int64_t off = liz_ptr[atom];
  const int nl = (int)(liz_ptr[atom + 1] - off);
  const int t = threadIdx.x, i = t >> 4, j = t & 15;
  __shared__ double2 sJ0[12][NL][NL + 1];
  __shared__ double2 sJa[12][NL][NL + 1];
  __shared__ double2 sX[2][NL][NL + 1];
  __shared__ double2 sred[4][12];
  const int s0 = species[atom];
  // an out-of-range species index poisons this atom's sums instead of reading past J
  bool bad = s0 < 0 || s0 >= n_species;
  for (int a = 0; a < nl; ++a) {
    const int sa = species[liz_atom[off + a]];
    bad |= sa < 0 || sa >= n_species;
  }
  if (bad) {
    if (t < 12) per_atom[(int64_t)atom * 12 + t] = make_double2(NAN, NAN);
    return;
  }
  for (int idx = t; idx < 12 * NL * NL; idx += 256) {
    const int cm = idx / (NL * NL), e = idx % (NL * NL);
    sJ0[cm][e / NL][e % NL] = J[((int64_t)s0 * 12 + cm) * NL * NL + e];
  }
  double2 acc[12];
#pragma unroll
  for (int q = 0; q < 12; ++q) acc[q] = make_double2(0.0, 0.0);
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
#pragma unroll
      for (int mu = 0; mu < 3; ++mu) {
        double2 p1 = make_double2(0.0, 0.0), p2 = make_double2(0.0, 0.0);
#pragma unroll
        for (int k = 0; k < NL; ++k) {
          p1 = cfma(p1, sJ0[crev * 3 + mu][i][k], sX[z1][j][k]);  // (J0 X1^T)_{ij}
          p2 = cfma(p2, sJa[c * 3 + mu][j][k], sX[z2][k][i]);     // (Ja X2)_{ji}
        }
        acc[c * 3 + mu] = cfma(acc[c * 3 + mu], p1, p2);
      }
    }
  }
  // workgroup reduction of the twelve accumulators (fixed order)
  const int lane = t & 63, wave = t >> 6;
#pragma unroll
  for (int q = 0; q < 12; ++q) {
    double2 v = acc[q];
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
      v.x += __shfl_xor(v.x, o);
      v.y += __shfl_xor(v.y, o);
    }
    if (lane == 0) sred[wave][q] = v;
  }
  __syncthreads();
  if (t < 12) {
    double2 v = sred[0][t];
    for (int w = 1; w < 4; ++w) v = cadd(v, sred[w][t]);
    per_atom[(int64_t)atom * 12 + t] = v;
  }
}

void launch_kubo_trace(int n_atoms, const int64_t* liz_ptr_dev, const int32_t* liz_atom, const double2* tau_plus,
                       const double2* tau_minus, const int32_t* species, int n_species, const double2* J,
                       double2* per_atom, hipStream_t s) {
  kubo_trace_kernel<<<n_atoms, 256, 0, s>>>(liz_ptr_dev, liz_atom, tau_plus, tau_minus, species, n_species, J,
                                            per_atom);
}

// sigma~[c][mu] = -(1/(pi V)) sum_m s_m[c][mu];  sigma[mu] = Re 1/4 (s~++ - s~+- - s~-+ + s~--)
__global__ __launch_bounds__(256) void kubo_reduce_kernel(int n_atoms, const double2* per_atom, double volume,
                                                          double* sigma, double2* sigma_tilde) {
  __shared__ double2 sbuf[256][12];
  const int t = threadIdx.x;
  double2 acc[12];
#pragma unroll
  for (int q = 0; q < 12; ++q) acc[q] = make_double2(0.0, 0.0);
  for (int a = t; a < n_atoms; a += 256) {
#pragma unroll
    for (int q = 0; q < 12; ++q) acc[q] = cadd(acc[q], per_atom[(int64_t)a * 12 + q]);
  }
#pragma unroll
  for (int q = 0; q < 12; ++q) sbuf[t][q] = acc[q];
  __syncthreads();
  for (int h = 128; h >= 1; h >>= 1) {
    if (t < h) {
#pragma unroll
      for (int q = 0; q < 12; ++q) sbuf[t][q] = cadd(sbuf[t][q], sbuf[t + h][q]);
    }
    __syncthreads();
  }
  if (t < 12) {
    const double f = -1.0 / (M_PI * volume);
    const double2 v = sbuf[0][t];
    sigma_tilde[t] = make_double2(f * v.x, f * v.y);
  }
  if (t < 3) {
    const double f = -1.0 / (M_PI * volume);
    const double re = sbuf[0][0 * 3 + t].x - sbuf[0][1 * 3 + t].x - sbuf[0][2 * 3 + t].x + sbuf[0][3 * 3 + t].x;
    sigma[t] = 0.25 * f * re;
  }
}

void launch_kubo_reduce(int n_atoms, const double2* per_atom, double volume, double* sigma, double2* sigma_tilde,
                        hipStream_t s) {
  kubo_reduce_kernel<<<1, 256, 0, s>>>(n_atoms, per_atom, volume, sigma, sigma_tilde);
}

}  // namespace lsms
