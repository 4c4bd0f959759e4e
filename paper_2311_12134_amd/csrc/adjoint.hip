// Adjoint of the tau-solve + Kubo path: d L / d delta_l for L = sum_mu dsigma_mu sigma_mu.
//
// From Eq. (3): with W = (1 - T g)^-1, tau = W T = T W^T and d tau = W dT W^T.  For one
// LIZ and one energy z, the column X = tau E0 therefore changes as dX = W dT W^T E0 and,
// with G = dL/dX (the holomorphic gradient of the Eq. (10) sums with respect to X(z)),
//   dL/dT_pp = sum_j (W^T E0)_pj (W^T G)_pj.
// W^T = (1 - g T)^-1 = M^-T, so one transposed solve with the right-hand sides [G, E0]
// (32 columns) per atom and energy, reusing the forward LU, gives both factors.
// The gradient of s = Tr[A X1^T B X2] (A = J^0(z2,z1), B = J^a(z1,z2)) is B X2 A with
// respect to X1 and B^T X1 A^T with respect to X2; every combo whose z1 or z2 is z adds
// its term with weight dsigma_mu * (+-1/4) * (-1/(pi V)).
// Finally dt_l(z+)/d delta_l = -exp(2 i delta_l)/kappa+ and dt(z-)/d delta = conj of it;
// the z+ and z- contributions are complex conjugates, so each adds its real part.
#include "lsms_internal.h"

namespace lsms {

__constant__ double c_sign[4] = {1.0, -1.0, -1.0, 1.0};

__global__ __launch_bounds__(256) void adjoint_rhs_kernel(const JobDesc* jobs, const int32_t* liz_atom,
                                                          const double2* tau_plus, const double2* tau_minus,
                                                          const int32_t* species, int n_species, const double2* J,
                                                          const double* dsigma, double volume, double2* x) {
  const JobDesc jd = jobs[blockIdx.y];
  const int a = blockIdx.x;
  if (a >= jd.npad / NL) return;  // uniform
  const int t = threadIdx.x, i = t >> 4, j = t & 15;
  double2* X = x + jd.x_off + (int64_t)(a * NL + i) * NRHS_MAX;
  if (a >= jd.nl) {  // padding rows
    X[j] = make_double2(0.0, 0.0);
    X[NL + j] = make_double2(0.0, 0.0);
    return;
  }
  __shared__ double2 sA[12][NL][NL + 1];
  __shared__ double2 sB[12][NL][NL + 1];
  __shared__ double2 sX[2][NL][NL + 1];
  __shared__ double2 sP[NL][NL + 1];
  const int s0 = species[liz_atom[jd.liz_off]];
  const int sa = species[liz_atom[jd.liz_off + a]];
  if (s0 < 0 || s0 >= n_species || sa < 0 || sa >= n_species) {  // never read past J
    X[j] = make_double2(NAN, NAN);
    X[NL + j] = make_double2(0.0, 0.0);
    return;
  }
  for (int idx = t; idx < 12 * NL * NL; idx += 256) {
    const int cm = idx / (NL * NL), e = idx % (NL * NL);
    sA[cm][e / NL][e % NL] = J[((int64_t)s0 * 12 + cm) * NL * NL + e];
    sB[cm][e / NL][e % NL] = J[((int64_t)sa * 12 + cm) * NL * NL + e];
  }
  sX[0][i][j] = tau_plus[(jd.liz_off + a) * NL * NL + t];
  sX[1][i][j] = tau_minus[(jd.liz_off + a) * NL * NL + t];
  __syncthreads();
  const double f = -1.0 / (M_PI * volume);
  const int z = jd.energy;
  double2 g = make_double2(0.0, 0.0);
  for (int c = 0; c < 4; ++c) {
    const int z1 = c >> 1, z2 = c & 1, crev = z2 * 2 + z1;
    for (int mu = 0; mu < 3; ++mu) {
      const double wcm = dsigma[mu] * 0.25 * c_sign[c] * f;
      const int ia = crev * 3 + mu, ib = c * 3 + mu;
      if (z1 == z) {
        // B X(z2) A : P = X(z2) A, then B P
        double2 p = make_double2(0.0, 0.0);
        for (int l = 0; l < NL; ++l) p = cfma(p, sX[z2][i][l], sA[ia][l][j]);
        __syncthreads();
        sP[i][j] = p;
        __syncthreads();
        double2 q = make_double2(0.0, 0.0);
        for (int k = 0; k < NL; ++k) q = cfma(q, sB[ib][i][k], sP[k][j]);
        g.x += wcm * q.x;
        g.y += wcm * q.y;
      }
      if (z2 == z) {
        // B^T X(z1) A^T : P = X(z1) A^T, then B^T P
        double2 p = make_double2(0.0, 0.0);
        for (int l = 0; l < NL; ++l) p = cfma(p, sX[z1][i][l], sA[ia][j][l]);
        __syncthreads();
        sP[i][j] = p;
        __syncthreads();
        double2 q = make_double2(0.0, 0.0);
        for (int k = 0; k < NL; ++k) q = cfma(q, sB[ib][k][i], sP[k][j]);
        g.x += wcm * q.x;
        g.y += wcm * q.y;
      }
    }
  }
  X[j] = g;
  X[NL + j] = make_double2((a == 0 && i == j) ? 1.0 : 0.0, 0.0);
}

void launch_adjoint_rhs(const JobDesc* jobs, int njobs, int npad_max, const int32_t* liz_atom,
                        const double2* tau_plus, const double2* tau_minus, const int32_t* species, int n_species,
                        const double2* J, const double* dsigma, double volume, double2* x, hipStream_t s) {
  dim3 grid(npad_max / NL, njobs);
  adjoint_rhs_kernel<<<grid, 256, 0, s>>>(jobs, liz_atom, tau_plus, tau_minus, species, n_species, J, dsigma, volume,
                                          x);
}

// dL/dt_{b,l}(z) = sum_{m in shell l} sum_j V[(b,L)][j] U[(b,L)][j], U = cols 0..15, V = cols 16..31
__global__ __launch_bounds__(256) void adjoint_contract_kernel(const JobDesc* jobs, const int32_t* liz_atom,
                                                               const double* phase, double2 kp, const double2* x,
                                                               double* dphase) {
  const JobDesc jd = jobs[blockIdx.y];
  const int b = blockIdx.x;
  if (b >= jd.nl) return;  // uniform
  const int t = threadIdx.x, L = t >> 4, j = t & 15;
  const double2* row = x + jd.x_off + (int64_t)(b * NL + L) * NRHS_MAX;
  double2 p = cmul(row[NL + j], row[j]);
  // sum over j (16 lanes of the same L)
#pragma unroll
  for (int o = 1; o < 16; o <<= 1) {
    p.x += __shfl_xor(p.x, o);
    p.y += __shfl_xor(p.y, o);
  }
  __shared__ double2 s_row[NL];
  if (j == 0) s_row[L] = p;
  __syncthreads();
  if (t < 4) {
    const int l = t;
    double2 sum = make_double2(0.0, 0.0);
    for (int m = 0; m < 2 * l + 1; ++m) sum = cadd(sum, s_row[l * l + m]);
    const int site = liz_atom[jd.liz_off + b];
    const double d = phase[(int64_t)site * 4 + l];
    double s2, c2;
    sincos(2.0 * d, &s2, &c2);
    double2 dt = cmul(make_double2(-c2, -s2), cinv(kp));  // -e^{2 i d} / kappa+
    if (jd.energy == 1) dt.y = -dt.y;
    const double2 contrib = cmul(sum, dt);
    atomicAdd(dphase + (int64_t)site * 4 + l, contrib.x);
  }
}

void launch_adjoint_contract(const JobDesc* jobs, int njobs, int npad_max, const int32_t* liz_atom,
                             const double* phase, double2 kappa_plus, const double2* x, double* dphase,
                             hipStream_t s) {
  dim3 grid(npad_max / NL, njobs);
  adjoint_contract_kernel<<<grid, 256, 0, s>>>(jobs, liz_atom, phase, kappa_plus, x, dphase);
}

}  // namespace lsms
