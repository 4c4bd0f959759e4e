// Real spherical harmonics without the Condon-Shortley phase, channel L = l*l + l + m:
//   Y_l0 = N_l0 P_l(cos t),  Y_lm = sqrt(2) N_l|m| P_l^|m|(cos t) {cos m p (m > 0), sin |m| p (m < 0)},
//   N_lm = sqrt((2l+1)/(4 pi) (l-m)!/(l+m)!).
// Evaluated without angles: P_l^m(cos t) = sin^m t * Q_l^m(cos t) with Q a polynomial, and
// sin^m t (cos m p + i sin m p) = (x + i y)^m for a unit vector (x, y, z).
#pragma once

#include <math.h>

namespace lsms {

// Normalisation N_lm for 0 <= m <= l <= LM (host and device).
template <int LM>
__host__ __device__ inline double ylm_norm(int l, int m) {
  double r = (2.0 * l + 1.0) / (4.0 * M_PI);
  for (int q = l - m + 1; q <= l + m; ++q) r /= (double)q;  // (l-m)!/(l+m)!
  return sqrt(r);
}

// All (LM+1)^2 harmonics of the unit vector (x, y, z).
template <int LM>
__host__ __device__ inline void real_ylm_all(double x, double y, double z, double* Y) {
  double cm[LM + 1], sm[LM + 1];
  cm[0] = 1.0;
  sm[0] = 0.0;
  for (int m = 1; m <= LM; ++m) {
    cm[m] = cm[m - 1] * x - sm[m - 1] * y;
    sm[m] = cm[m - 1] * y + sm[m - 1] * x;
  }
  for (int m = 0; m <= LM; ++m) {
    double qmm = 1.0;
    for (int q = 1; q < 2 * m; q += 2) qmm *= q;  // (2m-1)!!
    double qlm2 = 0.0, qlm1 = qmm;
    for (int l = m; l <= LM; ++l) {
      double q;
      if (l == m) {
        q = qmm;
      } else if (l == m + 1) {
        q = z * (2 * m + 1) * qmm;
      } else {
        q = ((2 * l - 1) * z * qlm1 - (l + m - 1) * qlm2) / (double)(l - m);
      }
      if (l > m) {
        qlm2 = qlm1;
        qlm1 = q;
      }
      double nrm = ylm_norm<LM>(l, m);
      if (m == 0) {
        Y[l * l + l] = nrm * q;
      } else {
        Y[l * l + l + m] = M_SQRT2 * nrm * q * cm[m];
        Y[l * l + l - m] = M_SQRT2 * nrm * q * sm[m];
      }
    }
  }
}

}  // namespace lsms
