// Kubo-Greenwood sums of Eq. (10) and the four-term combination of Eq. (7).
//
// For atom m (one workgroup) and every LIZ member a, with X_a(z) = tau^{a0}(z) and the
// row tau^{0a}(z) = X_a(z)^T (reciprocity of the complex-symmetric T^-1 - g):
//   s_m[c][mu][nu] += Tr[ J^{m mu}(z2,z1) X_a(z1)^T J^{a nu}(z1,z2) X_a(z2) ]
//                  = sum_{ij} (J0_mu X1^T)_{ij} (Ja_nu X2)_{ji}
// Wavefront c of the workgroup takes combo c: per member it forms the six 16 x 16 x 16
// products P_mu = J0_mu X1^T and Q_nu = X2^T Ja_nu^T = (Ja_nu X2)^T on the FP64 matrix
// cores (both land in the same accumulator layout, so entry (i, j) of P_mu meets entry
// (j, i) of Ja_nu X2 in the same lane and register), then accumulates per lane either the
// diagonal mu = nu (three sums) or the full tensor (nine pairings), and reduces over the
// lanes at the end.  The sum over atoms then runs in a fixed order in a single
// workgroup, so sigma is reproducible.
#include <mutex>

#include "lsms_internal.h"
#include "strip_mma.h"

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
  __shared__ double2 sred[NQ];
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
  constexpr int NC = TENSOR ? 9 : 3;  // accumulators of this wavefront's combo
  const int lane = t & 63, wave = t >> 6;
  const int c = wave, z1 = combo_z1(c), z2 = combo_z2(c), crev = z2 * 2 + z1;
  double2 acc[NC];
#pragma unroll
  for (int q = 0; q < NC; ++q) acc[q] = make_double2(0.0, 0.0);
  int cur = -1;
  typedef StripMma<double2, 1, NL> Mma;
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
    Mma P[3], Q[3];
#pragma unroll
    for (int mu = 0; mu < 3; ++mu) {
      P[mu].zero();
      P[mu].run([&](int r, int k) { return sJ0[crev * 3 + mu][r][k]; }, [&](int k, int q) { return sX[z1][q][k]; },
                lane);
      Q[mu].zero();
      Q[mu].run([&](int r, int k) { return sX[z2][k][r]; }, [&](int k, int q) { return sJa[c * 3 + mu][q][k]; },
                lane);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
      for (int mu = 0; mu < 3; ++mu) {
        if (TENSOR) {
#pragma unroll
          for (int nu = 0; nu < 3; ++nu) acc[mu * 3 + nu] = cfma(acc[mu * 3 + nu], P[mu].value(0, r), Q[nu].value(0, r));
        } else {
          acc[mu] = cfma(acc[mu], P[mu].value(0, r), Q[mu].value(0, r));
        }
      }
  }
  // reduction of each wavefront's accumulators over its lanes (fixed order)
#pragma unroll
  for (int q = 0; q < NC; ++q) {
    double2 v = acc[q];
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
      v.x += __shfl_xor(v.x, o);
      v.y += __shfl_xor(v.y, o);
    }
    if (lane == 0) sred[c * NC + q] = v;
  }
  __syncthreads();
  if (t < NQ) per_atom[(int64_t)atom * NQ + t] = sred[t];
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

// ------------------------------------------------------------------------------------
// Fixed scratch of the allocation-free Kubo sum: the per-atom partial sums [atom][4][3]
// (complex) for up to NOALLOC_MAX_ATOMS atoms, one copy per GPU for the life of the
// process.  Host code never passes the array's name to a kernel (on the host it is only a
// stand-in for the symbol): noalloc_scratch_init looks up its device address once per
// device, with that device current, and everything else uses that address.
// ------------------------------------------------------------------------------------
static __device__ __align__(256) double2 scratch[(size_t)NOALLOC_MAX_ATOMS * 12];
static constexpr int kMaxDevices = 64;
static void* g_scratch_ptr[kMaxDevices] = {};
static std::mutex g_scratch_mu;

hipError_t noalloc_scratch_init(int device) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[device]) return hipSuccess;
  int prev = 0;
  hipError_t e = hipGetDevice(&prev);
  if (e != hipSuccess) return e;
  e = hipSetDevice(device);
  if (e != hipSuccess) return e;
  void* ptr = nullptr;
  e = hipGetSymbolAddress((void**)&ptr, HIP_SYMBOL(scratch));
  const hipError_t e2 = hipSetDevice(prev);
  if (e != hipSuccess) return e;
  if (e2 != hipSuccess) return e2;
  if (!ptr) return hipErrorInvalidSymbol;
  g_scratch_ptr[device] = ptr;
  return hipSuccess;
}

double2* noalloc_scratch(int device) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  return (double2*)g_scratch_ptr[device];
}

}  // namespace lsms
