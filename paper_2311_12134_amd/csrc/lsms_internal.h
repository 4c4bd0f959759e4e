// Internal declarations shared by the library's host and device translation units.
// Nothing here is part of the C ABI (see include/lsms_kkr.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lsms {

constexpr int NL = 16;        // channels per site, lmax = 3
constexpr int NL3 = 49;       // channels of the Gaunt-coupled harmonics, l'' <= 6
constexpr int NB = 64;        // outer panel width of the blocked LU
constexpr int PAD = 64;       // matrices are padded (identity) to a multiple of this
constexpr int MAX_GAUNT = 1024;

// Complex helpers (interleaved re, im) -------------------------------------------
struct cd { double x, y; };

__host__ __device__ inline double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__host__ __device__ inline double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__host__ __device__ inline double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
// a - b*c
__host__ __device__ inline double2 cfms(double2 a, double2 b, double2 c) {
  return make_double2(a.x - (b.x * c.x - b.y * c.y), a.y - (b.x * c.y + b.y * c.x));
}
// a + b*c
__host__ __device__ inline double2 cfma(double2 a, double2 b, double2 c) {
  return make_double2(a.x + (b.x * c.x - b.y * c.y), a.y + (b.x * c.y + b.y * c.x));
}
// the same in single precision (split-mode panel updates in the storage precision)
__host__ __device__ inline float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__host__ __device__ inline float2 cfms(float2 a, float2 b, float2 c) {
  return make_float2(a.x - (b.x * c.x - b.y * c.y), a.y - (b.x * c.y + b.y * c.x));
}
__host__ __device__ inline double2 cinv(double2 a) {
  // Smith-style scaling avoids overflow for large components.
  if (fabs(a.x) >= fabs(a.y)) {
    double r = a.y / a.x, d = a.x + a.y * r;
    return make_double2(1.0 / d, -r / d);
  } else {
    double r = a.x / a.y, d = a.y + a.x * r;
    return make_double2(r / d, -1.0 / d);
  }
}

// Storage conversions: the working matrix is complex double (FP64 mode) or
// complex float (split mode); arithmetic in the panel and solves is FP64.
__device__ inline double2 ld2(const double2* p) { return *p; }
__device__ inline double2 ld2(const float2* p) {
  float2 v = *p;
  return make_double2((double)v.x, (double)v.y);
}
__device__ inline void st2(double2* p, double2 v) { *p = v; }
__device__ inline void st2(float2* p, double2 v) { *p = make_float2((float)v.x, (float)v.y); }
// LDS element type matching a storage type: FP32 factors stay FP32 in LDS (half the
// footprint, so two workgroups share a CU).
template <typename T> struct LdsOf { typedef double2 type; };
template <> struct LdsOf<float2> { typedef float2 type; };

// One (atom, energy) system.
struct JobDesc {
  int64_t a_off;    // working matrix (npad x npad, row-major, ld = npad), in complex elements
  int64_t v_off;    // packed FP64 structure-constant blocks (split mode), in complex elements; -1 if absent
  int64_t x_off;    // solution / right-hand-side block (npad x NRHS_MAX complex double)
  int64_t r_off;    // residual / correction block (split mode), same shape; -1 if absent
  int64_t piv_off;  // pivots (npad int32)
  int64_t liz_off;  // first LIZ member of this atom
  int32_t atom;     // atom index
  int32_t energy;   // 0: z+ ; 1: z-
  int32_t nl;       // LIZ members
  int32_t n;        // NL * nl
  int32_t npad;     // n rounded up to PAD
  int32_t info;     // host-side scratch
  int32_t ld;       // leading dimension if not npad (0: npad); set for the tall-panel sub-problems
  int32_t pad_;
};

constexpr int NRHS_MAX = 32;  // columns of the solution block (16 forward, 32 adjoint)

// Split mode keeps, per pair of LIZ members a < b, the FP64 Gaunt contraction
// v^{ab}_{LL'} = sum_{L''} C_{L L' L''} (-4 pi i kappa) i^{l''} h_{l''}(kappa |R|) Y_{L''}(R^), R = p_a - p_b,
// so that g^{ab} = i^l v^{ab} i^{-l'}.  v is symmetric in (L, L') and is stored as its upper
// triangle, row by row: VBLOCK complex entries per pair, the pair numbered like the upper
// triangle of the member grid (pair_index).  For the reversed pair v^{ba} = (-1)^{l + l'} v^{ab}.
constexpr int VBLOCK = NL * (NL + 1) / 2;
__host__ __device__ inline int vblock_index(int L, int Lp) { return L * NL - L * (L - 1) / 2 + (Lp - L); }  // L <= Lp
// pair a <= b of an nb x nb grid, numbered row by row
__host__ __device__ inline int64_t pair_index(int a, int b, int nb) {
  return (int64_t)a * nb - (int64_t)a * (a - 1) / 2 + (b - a);
}

// The NB interchanges of one panel permute at most 2 NB rows.  The panel kernel stores
// that permutation once per panel as (destination row, source row) pairs so that the
// trailing update and the solves apply it as one parallel gather instead of NB
// dependent swaps.  Per job, after the npad pivots: (npad / NB) lists of PERM_STRIDE ints
// laid out as [count, unused, dst[PERM_MAX], src[PERM_MAX]].
constexpr int PERM_MAX = 2 * NB;
constexpr int PERM_STRIDE = 2 + 2 * PERM_MAX;
__host__ __device__ inline int64_t piv_ints(int npad) { return (int64_t)npad + (int64_t)(npad / NB) * PERM_STRIDE; }
__host__ __device__ inline int64_t perm_off(int npad, int k) { return (int64_t)npad + (int64_t)(k / NB) * PERM_STRIDE; }

struct GauntTable {
  // CSR over the 256 (L, L') pairs: terms [start[p], start[p+1]) hold (L'', C).
  int32_t start[NL * NL + 1];
  int32_t l3[MAX_GAUNT];
  double coef[MAX_GAUNT];
};

// ---- launchers (defined in the .hip files) ---------------------------------------
hipError_t upload_gaunt(const GauntTable& g);

// t_l(z+-) for every atom: tpm[atom][e][l] (complex), e = 0 (+), 1 (-).
void launch_tmatrix(const double* phase, int n_atoms, double2 kappa_plus, double2* tpm, double2* spm,
                    hipStream_t s);

// M = 1 - T g over each job's LIZ (padded with identity), written to the working
// matrix (double2 or float2); spm != nullptr: the symmetric form 1 - S g S, S = T^{1/2}.
// Split mode also writes the packed FP64 contractions of every pair (vtab, at v_off).
void launch_assemble_f64(const JobDesc* jobs, int njobs, int npad_max, const double* liz_pos,
                         const int32_t* liz_atom, const double2* tpm, double2 kp, double2 km, double2* work,
                         const double2* spm, hipStream_t s);
void launch_assemble_split(const JobDesc* jobs, int njobs, int npad_max, const double* liz_pos,
                           const int32_t* liz_atom, const double2* tpm, double2 kp, double2 km, float2* work,
                           double2* vtab, const double2* spm, hipStream_t s);
// Residual r = B - M X of the split-mode refinement from the packed contractions (vtab) and
// the t-matrices (spm != nullptr: the symmetric form); norms[job][0..4] as in the refinement
// (first: also ||M||_inf); jobs with done[job] set are skipped.
void launch_residual(const JobDesc* jobs, int njobs, int npad_max, const double2* vtab, const int32_t* liz_atom,
                     const double2* tpm, const double2* spm, const double2* x, double2* r, double* norms,
                     const int32_t* done, int first, hipStream_t s);
// B = E0 t_centre in the solution block (first NL columns), zero elsewhere.
void launch_init_rhs(const JobDesc* jobs, int njobs, int npad_max, const int32_t* liz_atom, const double2* tpm,
                     double2* x, hipStream_t s);

// Optional timing of the trailing-update launches (the dominant kernel): before()/after()
// bracket every launch; n_true holds the unpadded size of each job of the wave (host),
// from which the algorithmic flops of the launch (8 m^2 NB per job, m = n - k - NB) follow.
struct GemmProfiler {
  const int* n_true = nullptr;
  virtual void before(hipStream_t s) = 0;
  // kind 0: narrow update of a panel's columns within its group (K < G NB); 1: wide update
  // (K = G NB, G panels per group)
  virtual void after(hipStream_t s, double alg_flops, double alg_bytes, int kind) = 0;
  virtual ~GemmProfiler() {}
};

// Trailing update A22 -= L21 U12: rows [r_begin, npad) x cols [c_begin, c_end or npad),
// K = kd columns of L from column k; rows x cols is the extent over the largest job.
// The FP32 update comes in several tilings (variant 0 .. gemm_f32_variants() - 1).
void launch_gemm_f64(const JobDesc* jobs, int njobs, int rows, int cols, int k, int kd, int r_begin, int c_begin,
                     int c_end, double2* work, hipStream_t s);
// The FP64 update's tilings (gemm64.hip): variant 0 .. gemm_f64_variants() - 1, 0 = the plain kernel above.
int gemm_f64_variants();
void launch_gemm_f64_variant(int variant, const JobDesc* jobs, int njobs, int rows, int cols, int k, int kd,
                             int r_begin, int c_begin, int c_end, double2* work, hipStream_t s);
// Split-mode panels of at most PANEL_SMALL_ROWS rows (the default; autotuned or set per
// context up to PANEL_SMALL_MAX) use 256-thread workgroups with 8-wide leaves.
constexpr int PANEL_SMALL_ROWS = 3 * 256;
constexpr int PANEL_SMALL_MAX = 3 * 256;
// Panels per group of the blocked LU: 2 .. GROUP_MAX.
constexpr int GROUP_MAX = 4;
// Kernel choices of one LU: the panels per group (the big trailing update has K = group NB),
// the tilings of the wide (K = group NB) and narrow (a panel's columns within its group,
// K < group NB) trailing updates, and the height up to which split-mode panels take the
// small-workgroup variant.
struct Tiling {
  int wide = 0;
  int narrow = 0;
  int panel_small_rows = PANEL_SMALL_ROWS;
  int group = 2;
};
// The split-mode panel at k = 0 in one of its two variants (autotuner; lu.hip).
void launch_panel_f32_variant(int variant, const JobDesc* jobs, int njobs, int rows, float2* work, int32_t* piv,
                              int32_t* info, hipStream_t s);
// Autotuner (tune.hip): precision 0 FP64, 1 split; kind 1 wide (K = group NB), 0 narrow
// (64 columns, K = (group - 1) NB).  ms[variant] gets the best of three launches, *best the
// fastest; panel_autotune times the two split-mode panel variants at one height (ms[2]).
// Return 0 or -1 (allocation or launch failure).
int update_autotune(int precision, int kind, int npad, int batch, int group, hipStream_t s, float* ms, int* best);
int panel_autotune(int rows, int batch, hipStream_t s, float* ms);
// Peak-rate probes (probe.hip); what as in lsms_peak_probe.  Returns 0 or -1.
int peak_probe(int what, int cu_count, hipStream_t s, double* value);
int gemm_f32_variants();
// All FP32 tilings: those of gemm.hip and the persistent forms (gemm_persist.hip).
int gemm_f32_variants_all();
void launch_gemm_f32_any(int variant, const JobDesc* jobs, int njobs, int rows, int cols, int k, int kd, int r_begin,
                         int c_begin, int c_end, float2* work, hipStream_t s);
void launch_gemm_f32(int variant, const JobDesc* jobs, int njobs, int rows, int cols, int k, int kd, int r_begin,
                     int c_begin, int c_end, float2* work, hipStream_t s);
void launch_gemm_f32_lower(const JobDesc* jobs, int njobs, int rows, int k, int kd, int rc_begin, float2* work,
                           hipStream_t s);

// Blocked LU with partial pivoting of every job's working matrix.
// Panels taller than 2 * chunk rows are factored with tournament pivoting (lu.hip);
// they need device scratch laid out for the wave's job count and padded size.
struct TallScratch {
  int chunk = 0;         // rows per tournament chunk (64 .. 2048, a multiple of 64)
  void* base = nullptr;  // tall_scratch_bytes(njobs, npad_max, chunk) bytes, or nullptr if none needed
  int njobs = 0, npad_max = 0;
};
size_t tall_scratch_bytes(int njobs, int npad_max, int chunk);

// Optional second stream for the look-ahead panel (lu.hip); nullptr: one stream.
struct SideStream {
  hipStream_t stream = nullptr;
  hipEvent_t update_done = nullptr;  // the next panel's columns are updated
  hipEvent_t panel_done = nullptr;   // that panel is factored
};

void lu_factor_f64(const JobDesc* jobs, int njobs, int npad_max, double2* work, int32_t* piv, int32_t* info,
                   hipStream_t s, GemmProfiler* prof, Tiling tiling, const TallScratch& tall,
                   const SideStream* side = nullptr);
void lu_factor_f32(const JobDesc* jobs, int njobs, int npad_max, float2* work, int32_t* piv, int32_t* info,
                   hipStream_t s, GemmProfiler* prof, Tiling tiling, const TallScratch& tall,
                   const SideStream* side = nullptr);
// Symmetric factorization S = L D L^T of complex-symmetric systems (no pivoting), stored as
// an LU with U = D L^T so the LU solves apply.  Panels taller than tall_rows take the
// diagonal-block path, which needs ldlt_scratch_bytes(njobs) bytes of device scratch.
size_t ldlt_scratch_bytes(int njobs);
void ldlt_factor_f32(const JobDesc* jobs, int njobs, int npad_max, float2* work, int32_t* piv, int32_t* info,
                     hipStream_t s, GemmProfiler* prof, int gemm_variant, int tall_rows, void* scratch);
// Solve with the factors: trans = 0 solves M X = B, trans = 1 solves M^T X = B (in place on X);
// group = the panels per group the factorization used.
void lu_solve_f64(const JobDesc* jobs, int njobs, int npad_max, const double2* work, const int32_t* piv,
                  double2* x, int64_t x_col_off, int nrhs, int trans, int group, hipStream_t s);
void lu_solve_f32(const JobDesc* jobs, int njobs, int npad_max, const float2* work, const int32_t* piv,
                  double2* x, int64_t x_col_off, int nrhs, int trans, int group, hipStream_t s);
// The split-mode refinement's solves (16 columns) in FP32 on the FP32 copy of the right-hand
// side in columns 16 .. 23 of each solution row (launch_x32 fills and drains it); jobs
// flagged in skip[] (may be null) are left alone.
void lu_solve_f32_single(const JobDesc* jobs, int njobs, int npad_max, const float2* work, const int32_t* piv,
                         double2* x, const int32_t* skip, int group, hipStream_t s);
// mode 0: FP32 copy <- src columns 0 .. 15 (rounded); 1: x columns 0 .. 15 <- the copy;
// 2: x columns 0 .. 15 += the copy (src used by mode 0 only; jobs flagged in done skipped)
void launch_x32(const JobDesc* jobs, int njobs, int npad_max, int mode, const double2* src, double2* x,
                const int32_t* done, hipStream_t s);

// Split-mode refinement helpers.
void launch_residual(const JobDesc* jobs, int njobs, int npad_max, const double2* m64, const double2* x,
                     double2* r, double* norms, hipStream_t s);
void launch_refine_update(const JobDesc* jobs, int njobs, double2* x, const double2* d, double* norms,
                          double tol, int32_t* done, hipStream_t s);
// Copy tau^{a0} (first n rows, NL columns) out of each job's solution block.
// mirror: only z+ jobs were solved; also write the z- blocks and status from them.
void launch_copy_tau(const JobDesc* jobs, int njobs, int npad_max, const double2* x, double2* tau_plus,
                     double2* tau_minus, bool mirror, const double2* spm, const int32_t* liz_atom, hipStream_t s);
void launch_write_status(const JobDesc* jobs, int njobs, const int32_t* job_info, const double* norms,
                         int32_t* info, double* berr, bool mirror, hipStream_t s);
void launch_check_inputs(const JobDesc* jobs, int njobs, const double* liz_pos, const int32_t* liz_atom,
                         const double* phase, int32_t* job_info, hipStream_t s);

// Kubo-Greenwood sums: diagonal (per atom [4][3]) or full tensor (per atom [4][3][3]).
void launch_kubo_trace(int n_atoms, const int64_t* liz_ptr_dev, const int32_t* liz_atom, const double2* tau_plus,
                       const double2* tau_minus, const int32_t* species, int n_species, const double2* J,
                       double2* per_atom, bool tensor, hipStream_t s);
// allocation-free Kubo sum: fixed per-device scratch of per-atom partial sums (kubo.hip)
constexpr int NOALLOC_MAX_ATOMS = 32768;
hipError_t noalloc_scratch_init(int device);  // once per device, at context creation
double2* noalloc_scratch(int device);         // its device address (nullptr before init)
void launch_kubo_reduce(int n_atoms, const double2* per_atom, double volume, double* sigma, double2* sigma_tilde,
                        bool tensor, hipStream_t s);

// Adjoint.
void launch_adjoint_rhs(const JobDesc* jobs, int njobs, int npad_max, const int32_t* liz_atom,
                        const double2* tau_plus, const double2* tau_minus, const int32_t* species, int n_species,
                        const double2* J, const double* dsigma, double volume, double2* x, hipStream_t s);
void launch_adjoint_contract(const JobDesc* jobs, int njobs, int npad_max, const int32_t* liz_atom,
                             const double* phase, double2 kappa_plus, const double2* x, double* dphase,
                             hipStream_t s);
void launch_zero(double* p, int64_t n, hipStream_t s);

}  // namespace lsms
