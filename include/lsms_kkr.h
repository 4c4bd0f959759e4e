/*
 * lsms_kkr.h -- C ABI of the MI355X (gfx950) library for the hot path of
 * LSMS residual-resistivity calculations (Raghuraman, Eisenbach, Widom,
 * Wang, "First principles residual resistivity using locally
 * self-consistent multiple scattering method", arXiv:2311.12134).
 *
 * For every atom m the library
 *   1. builds the local interaction zone (LIZ) of m           (Sec. II.A, Fig. 1),
 *   2. assembles M = 1 - t g over that LIZ at z = eF +- i eta  (Eq. (3)-(4), Eq. (7)),
 *      g = free-electron structure constants (spherical Hankel functions
 *      times Gaunt coefficients times real spherical harmonics),
 *   3. factors M (complex LU with partial pivoting; panels of more than 4096 rows by
 *      tournament pivoting; optionally the symmetric form by L D L^T, see
 *      LSMS_TUNE_SYMMETRIC) and solves for the tau blocks tau^{a0} linking every LIZ
 *      member a to the centre (Eq. (3), Eq. (10)),
 *   4. contracts tau with current matrix elements into the Kubo-Greenwood
 *      sums of Eq. (10) and combines the four energy pairs with Eq. (7).
 *
 * Conventions shared by every call:
 *   - Rydberg atomic units (hbar = 1, 2 m_e = 1): kappa = sqrt(z), bohr, Ry.
 *   - lmax = 3: 16 angular channels, L = l*l + l + m, real spherical harmonics
 *     without the Condon-Shortley phase.
 *   - Complex numbers are interleaved (re, im) pairs of double (the layout of
 *     C99 double _Complex and torch.complex128).
 *   - t_l(z+) = -sin(delta_l) exp(i delta_l) / kappa+, t(z-) = conj(t(z+)),
 *     kappa+ = principal sqrt(z+), kappa- = -conj(kappa+).
 *   - Energy pairs ("combos") are ordered (z1, z2) = (+,+), (+,-), (-,+), (-,-);
 *     directions x, y, z.
 *   - "host" pointers are ordinary CPU memory; "device" pointers are HIP
 *     device memory of the context's GPU.  The caller owns every array it
 *     passes; the library never frees or keeps a caller pointer beyond the
 *     completion of the work it enqueued.
 *   - Every call returns an lsms_status.  On failure lsms_last_error() gives a
 *     thread-local message; no C++ exception crosses this boundary.
 *   - Device work is enqueued on the caller's HIP stream (NULL = the null
 *     stream) and is asynchronous unless stated otherwise; argument errors are
 *     detected synchronously, before anything is enqueued.
 */
#ifndef LSMS_KKR_H
#define LSMS_KKR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LSMS_LMAX 3
#define LSMS_NL 16        /* (LSMS_LMAX + 1)^2 channels per site */
#define LSMS_MAX_LIZ 1024 /* largest LIZ (members) a single solve accepts (n = 16384) */

typedef enum {
  LSMS_OK = 0,
  LSMS_E_ARG = -1,      /* invalid argument (null pointer, size, NaN, lmax != 3, ...) */
  LSMS_E_CAPACITY = -2, /* caller-provided capacity too small; *needed tells the size */
  LSMS_E_DEVICE = -3,   /* HIP runtime error */
  LSMS_E_NOMEM = -4,    /* workspace limit too small for the request */
  LSMS_E_STATE = -5     /* object used in the wrong state (e.g. stale factors) */
} lsms_status;

typedef enum {
  LSMS_FP64 = 0,  /* whole factorization and solve in FP64 */
  LSMS_SPLIT = 1  /* FP32 LU updates, FP64 pivot selection, residuals, refinement */
} lsms_precision;

/* Per-job status codes written to info[] by lsms_tau_solve. */
#define LSMS_INFO_OK 0
/* k > 0 : exact zero pivot met at column k (1-based); tau of that job is not valid */
#define LSMS_INFO_NOCONV (-1)   /* split mode: refinement did not reach refine_tol */
#define LSMS_INFO_BADINPUT (-2) /* non-finite phase shift or position in this LIZ */

typedef struct lsms_ctx lsms_ctx;
typedef struct lsms_factors lsms_factors;

/* Message of the last failing call on this thread ("" if none). */
const char* lsms_last_error(void);

/*
 * Create a context on HIP device `hip_device`.  `lmax` must be 3.
 * `workspace_limit` bounds the device memory the library may hold for
 * factorizations (bytes; 0 = 60% of the device's free memory).  The Gaunt
 * table (integrals of three real spherical harmonics) is built here on the
 * host and uploaded once.
 */
int lsms_create(int hip_device, int lmax, size_t workspace_limit, lsms_ctx** out);

/* Release the context and everything it owns (factors handles must be freed first). */
int lsms_destroy(lsms_ctx* ctx);

/*
 * LIZ construction (Sec. II.A, Fig. 1; the inner sum of Eq. (10) runs over
 * the LIZ of m).  Host-only, synchronous; ctx is not used (may be NULL).
 *   pos      host [n_atoms][3]  atom positions (bohr)
 *   cell     host [3][3]        lattice vectors as rows, or NULL for an open cluster
 *   r_liz    LIZ radius (bohr, > 0); a member is any periodic image R_j + T of
 *            any atom j with |R_j + T - R_m| < r_liz (strict)
 *   capacity number of members the output arrays can hold
 *   liz_ptr  host [n_atoms + 1]      CSR offsets (always written when capacity suffices)
 *   liz_atom host [capacity]         atom index of each member
 *   liz_pos  host [capacity][3]      displacement (R_j + T) - R_m of each member
 *   needed   host [1]                total number of members (always written)
 * Order inside each LIZ: the centre first, then by increasing distance, ties
 * by the displacement's x, y, z (all compared after rounding to 1e-9).
 * Returns LSMS_E_CAPACITY (with *needed) when capacity is too small,
 * LSMS_E_ARG for coincident sites (distance < 1e-8 bohr), non-finite input,
 * a LIZ larger than LSMS_MAX_LIZ or r_liz <= 0.
 */
int lsms_build_liz(lsms_ctx* ctx, int32_t n_atoms, const double* pos, const double* cell, double r_liz,
                   int64_t capacity, int64_t* liz_ptr, int32_t* liz_atom, double* liz_pos, int64_t* needed);

/*
 * As lsms_build_liz, for the listed centre atoms only: every other atom gets an empty
 * LIZ (liz_ptr[a + 1] == liz_ptr[a]), which lsms_tau_solve and the Kubo sums skip.
 * The members of a centre's LIZ are the same as in the full build.
 *   n_centres >= 1, centres host [n_centres] in [0, n_atoms) (duplicates allowed)
 * Cost O(n_centres * n_atoms) instead of O(n_atoms^2).
 */
int lsms_build_liz_subset(lsms_ctx* ctx, int32_t n_atoms, const double* pos, const double* cell, double r_liz,
                          int32_t n_centres, const int32_t* centres, int64_t capacity, int64_t* liz_ptr,
                          int32_t* liz_atom, double* liz_pos, int64_t* needed);

/*
 * tau solve (Eq. (3)-(4)): for every atom m and both energies z+- = e_fermi +- i eta,
 * assemble M = 1 - T g over LIZ_m, factor it, and solve M X = E0 t_m so that
 * block a of X is tau^{a0}(z) (the row tau^{0a} equals its transpose, since
 * g_{LL'}(R) = g_{L'L}(-R) makes T^-1 - g complex symmetric).
 *   liz_ptr   host   [n_atoms + 1]       from lsms_build_liz
 *   liz_atom  device [liz_ptr[n]]        member atom indices
 *   liz_pos   device [liz_ptr[n]][3]     member displacements (bohr)
 *   phase     device [n_atoms][4]        phase shifts delta_l (radians), l = 0..3
 *   e_fermi, eta   eta > 0 (Ry)
 *   precision LSMS_FP64 or LSMS_SPLIT
 *   refine_tol, max_refine  split mode only: stop when the normwise backward
 *             error ||r||_inf / (||M||_inf ||X||_inf + ||B||_inf) <= refine_tol,
 *             or after max_refine corrections (then info = LSMS_INFO_NOCONV and
 *             the job is recomputed in FP64)
 *   tau_plus, tau_minus device [liz_ptr[n]][16][16] complex (out): tau^{a0}_{LL'}
 *   info      device [n_atoms][2] int32 (out), per atom and energy (0 = +, 1 = -):
 *             0; LSMS_INFO_NOCONV when the split-mode refinement missed refine_tol (or, in
 *             the symmetric form, met a zero pivot) and the system was recomputed by the
 *             FP64 LU (tau valid); k > 0 for an exact zero pivot of the FP64 LU (tau not
 *             valid); LSMS_INFO_BADINPUT
 *   berr      device [n_atoms][2] double (out): final backward error of the refined solution
 *             (split mode); -1 for a system recomputed by the FP64 LU (info = LSMS_INFO_NOCONV
 *             or a zero pivot after it), whose solution no split-mode residual describes;
 *             0 in FP64 mode
 *   keep      NULL, or receives a library-owned handle that keeps every LU factor
 *             alive for lsms_kubo_sigma_grad (free with lsms_factors_free)
 *   hip_stream  hipStream_t (NULL = null stream)
 * Device memory used: the jobs are processed in waves that fit the workspace
 * limit (all at once when keep != NULL, else LSMS_E_NOMEM).  Per system: the working
 * matrix (npad^2 complex, npad = n rounded up to 64; complex64 in split mode, complex128 in
 * FP64 mode), in split mode the FP64 Gaunt contractions of every pair of LIZ members that the
 * refinement's residual reads (2176 bytes per pair; no FP64 copy of M is kept), solution and
 * residual blocks (npad x 32 complex128 each) and the pivots.  Systems recomputed in FP64 take
 * the wave's matrix area once their FP32 factors are done with (a wave of one system borrows
 * a buffer for its FP64 matrix).
 * An atom whose LIZ is empty (liz_ptr[a + 1] == liz_ptr[a]) is skipped: no system is
 * solved for it and its info and berr are 0 (not allowed with keep).  This lets a
 * caller solve a subset of a structure's atoms with the structure's phase array.
 * Panels of more than 2 C rows (C = LSMS_TUNE_TSLU_CHUNK, default 2048, so LIZ of more
 * than 256 members) choose their pivot rows by tournament pivoting (see lsms_set_tuning).
 */
int lsms_tau_solve(lsms_ctx* ctx, int32_t n_atoms, const int64_t* liz_ptr, const int32_t* liz_atom,
                   const double* liz_pos, const double* phase, double e_fermi, double eta, int precision,
                   double refine_tol, int max_refine, void* tau_plus, void* tau_minus, int32_t* info,
                   double* berr, lsms_factors** keep, void* hip_stream);

/*
 * Kubo-Greenwood sum (Eq. (10)) and four-term combination (Eq. (7)):
 *   s_m[c][mu] = sum_{a in LIZ_m} Tr[ J^{m mu}(z2,z1) tau^{0a}(z1) J^{a mu}(z1,z2) tau^{a0}(z2) ]
 *   sigma~[c][mu] = -(1 / (pi * volume)) * sum_m s_m[c][mu]
 *   sigma[mu]     = 1/4 (sigma~[++] - sigma~[+-] - sigma~[-+] + sigma~[--])   (real part)
 * (Rydberg units make 4 m_e^2 / hbar^3 = 1; volume = N Omega, the supercell volume.)
 *   liz_ptr    host   [n_atoms + 1]
 *   liz_atom   device [liz_ptr[n]]
 *   tau_plus, tau_minus device [liz_ptr[n]][16][16] complex, as written by lsms_tau_solve
 *   species    device [n_atoms] int32 in [0, n_species)
 *   J          device [n_species][4][3][16][16] complex: J[s][c][mu] = J^{s mu}(zA, zB)
 *              for the energy pair (zA, zB) of combo c
 *   volume     > 0 (bohr^3)
 *   sigma      device [3] double (out)
 *   sigma_tilde device [4][3] complex (out)
 *   per_atom   device [n_atoms][4][3] complex (out) or NULL
 * The reduction over atoms has a fixed order (bitwise reproducible).  Atoms with an
 * empty LIZ contribute nothing.
 */
int lsms_kubo_sigma(lsms_ctx* ctx, int32_t n_atoms, const int64_t* liz_ptr, const int32_t* liz_atom,
                    const void* tau_plus, const void* tau_minus, const int32_t* species, int32_t n_species,
                    const void* J, double volume, double* sigma, void* sigma_tilde, void* per_atom,
                    void* hip_stream);

/*
 * Allocation-free variant of lsms_kubo_sigma, for callers that cannot allocate device or
 * pinned memory while they run (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc): the same sums, the same kernels and the same fixed reduction
 * order, so the outputs equal lsms_kubo_sigma's bitwise.  The call allocates nothing and
 * never waits for the device: no hipMalloc / hipFree / hipHostMalloc, no host staging.
 *   liz_ptr   DEVICE [n_atoms + 1] int64 CSR offsets (the host array of lsms_build_liz,
 *             copied to the device by the caller; read by the kernels, not validated on
 *             the host, so it must be consistent with liz_atom and the tau arrays)
 *   n_atoms   1 .. LSMS_NOALLOC_MAX_ATOMS, else LSMS_E_ARG
 *   other arguments as for lsms_kubo_sigma (per_atom may be NULL)
 * With per_atom == NULL the per-atom partial sums go to a fixed scratch array of the
 * library (LSMS_NOALLOC_MAX_ATOMS x 4 x 3 complex = 6 MiB per GPU, held from the first
 * lsms_create on that GPU until the process ends).  Every call on one GPU shares that
 * array and leaves its partial sums there; each call writes all n_atoms entries before it
 * reads them, so nothing needs clearing, but calls that overlap on one GPU (two streams,
 * two threads, two contexts) race on it and must be ordered by the caller.
 */
#define LSMS_NOALLOC_MAX_ATOMS 32768
int lsms_kubo_sigma_noalloc(lsms_ctx* ctx, int32_t n_atoms, const int64_t* liz_ptr, const int32_t* liz_atom,
                            const void* tau_plus, const void* tau_minus, const int32_t* species, int32_t n_species,
                            const void* J, double volume, double* sigma, void* sigma_tilde, void* per_atom,
                            void* hip_stream);

/*
 * Full conductivity tensor: Eq. (10) for every pair of Cartesian directions, with mu
 * on the centre atom's current J^{m mu}(z2,z1) and nu on the member's J^{n nu}(z1,z2),
 * then Eq. (7) for each (mu, nu):
 *   s_m[c][mu][nu] = sum_{a in LIZ_m} Tr[ J^{m mu}(z2,z1) tau^{0a}(z1) J^{a nu}(z1,z2) tau^{a0}(z2) ]
 *   sigma~[c][mu][nu] = -(1 / (pi * volume)) * sum_m s_m[c][mu][nu]
 *   sigma[mu][nu]     = 1/4 (sigma~[++] - sigma~[+-] - sigma~[-+] + sigma~[--])   (real part)
 * Arguments as for lsms_kubo_sigma, except the outputs:
 *   sigma       device [3][3] double (out), row mu, column nu
 *   sigma_tilde device [4][3][3] complex (out)
 *   per_atom    device [n_atoms][4][3][3] complex (out) or NULL
 * The diagonal equals lsms_kubo_sigma's sigma; the reduction order is fixed.
 */
int lsms_kubo_sigma_tensor(lsms_ctx* ctx, int32_t n_atoms, const int64_t* liz_ptr, const int32_t* liz_atom,
                           const void* tau_plus, const void* tau_minus, const int32_t* species, int32_t n_species,
                           const void* J, double volume, double* sigma, void* sigma_tilde, void* per_atom,
                           void* hip_stream);

/*
 * Adjoint of the whole path: gradient of L = sum_mu dsigma[mu] sigma_mu with
 * respect to every phase shift, d L / d phase[k][l].  Derived from Eq. (3)
 * (d tau = W dT W^T with W = (1 - T g)^-1) and Eq. (10): one transposed solve
 * M^T Y = [R, E0] per atom and energy with the factors kept by lsms_tau_solve,
 * then a contraction over each LIZ, then the chain rule
 * dt_l(z+)/d delta_l = -exp(2 i delta_l)/kappa+ (conjugate at z-), summed
 * over every LIZ image of site k.
 *   factors   handle from lsms_tau_solve(..., keep) with the same inputs
 *   phase, tau_plus, tau_minus, species, J, volume as in the forward calls
 *   dsigma    device [3] double: upstream gradient
 *   dphase    device [n_atoms][4] double (out, overwritten)
 */
int lsms_kubo_sigma_grad(lsms_ctx* ctx, const lsms_factors* factors, int32_t n_atoms, const int64_t* liz_ptr,
                         const int32_t* liz_atom, const double* phase, const void* tau_plus,
                         const void* tau_minus, const int32_t* species, int32_t n_species, const void* J,
                         double volume, const double* dsigma, double* dphase, void* hip_stream);

/* Free a factors handle (waits for outstanding work on the context's device). */
int lsms_factors_free(lsms_factors* factors);

/*
 * Diagnostic entry: factor caller-supplied matrices with the library's batched
 * LU (partial pivoting) and solve A X = B in place of B.
 *   batch     number of systems
 *   n         host [batch] sizes (1 .. 16 * LSMS_MAX_LIZ)
 *   A         host [batch] device pointers to row-major n x n complex matrices (read only)
 *   B         host [batch] device pointers to row-major n x nrhs complex right-hand sides (overwritten by X)
 *   nrhs      1 .. 16
 *   precision LSMS_FP64 (or LSMS_SPLIT: FP32 factors, no refinement)
 *   info      device [batch] int32 (out): 0, or k > 0 for an exact zero pivot at column k
 */
int lsms_batched_lu_solve(lsms_ctx* ctx, int32_t batch, const int32_t* n, void* const* A, void* const* B,
                          int32_t nrhs, int precision, int32_t* info, void* hip_stream);

/*
 * Measurement of the dominant kernel, the trailing-matrix update A22 -= L21 U12 of the
 * blocked LU (the matrix inverse of Eq. (3) dominates the cost, Sec. II.A).
 * lsms_set_profiling(ctx, 1) waits for the device, clears the statistics and makes every
 * later lsms_tau_solve record a pair of HIP events around each trailing-update launch on
 * the caller's stream (0 switches recording off).  lsms_kernel_stats waits for the
 * recorded events and returns, over the launches of the given kind, the summed launch
 * time (ms), the number of launches, their algorithmic flops and their algorithmic bytes.
 * kind 1 selects the wide updates (K = 64 G, the trailing matrix past a group of G panels,
 * LSMS_TUNE_GROUP_F32 / _F64), kind 0 the narrow updates of a panel's columns within its
 * group (K = 64, 128, .. 64 (G - 1)), -1 both.  A launch updates,
 * in every system, the unpadded block of m rows and c columns: 8 m c K flops (the
 * standard complex count; the split mode executes 3/4 of it on the matrix cores) and
 * es (m K + K c + 2 m c) bytes, es = 8 (split) or 16 (FP64).  All outputs are host
 * scalars; the call returns LSMS_E_ARG for a NULL pointer or an unknown kind.
 */
int lsms_set_profiling(lsms_ctx* ctx, int on);

/*
 * Tuning of the split-mode trailing update (the FP32 matrix-core part of the LU of Eq. (3)).
 * knob LSMS_TUNE_GEMM_F32 selects the tiling of the wide update, 0 .. LSMS_GEMM_F32_VARIANTS - 1,
 * or -1 for the autotuned choice or the library's default, 19 (0: 64 x 64 tiles; 1, 2: 64 x 64 pipelined through two LDS stages,
 * 2 with an XCD-aware workgroup order; 3 - 6: 128-row / 128-column tiles; 7: as 2 with the C
 * tile prefetched early; 8: as 2 with K chunks of 32; 9: as 2 on FP32 MFMA 32x32x2; 10: as 2 in a
 * persistent grid of resident workgroups that loops over the tiles; 11: as 10 with the C tile
 * prefetched early; 12, 13, 14: 128 x 64, 64 x 128 and 128 x 128 tiles of 8, 8 and 16 waves of
 * 32 x 32; 15, 16: 64 x 64 and 64 x 128 tiles with the K chunks prefetched two ahead; 17, 18:
 * the streaming persistent form, whose next tile's first K chunk is loaded during the current
 * tile's last one, without and with the C tile loaded early; 19: as 2 with each job's tiles
 * numbered in bands of eight tile rows, so one XCD's resident workgroups share few L21 and
 * U12 panels in its L2; 20: as 13 in bands of eight tile rows); every
 * tiling computes the same update (results may differ in FP32 rounding order only).  Host-side setting of the context, no device work; returns
 * LSMS_E_ARG for an unknown knob or value.  lsms_get_tuning reports the tiling in effect.
 */
#define LSMS_TUNE_GEMM_F32 0
#define LSMS_GEMM_F32_VARIANTS 21
/*
 * knob LSMS_TUNE_GRAPHS (0 or 1, default 0): with 1, lsms_tau_solve captures each wave's
 * factorization and first solve (a fixed sequence of a few hundred launches) into a HIP
 * graph on a stream of its own the first time a wave shape and buffer set occurs, and from
 * then on replays that graph on the caller's stream.  Results are bitwise those of the
 * eager launches.  Graphs are not used while profiling is on.
 */
#define LSMS_TUNE_GRAPHS 1
/*
 * knob LSMS_TUNE_CONJ_SYMMETRY (0 or 1, default 0): with 1, lsms_tau_solve factors and
 * solves only the z+ = eF + i eta systems and writes tau(z-) from them as
 * tau(z-)_{LL'} = (-1)^{l+l'} conj(tau(z+)_{LL'}), which holds exactly because
 * kappa- = -conj(kappa+) and t(z-) = conj t(z+) make the structure constants of Eq. (3)
 * at z- the parity-conjugate of those at z+ (Eq. (7) needs both energies).  Half the
 * LU work; info and berr of z- repeat those of z+.  Ignored when factors are kept for
 * the adjoint (lsms_kubo_sigma_grad needs both energies' factors).
 */
#define LSMS_TUNE_CONJ_SYMMETRY 2
/*
 * knob LSMS_TUNE_TSLU_CHUNK (a multiple of 64 in [64, 2048], default 2048): a panel of the
 * LU with more than 2 C rows is not factored by one workgroup but by tournament pivoting
 * (communication-avoiding LU): chunks of C rows each nominate 64 rows by partial
 * pivoting, one more partial-pivoting factorization of the nominees picks the panel's 64
 * pivot rows, and the rows below are L21 = A21 U11^-1.  C is raised where needed so that
 * the nominees fit one 4096-row block.  Smaller C exercises the path on smaller systems;
 * the result is a stable LU either way (tau agrees to rounding).
 */
#define LSMS_TUNE_TSLU_CHUNK 3
/*
 * knob LSMS_TUNE_LOOKAHEAD (0 or 1, default 0): with 1, lsms_tau_solve factors the first
 * panel of the next group on a second stream of the context (default priority) while the
 * rest of the current trailing update runs on the caller's stream; events order them and
 * the call's work is complete on the caller's stream when its last launch is.  Results
 * are bitwise those of 0.  Not used inside captured graphs (LSMS_TUNE_GRAPHS).
 */
#define LSMS_TUNE_LOOKAHEAD 4
/*
 * knob LSMS_TUNE_SYMMETRIC (0 or 1, default 0): with 1, split-mode lsms_tau_solve works on
 * the complex-symmetric form S = T^{1/2} M T^{-1/2} = 1 - T^{1/2} g T^{1/2} (g is symmetric by
 * reciprocity; T^{1/2} holds the principal square roots of the t_l, so no t is inverted):
 * S Y = T^{1/2} E0 is solved with an unpivoted L D L^T factorization in FP32 (half the
 * trailing-update work of the LU), refined in FP64 (residuals of S formed from the same FP64
 * pair contractions as in the LU path), and
 * tau^{a0} = t_a^{1/2} Y_a.  Systems whose refinement does not converge (e.g. large
 * element growth without pivoting) fall back to the FP64 LU with partial pivoting of S, as
 * in the LU path.  With no pivots to choose, each panel factors only its diagonal block
 * and forms L21 = A21 U11^-1 on the matrix cores.  Not used with kept factors (the LU path
 * runs).
 * Not the paper's LU: reported apart from the LU rate.
 */
#define LSMS_TUNE_SYMMETRIC 5
/*
 * knob LSMS_TUNE_PIPELINE (0 or 1, default 0): with 1 and a batch of two or more waves,
 * lsms_tau_solve alternates waves between the caller's stream and a second, non-blocking
 * stream of the context (default priority), each with half of the workspace, and issues
 * the next wave's assembly, factorization and first solve before the current wave's
 * refinement, so memory-bound refinement overlaps matrix-core factorization.  The call's
 * work is complete on the caller's stream when its last launch is (an event joins the
 * second stream).  When all systems share one padded size, every system goes through the
 * same kernels as with 0 and the results are bitwise those of 0; with uneven sizes the
 * waves group the systems differently, and since a wave's panel launches are shaped by its
 * largest system, a system may take a different panel variant (leaf width) and round
 * differently.  Not used with kept factors, the symmetric form, the look-ahead stream,
 * tournament panels (LIZ above 2 C rows) or profiling (lsms_set_profiling).  Off by
 * default: on the 4000-atom fcc alloy it measured within 0.3 % of one stream, since halving
 * the waves costs about what the overlap gains.
 */
#define LSMS_TUNE_PIPELINE 6
/*
 * knobs LSMS_TUNE_GEMM_F32_NARROW (split mode, 0 .. LSMS_GEMM_F32_VARIANTS - 1),
 * LSMS_TUNE_GEMM_F64 and LSMS_TUNE_GEMM_F64_NARROW (FP64 mode, 0 .. LSMS_GEMM_F64_VARIANTS - 1:
 * 0 the single-buffered 64 x 64 kernel; 1 64 x 64 with two LDS stages of K = 8 and the XCD
 * order; 2 32 x 64; 3 128 x 64; 4 64 x 128; 5 as 1 without the XCD order): the
 * tilings of the narrow (a panel's 64 columns within its group, K < 64 x group) and wide
 * (K = 64 x group) trailing updates.
 * knob LSMS_TUNE_PANEL_SMALL_ROWS (0 .. 768, default 768): split-mode panels of at most this
 * many rows run in 256-thread workgroups with 8-wide leaves (three jobs per compute unit),
 * taller ones in 512-thread workgroups with 16-wide leaves (one job per compute unit).
 * For every such choice (and LSMS_TUNE_GEMM_F32), -1 (the initial value) means: the
 * autotuned choice for the wave's padded size (lsms_autotune_kernel), else the library
 * default.  lsms_get_tuning reports the explicit setting (-1 if none), except for
 * LSMS_TUNE_GEMM_F32, where it reports the explicit setting or the default.
 */
#define LSMS_TUNE_GEMM_F32_NARROW 7
#define LSMS_TUNE_GEMM_F64 8
#define LSMS_TUNE_GEMM_F64_NARROW 9
#define LSMS_TUNE_PANEL_SMALL_ROWS 10
/* knobs LSMS_TUNE_GROUP_F32 (split mode) and LSMS_TUNE_GROUP_F64 (FP64 mode): panels per
 * group of the blocked LU, 2 .. 4, or -1 for the default (4).  The trailing matrix is updated
 * once per group with K = 64 x group (the wide update), the panels inside a group left-looking
 * (the narrow updates, K < 64 x group); larger groups move work from the wide update, whose
 * efficiency grows with K, to the narrow updates and the interchange kernel.  The autotuner
 * times the shapes of the group in effect when it runs. */
#define LSMS_TUNE_GROUP_F32 11
#define LSMS_TUNE_GROUP_F64 12
#define LSMS_GEMM_F64_VARIANTS 6
int lsms_set_tuning(lsms_ctx* ctx, int knob, int value);
int lsms_get_tuning(lsms_ctx* ctx, int knob, int* value);

/*
 * Autotuner over the kernels of the blocked LU (the inverse of Eq. (3), the dominant cost of
 * the method, Sec. II.A).  `what` selects the target:
 *   LSMS_AUTOTUNE_F32_WIDE / LSMS_AUTOTUNE_F64_WIDE: every tiling of the split-mode / FP64
 *     wide trailing update (K = 64 G over the trailing (npad - 64 G)^2 block of an LU of size
 *     npad, G the precision's panels per group in effect);
 *   LSMS_AUTOTUNE_F32_NARROW / LSMS_AUTOTUNE_F64_NARROW: every tiling of the narrow update
 *     of a group's last panel (K = 64 (G - 1) over (npad - 64 (G - 1)) rows x 64 columns);
 *   LSMS_AUTOTUNE_F32_PANEL: the two split-mode panel variants at the LSMS_PANEL_HEIGHTS
 *     heights 256, 512 and 768 (npad ignored; batch systems of the
 *     panel's 64 columns); ms[2 h + v] (ms_len >= 2 LSMS_PANEL_HEIGHTS) receives variant v
 *     (0: 256 threads, 8-wide leaves; 1: 512 threads) at height h, and the context's panel
 *     threshold becomes the height T (0: none) for which the small variant up to T and the
 *     large one above give the least summed time over the measured heights; *best receives T.
 * For the updates the fastest tiling (the library default unless another is faster by more
 * than 1 %, the spread of repeated timings) becomes the context's choice for every wave whose
 * largest padded size falls in npad's bucket (npad in (256 b, 256 (b + 1)]), *best receives
 * it and ms (NULL, or host [ms_len >= number of tilings]) the best-of-three launch time of
 * each tiling.  Each call allocates and frees a synthetic batch of `batch` systems (bounded
 * pseudo-random values) and is synchronous on hip_stream.  npad: a multiple of 64 in
 * (64 G, 16384]; batch in [1, 65535].  LSMS_E_ARG for bad sizes or target, LSMS_E_NOMEM if the
 * batch cannot be allocated.  Explicit lsms_set_tuning choices take precedence over these.
 */
#define LSMS_AUTOTUNE_F32_WIDE 0
#define LSMS_AUTOTUNE_F32_NARROW 1
#define LSMS_AUTOTUNE_F64_WIDE 2
#define LSMS_AUTOTUNE_F64_NARROW 3
#define LSMS_AUTOTUNE_F32_PANEL 4
#define LSMS_PANEL_HEIGHTS 3
#define LSMS_TUNE_BUCKETS 64
int lsms_autotune_kernel(lsms_ctx* ctx, int what, int npad, int batch, int* best, float* ms, int ms_len,
                         void* hip_stream);
/* The autotuned choices of a target: out host [LSMS_TUNE_BUCKETS], the tiling of each npad
 * bucket (-1: none); for LSMS_AUTOTUNE_F32_PANEL out[0] = the panel threshold (-1: none). */
int lsms_tuning_table(lsms_ctx* ctx, int what, int* out);
/*
 * Tuning cache: lsms_tuning_save writes every autotuned choice of the context to a text file
 * (first line "lsms-tune 1 <architecture>/<compute units>"), with the explicit panels-per-group
 * settings (LSMS_TUNE_GROUP_F32 / _F64) the tilings were timed with; lsms_tuning_load replaces
 * the context's autotuned choices by a file's and applies its group settings (LSMS_E_STATE if
 * it was written on another kind of
 * device, LSMS_E_ARG if it cannot be read or parsed; the context is unchanged on error).
 * lsms_create loads the file named by the environment variable LSMS_TUNE_CACHE when it
 * exists and was written on this kind of device.  Host-side, no device work.
 */
int lsms_tuning_save(lsms_ctx* ctx, const char* path);
int lsms_tuning_load(lsms_ctx* ctx, const char* path);

/*
 * Autotuner for the split-mode trailing update: times every tiling on the widest update
 * of an LU of size npad (K = 64 G over the trailing (npad - 64 G)^2 block, G the split
 * mode's panels per group) for a synthetic
 * batch of `batch` systems (bounded random FP32 values, allocated and freed by the call,
 * npad^2 * 8 * batch bytes), then makes the fastest (the default 19 unless another is more
 * than 1 % faster) the context's tiling (as
 * lsms_set_tuning would).  *best receives it; ms (NULL, or host [LSMS_GEMM_F32_VARIANTS])
 * the best-of-three launch time of each tiling.  npad: a multiple of 64 in (64 G, 4096];
 * batch in [1, 65535].  Synchronous on hip_stream; LSMS_E_ARG for bad sizes,
 * LSMS_E_NOMEM if the batch cannot be allocated.
 */
int lsms_autotune(lsms_ctx* ctx, int npad, int batch, int* best, float* ms, void* hip_stream);
int lsms_kernel_stats(lsms_ctx* ctx, int kind, double* total_ms, int64_t* launches, double* alg_flops,
                      double* alg_bytes);

/*
 * Peak-rate probes of the context's device, the ceilings against which the measured kernel
 * rates can be read: `what` 0 FP64 matrix cores (v_mfma_f64_16x16x4), 1 FP32 matrix cores
 * (16x16x4), 2 FP32 matrix cores (32x32x2), all in TFLOP/s of independent instruction
 * streams filling every compute unit; 3 FP64 vector FMA (TFLOP/s); 4 a 1 GiB device-to-device
 * copy (GB/s, bytes read plus written); 5 writes of 1 GiB; 6 reads of 1 GiB (GB/s).  *value
 * receives the best of three timed launches.  Allocates and frees its buffers (2 GiB for the
 * bandwidth probes); synchronous on hip_stream.
 * LSMS_E_ARG for an unknown probe, LSMS_E_DEVICE on a HIP error.
 */
int lsms_peak_probe(lsms_ctx* ctx, int what, double* value, void* hip_stream);

/*
 * Host-only query of the library's Gaunt table (Sec. II.A: g is built from these
 * integrals): out[(L * 16 + L') * 49 + L''] = integral of Y_L Y_L' Y_L'' over the unit
 * sphere for l, l' <= 3 and l'' <= 6 (real harmonics as above).  out is host
 * [16][16][49] double.  Needs no context and no GPU.
 */
int lsms_gaunt_table(double* out);

#ifdef __cplusplus
}
#endif

#endif /* LSMS_KKR_H */
