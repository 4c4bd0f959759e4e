// Host side of the library: C ABI entry points, argument checking, the Gaunt table,
// LIZ construction, and the scheduler that groups (atom, energy) systems into waves
// that fit the workspace and drives the HIP kernels over each wave.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <new>
#include <string>
#include <vector>

#include "../../include/lsms_kkr.h"
#include "lsms_internal.h"
#include "ylm.h"

using namespace lsms;

static_assert(LSMS_NOALLOC_MAX_ATOMS == lsms::NOALLOC_MAX_ATOMS, "fixed Kubo scratch size");


// ---------------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------------
static thread_local std::string g_err;

static int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

#define HIP_TRY(expr)                                                                                \
  do {                                                                                               \
    hipError_t e_ = (expr);                                                                          \
    if (e_ != hipSuccess) return fail(LSMS_E_DEVICE, "%s failed: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

extern "C" const char* lsms_last_error(void) { return g_err.c_str(); }

// ---------------------------------------------------------------------------------
// context
// ---------------------------------------------------------------------------------
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
};

// Records a pair of events around every trailing-update launch (see GemmProfiler).
struct EventProf : GemmProfiler {
  std::vector<hipEvent_t> pool;
  size_t used = 0;
  std::vector<double> flops, bytes;
  std::vector<int> kinds;
  hipEvent_t get() {
    if (used < pool.size()) return pool[used++];
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    pool.push_back(e);
    ++used;
    return e;
  }
  void before(hipStream_t s) override {
    hipEvent_t e = get();
    if (e) hipEventRecord(e, s);
  }
  void after(hipStream_t s, double f, double b, int kind) override {
    hipEvent_t e = get();
    if (e) hipEventRecord(e, s);
    flops.push_back(f);
    bytes.push_back(b);
    kinds.push_back(kind);
  }
  void reset() {
    used = 0;
    flops.clear();
    bytes.clear();
    kinds.clear();
  }
  ~EventProf() override {
    for (hipEvent_t e : pool) hipEventDestroy(e);
  }
};

// Autotuned kernel choices are kept per bucket of padded system size: bucket b holds
// npad in (256 b, 256 (b + 1)].
static inline int tune_bucket(int npad) { return std::min(std::max((npad - 1) / 256, 0), LSMS_TUNE_BUCKETS - 1); }

struct lsms_ctx {
  int device = 0;
  bool profiling = false;
  // explicit kernel choices (lsms_set_tuning); -1: the autotuned table, else the default
  int gemm_f32 = -1;  // tiling of the split-mode wide trailing update
  int gemm_f32_narrow = -1;
  int gemm_f64 = -1;
  int gemm_f64_narrow = -1;
  int panel_small_rows = -1;
  int group_f32 = -1;  // panels per group of the split-mode LU (-1: the default)
  int group_f64 = -1;  // the same for the FP64 LU
  // autotuned choices: tuned[precision][kind][bucket] (kind 0 narrow, 1 wide), -1 unset;
  // tuned_panel_rows: split-mode panels up to this height take the small variant
  int8_t tuned[2][2][LSMS_TUNE_BUCKETS];
  int tuned_panel_rows = -1;
  bool graphs = false;  // replay each wave's factorization + first solve from a HIP graph
  bool conj_symmetry = false;  // solve z+ only and derive z- (tau(z-) = P conj tau(z+) P)
  int tslu_chunk = 2048;       // rows per chunk of the tall-panel tournament
  DevBuf tall;                 // tall-panel scratch
  bool lookahead = false;      // factor the next group's first panel on a side stream
  bool symmetric = false;      // split mode: symmetric form and L D L^T instead of LU
  DevBuf ldlt;                 // scratch of its tall panels
  SideStream side;             // created on first use
  hipStream_t capture = nullptr;  // non-blocking stream the graphs are captured on
  std::map<std::vector<intptr_t>, hipGraphExec_t> graph_cache;
  EventProf prof;
  std::vector<int> n_true;
  size_t workspace_limit = 0;
  GauntTable gaunt;
  DevBuf work;      // wave workspace
  DevBuf small;     // per-call small arrays
  void* pinned = nullptr;
  size_t pinned_bytes = 0;
  int32_t* pinned_flag = nullptr;  // host-visible counter read back between refinement sweeps
  DevBuf fallback;                 // job list of the FP64 fallback
  DevBuf fallback_mat;             // its matrix when a wave's matrix area cannot hold one
  bool pipeline = false;           // alternate waves between two streams (see lsms_tau_solve)
  int cu_count = 1;                // compute units of the device (wave sizes are trimmed to multiples)
  hipStream_t pipe = nullptr;      // the second stream (non-blocking, default priority)
  hipEvent_t pipe_start = nullptr, pipe_end = nullptr;
};

// Library defaults where neither an explicit choice nor an autotuned one exists.
static constexpr int kDefaultF32Wide = 19, kDefaultF32Narrow = 7, kDefaultF64Wide = 1, kDefaultF64Narrow = 1;
static constexpr int kDefaultGroupF32 = 4, kDefaultGroupF64 = 4;

// Tiling of the split-mode trailing update in effect for a context (explicit or default).
static int gemm_f32_variant(const lsms_ctx* ctx) { return ctx->gemm_f32 >= 0 ? ctx->gemm_f32 : kDefaultF32Wide; }

// Kernel choices for a wave whose largest system has padded size npad: an explicit setting,
// else the autotuned choice of npad's bucket, else the default.
static Tiling pick_tiling(const lsms_ctx* c, int precision, int npad) {
  const int b = tune_bucket(npad);
  const int p = precision == LSMS_SPLIT ? 1 : 0;
  auto choose = [&](int expl, int kind, int def) {
    if (expl >= 0) return expl;
    return c->tuned[p][kind][b] >= 0 ? (int)c->tuned[p][kind][b] : def;
  };
  Tiling t;
  if (p == 1) {
    t.wide = choose(c->gemm_f32, 1, kDefaultF32Wide);
    t.narrow = choose(c->gemm_f32_narrow, 0, kDefaultF32Narrow);
  } else {
    t.wide = choose(c->gemm_f64, 1, kDefaultF64Wide);
    t.narrow = choose(c->gemm_f64_narrow, 0, kDefaultF64Narrow);
  }
  t.panel_small_rows = c->panel_small_rows >= 0 ? c->panel_small_rows
                       : c->tuned_panel_rows >= 0 ? c->tuned_panel_rows
                                                  : PANEL_SMALL_ROWS;
  t.group = p == 1 ? (c->group_f32 > 0 ? c->group_f32 : kDefaultGroupF32)
                   : (c->group_f64 > 0 ? c->group_f64 : kDefaultGroupF64);
  return t;
}

struct lsms_factors {
  lsms_ctx* ctx = nullptr;
  int precision = 0;
  int n_atoms = 0;
  std::vector<JobDesc> jobs;
  int npad_max = 0;
  void* work = nullptr;  // factors, pivots, solution blocks (device)
  size_t work_bytes = 0;
  JobDesc* jobs_dev = nullptr;
  int64_t x_base = 0, piv_base = 0;  // byte offsets inside work (matrices start at 0)
  double2 kp{0, 0}, km{0, 0};
  const int32_t* liz_atom = nullptr;     // the forward call's arrays, for a consistency check
  int64_t total_members = 0;
  int group = 2;  // panels per group of the factorization (the solves must match)
};

static int ensure_dev(DevBuf& b, size_t bytes, hipStream_t s) {
  if (b.bytes >= bytes) return LSMS_OK;
  if (b.p) {
    HIP_TRY(hipStreamSynchronize(s));
    HIP_TRY(hipFree(b.p));
    b.p = nullptr;
    b.bytes = 0;
  }
  hipError_t e = hipMalloc(&b.p, bytes);
  if (e != hipSuccess) return fail(LSMS_E_NOMEM, "hipMalloc(%zu) failed: %s", bytes, hipGetErrorString(e));
  b.bytes = bytes;
  return LSMS_OK;
}

// Scratch for the tournament-pivoting panels of a batch of njobs systems of padded size
// npad_max (none below 2 chunks).  The chunk is raised if needed so that the candidates
// of all chunks (NB rows each) form a block of at most 4096 rows.
static int tall_scratch(lsms_ctx* ctx, int njobs, int npad_max, TallScratch* ts, hipStream_t s) {
  const int min_chunk = ((npad_max + 64 * NB - 1) / (64 * NB)) * NB;
  ts->chunk = std::max(ctx->tslu_chunk, min_chunk);
  ts->njobs = njobs;
  ts->npad_max = npad_max;
  ts->base = nullptr;
  const size_t bytes = tall_scratch_bytes(njobs, npad_max, ts->chunk);
  if (bytes == 0) return LSMS_OK;
  int rc = ensure_dev(ctx->tall, bytes, s);
  if (rc) return rc;
  ts->base = ctx->tall.p;
  return LSMS_OK;
}

static int ensure_pinned(lsms_ctx* c, size_t bytes, hipStream_t s) {
  // the previous call's uploads may still read from the pinned buffer
  HIP_TRY(hipStreamSynchronize(s));
  if (c->pinned_bytes >= bytes) return LSMS_OK;
  if (c->pinned) HIP_TRY(hipHostFree(c->pinned));
  c->pinned = nullptr;
  c->pinned_bytes = 0;
  HIP_TRY(hipHostMalloc(&c->pinned, bytes, hipHostMallocDefault));
  c->pinned_bytes = bytes;
  return LSMS_OK;
}

// Gaunt integrals C[L][L'][L''] = int Y_L Y_L' Y_L'' dOmega for l, l' <= 3, l'' <= 6, by a
// Gauss-Legendre (cos t) x uniform (p) product rule that is exact at these degrees.
static void gauss_legendre(int n, std::vector<double>& x, std::vector<double>& w) {
  x.resize(n);
  w.resize(n);
  for (int i = 0; i < n; ++i) {
    double z = cos(M_PI * (i + 0.75) / (n + 0.5));
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = z;
      for (int l = 2; l <= n; ++l) {
        double p2 = ((2 * l - 1) * z * p1 - (l - 1) * p0) / l;
        p0 = p1;
        p1 = p2;
      }
      // p1 = P_n(z), p0 = P_{n-1}(z)
      double dp = n * (z * p1 - p0) / (z * z - 1.0);
      double dz = p1 / dp;
      z -= dz;
      if (fabs(dz) < 1e-16) break;
    }
    double p0 = 1.0, p1 = z;
    for (int l = 2; l <= n; ++l) {
      double p2 = ((2 * l - 1) * z * p1 - (l - 1) * p0) / l;
      p0 = p1;
      p1 = p2;
    }
    double dp = n * (z * p1 - p0) / (z * z - 1.0);
    x[i] = z;
    w[i] = 2.0 / ((1.0 - z * z) * dp * dp);
  }
}

static void gaunt_dense(std::vector<double>& C) {
  const int nt = 12, np = 20;
  std::vector<double> xt, wt;
  gauss_legendre(nt, xt, wt);
  C.assign(NL * NL * NL3, 0.0);
  double Y[NL3];
  for (int it = 0; it < nt; ++it) {
    double z = xt[it], st = sqrt(1.0 - z * z);
    for (int ip = 0; ip < np; ++ip) {
      double ph = 2.0 * M_PI * ip / np;
      double w = wt[it] * 2.0 * M_PI / np;
      real_ylm_all<6>(st * cos(ph), st * sin(ph), z, Y);
      for (int a = 0; a < NL; ++a)
        for (int b = 0; b < NL; ++b) {
          double wab = w * Y[a] * Y[b];
          for (int c = 0; c < NL3; ++c) C[(a * NL + b) * NL3 + c] += wab * Y[c];
        }
    }
  }
  for (double& v : C)
    if (fabs(v) < 1e-13) v = 0.0;
}

static int build_gaunt(GauntTable& g) {
  std::vector<double> C;
  gaunt_dense(C);
  int q = 0;
  for (int p = 0; p < NL * NL; ++p) {
    g.start[p] = q;
    for (int c = 0; c < NL3; ++c) {
      double v = C[p * NL3 + c];
      if (v != 0.0) {
        if (q >= MAX_GAUNT) return fail(LSMS_E_ARG, "Gaunt table overflow");
        g.l3[q] = c;
        g.coef[q] = v;
        ++q;
      }
    }
  }
  g.start[NL * NL] = q;
  return LSMS_OK;
}

extern "C" int lsms_gaunt_table(double* out) {
  if (!out) return fail(LSMS_E_ARG, "out is NULL");
  std::vector<double> C;
  gaunt_dense(C);
  std::memcpy(out, C.data(), C.size() * sizeof(double));
  return LSMS_OK;
}

extern "C" int lsms_create(int hip_device, int lmax, size_t workspace_limit, lsms_ctx** out) {
  if (!out) return fail(LSMS_E_ARG, "out is NULL");
  *out = nullptr;
  if (lmax != LSMS_LMAX) return fail(LSMS_E_ARG, "lmax must be %d (got %d)", LSMS_LMAX, lmax);
  int ndev = 0;
  HIP_TRY(hipGetDeviceCount(&ndev));
  if (hip_device < 0 || hip_device >= ndev) return fail(LSMS_E_ARG, "hip_device %d out of range [0, %d)", hip_device, ndev);
  HIP_TRY(hipSetDevice(hip_device));
  std::unique_ptr<lsms_ctx> c(new (std::nothrow) lsms_ctx());
  if (!c) return fail(LSMS_E_NOMEM, "host allocation failed");
  c->device = hip_device;
  std::memset(c->tuned, -1, sizeof(c->tuned));
  if (workspace_limit == 0) {
    size_t fr = 0, tot = 0;
    HIP_TRY(hipMemGetInfo(&fr, &tot));
    workspace_limit = (size_t)(0.6 * (double)fr);
  }
  c->workspace_limit = workspace_limit;
  {
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, hip_device) == hipSuccess && cus > 0)
      c->cu_count = cus;
  }
  int rc = build_gaunt(c->gaunt);
  if (rc) return rc;
  HIP_TRY(upload_gaunt(c->gaunt));
  HIP_TRY(noalloc_scratch_init(hip_device));
  // a tuning cache named by the environment is read when it exists (and fits this device)
  if (const char* path = std::getenv("LSMS_TUNE_CACHE")) {
    FILE* f = std::fopen(path, "r");
    if (f) {
      std::fclose(f);
      rc = lsms_tuning_load(c.get(), path);
      if (rc != LSMS_OK && rc != LSMS_E_STATE) return rc;
    }
  }
  HIP_TRY(hipHostMalloc((void**)&c->pinned_flag, 256, hipHostMallocDefault));
  *out = c.release();
  return LSMS_OK;
}

extern "C" int lsms_destroy(lsms_ctx* ctx) {
  if (!ctx) return fail(LSMS_E_ARG, "ctx is NULL");
  hipSetDevice(ctx->device);
  hipDeviceSynchronize();
  if (ctx->work.p) hipFree(ctx->work.p);
  if (ctx->small.p) hipFree(ctx->small.p);
  if (ctx->pinned) hipHostFree(ctx->pinned);
  if (ctx->pinned_flag) hipHostFree(ctx->pinned_flag);
  if (ctx->fallback.p) hipFree(ctx->fallback.p);
  if (ctx->fallback_mat.p) hipFree(ctx->fallback_mat.p);
  if (ctx->tall.p) hipFree(ctx->tall.p);
  if (ctx->ldlt.p) hipFree(ctx->ldlt.p);
  for (auto& kv : ctx->graph_cache) hipGraphExecDestroy(kv.second);
  if (ctx->capture) hipStreamDestroy(ctx->capture);
  if (ctx->side.update_done) hipEventDestroy(ctx->side.update_done);
  if (ctx->side.panel_done) hipEventDestroy(ctx->side.panel_done);
  if (ctx->side.stream) hipStreamDestroy(ctx->side.stream);
  if (ctx->pipe_start) hipEventDestroy(ctx->pipe_start);
  if (ctx->pipe_end) hipEventDestroy(ctx->pipe_end);
  if (ctx->pipe) hipStreamDestroy(ctx->pipe);
  delete ctx;
  return LSMS_OK;
}

// ---------------------------------------------------------------------------------
// LIZ construction (Sec. II.A, Fig. 1)
// ---------------------------------------------------------------------------------
static inline int64_t quant(double v) { return (int64_t)floor(v * 1e9 + 0.5); }

// centre: nullptr (every atom) or a per-atom flag; atoms without it get an empty LIZ.
static int build_liz_impl(int32_t n_atoms, const double* pos, const double* cell, double r_liz, int64_t capacity,
                          int64_t* liz_ptr, int32_t* liz_atom, double* liz_pos, int64_t* needed,
                          const std::vector<char>* centre) {
  if (!pos || !needed || !liz_ptr) return fail(LSMS_E_ARG, "NULL argument");
  if (n_atoms <= 0) return fail(LSMS_E_ARG, "n_atoms must be positive");
  if (!(r_liz > 0.0) || !std::isfinite(r_liz)) return fail(LSMS_E_ARG, "r_liz must be a positive finite number");
  for (int64_t i = 0; i < 3 * (int64_t)n_atoms; ++i)
    if (!std::isfinite(pos[i])) return fail(LSMS_E_ARG, "non-finite position");
  double c[3][3] = {{0}};
  double inv[3][3] = {{0}};
  int K[3] = {0, 0, 0};
  double h[3] = {0, 0, 0};
  if (cell) {
    for (int i = 0; i < 9; ++i) {
      if (!std::isfinite(cell[i])) return fail(LSMS_E_ARG, "non-finite cell");
      c[i / 3][i % 3] = cell[i];
    }
    double det = c[0][0] * (c[1][1] * c[2][2] - c[1][2] * c[2][1]) - c[0][1] * (c[1][0] * c[2][2] - c[1][2] * c[2][0]) +
                 c[0][2] * (c[1][0] * c[2][1] - c[1][1] * c[2][0]);
    if (fabs(det) < 1e-12) return fail(LSMS_E_ARG, "singular cell");
    // inverse (columns map cartesian -> fractional): f = x * inv
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) {
        int i1 = (j + 1) % 3, i2 = (j + 2) % 3, j1 = (i + 1) % 3, j2 = (i + 2) % 3;
        inv[i][j] = (c[i1][j1] * c[i2][j2] - c[i1][j2] * c[i2][j1]) / det;
      }
    for (int d = 0; d < 3; ++d) {
      const double* e = c[(d + 1) % 3];
      const double* f = c[(d + 2) % 3];
      double cx = e[1] * f[2] - e[2] * f[1], cy = e[2] * f[0] - e[0] * f[2], cz = e[0] * f[1] - e[1] * f[0];
      h[d] = fabs(det) / sqrt(cx * cx + cy * cy + cz * cz);
      K[d] = (int)ceil(r_liz / h[d]) + 1;
    }
  }
  const double r2max = r_liz * r_liz;
  struct Mem {
    int64_t k0, k1, k2, k3;
    int32_t atom;
    double d[3];
  };
  std::vector<Mem> mem;
  std::vector<double> frac;
  if (cell) {
    frac.resize(3 * (size_t)n_atoms);
    for (int j = 0; j < n_atoms; ++j)
      for (int d = 0; d < 3; ++d)
        frac[3 * j + d] = pos[3 * j] * inv[0][d] + pos[3 * j + 1] * inv[1][d] + pos[3 * j + 2] * inv[2][d];
  }
  int64_t total = 0;
  liz_ptr[0] = 0;
  for (int i = 0; i < n_atoms; ++i) {
    mem.clear();
    if (centre && !(*centre)[i]) {
      liz_ptr[i + 1] = total;
      continue;
    }
    const double* pi = pos + 3 * (size_t)i;
    for (int j = 0; j < n_atoms; ++j) {
      const double* pj = pos + 3 * (size_t)j;
      int lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
      if (cell) {
        for (int d = 0; d < 3; ++d) {
          double f = frac[3 * j + d] - frac[3 * i + d];
          lo[d] = std::max(-K[d], (int)ceil(-r_liz / h[d] - f) - 1);
          hi[d] = std::min(K[d], (int)floor(r_liz / h[d] - f) + 1);
        }
      }
      for (int n1 = lo[0]; n1 <= hi[0]; ++n1)
        for (int n2 = lo[1]; n2 <= hi[1]; ++n2)
          for (int n3 = lo[2]; n3 <= hi[2]; ++n3) {
            double T[3];
            for (int d = 0; d < 3; ++d) {
              double t = (double)n1 * c[0][d] + (double)n2 * c[1][d];
              T[d] = t + (double)n3 * c[2][d];
            }
            double dd[3];
            for (int d = 0; d < 3; ++d) dd[d] = (pj[d] + T[d]) - pi[d];
            double d2 = dd[0] * dd[0] + dd[1] * dd[1];
            d2 = d2 + dd[2] * dd[2];
            if (d2 < r2max) {
              Mem m;
              m.k0 = quant(d2);
              m.k1 = quant(dd[0]);
              m.k2 = quant(dd[1]);
              m.k3 = quant(dd[2]);
              m.atom = j;
              m.d[0] = dd[0];
              m.d[1] = dd[1];
              m.d[2] = dd[2];
              mem.push_back(m);
            }
          }
    }
    std::stable_sort(mem.begin(), mem.end(), [](const Mem& a, const Mem& b) {
      if (a.k0 != b.k0) return a.k0 < b.k0;
      if (a.k1 != b.k1) return a.k1 < b.k1;
      if (a.k2 != b.k2) return a.k2 < b.k2;
      return a.k3 < b.k3;
    });
    if (mem.empty() || mem[0].atom != i || mem[0].k0 != 0)
      return fail(LSMS_E_ARG, "atom %d is not at the centre of its own LIZ", i);
    if (mem.size() > 1) {
      const Mem& m = mem[1];
      double d2 = m.d[0] * m.d[0] + m.d[1] * m.d[1] + m.d[2] * m.d[2];
      if (d2 < 1e-16) return fail(LSMS_E_ARG, "coincident sites near atom %d", i);
    }
    if ((int64_t)mem.size() > LSMS_MAX_LIZ)
      return fail(LSMS_E_ARG, "LIZ of atom %d has %zu members (limit %d)", i, mem.size(), LSMS_MAX_LIZ);
    if (total + (int64_t)mem.size() <= capacity && liz_atom && liz_pos) {
      for (size_t q = 0; q < mem.size(); ++q) {
        liz_atom[total + q] = mem[q].atom;
        for (int d = 0; d < 3; ++d) liz_pos[3 * (total + q) + d] = mem[q].d[d];
      }
    }
    total += (int64_t)mem.size();
    liz_ptr[i + 1] = total;
  }
  *needed = total;
  if (total > capacity || !liz_atom || !liz_pos)
    return fail(LSMS_E_CAPACITY, "capacity %lld < needed %lld", (long long)capacity, (long long)total);
  return LSMS_OK;
}

extern "C" int lsms_build_liz(lsms_ctx* ctx, int32_t n_atoms, const double* pos, const double* cell, double r_liz,
                              int64_t capacity, int64_t* liz_ptr, int32_t* liz_atom, double* liz_pos,
                              int64_t* needed) {
  (void)ctx;
  return build_liz_impl(n_atoms, pos, cell, r_liz, capacity, liz_ptr, liz_atom, liz_pos, needed, nullptr);
}

extern "C" int lsms_build_liz_subset(lsms_ctx* ctx, int32_t n_atoms, const double* pos, const double* cell,
                                     double r_liz, int32_t n_centres, const int32_t* centres, int64_t capacity,
                                     int64_t* liz_ptr, int32_t* liz_atom, double* liz_pos, int64_t* needed) {
  (void)ctx;
  if (n_atoms <= 0) return fail(LSMS_E_ARG, "n_atoms must be positive");
  if (n_centres < 1 || !centres) return fail(LSMS_E_ARG, "at least one centre atom is needed");
  std::vector<char> mask((size_t)n_atoms, 0);
  for (int c = 0; c < n_centres; ++c) {
    if (centres[c] < 0 || centres[c] >= n_atoms) return fail(LSMS_E_ARG, "centre %d out of range", centres[c]);
    mask[centres[c]] = 1;
  }
  return build_liz_impl(n_atoms, pos, cell, r_liz, capacity, liz_ptr, liz_atom, liz_pos, needed, &mask);
}

// ---------------------------------------------------------------------------------
// scheduling helpers
// ---------------------------------------------------------------------------------
static inline int64_t align_up(int64_t v, int64_t a) { return (v + a - 1) / a * a; }

struct JobBytes {
  int64_t a, v, x, r, piv;
};

static JobBytes job_bytes(int npad, int precision) {
  JobBytes b;
  const int64_t n2 = (int64_t)npad * npad;
  b.a = align_up(n2 * (precision == LSMS_SPLIT ? 8 : 16), 256);
  const int64_t nb = npad / NL;
  b.v = precision == LSMS_SPLIT ? align_up(nb * (nb + 1) / 2 * VBLOCK * 16, 256) : 0;
  b.x = align_up((int64_t)npad * NRHS_MAX * 16, 256);
  b.r = precision == LSMS_SPLIT ? b.x : 0;
  b.piv = align_up(piv_ints(npad) * 4, 256);
  return b;
}

// allow_empty: an atom with no LIZ members is skipped (its outputs are zero).
static int validate_liz_ptr(int32_t n_atoms, const int64_t* liz_ptr, bool allow_empty = false) {
  if (n_atoms <= 0) return fail(LSMS_E_ARG, "n_atoms must be positive");
  if (!liz_ptr) return fail(LSMS_E_ARG, "liz_ptr is NULL");
  if (liz_ptr[0] != 0) return fail(LSMS_E_ARG, "liz_ptr[0] must be 0");
  for (int i = 0; i < n_atoms; ++i) {
    int64_t nl = liz_ptr[i + 1] - liz_ptr[i];
    if (nl < (allow_empty ? 0 : 1) || nl > LSMS_MAX_LIZ)
      return fail(LSMS_E_ARG, "LIZ of atom %d has %lld members", i, (long long)nl);
  }
  return LSMS_OK;
}

// One wave: jobs [b, e) of the sorted job list share the workspace.
struct Wave {
  int b, e;
  int64_t bytes;
};

// Jobs (sorted by size) grouped into waves of at most `limit` bytes.  A wave that the limit
// cuts is trimmed to a multiple of `round` jobs (the compute units: the panel, inverse and
// diagonal-solve launches run one workgroup per job, one per compute unit at a time), so no
// wave but the last ends in a nearly empty round of those latency-bound launches.  The waves
// are then evened out: with w waves needed, each takes about 1/w of the jobs (rounded to the
// same multiple), so that the last is not a small remainder whose launches fill the chip
// poorly.
static std::vector<Wave> make_waves_capped(std::vector<JobDesc>& jobs, int precision, int64_t limit, bool single,
                                           int round, int cap) {
  std::vector<Wave> waves;
  const int n = (int)jobs.size();
  std::vector<int64_t> need(n);
  for (int j = 0; j < n; ++j) {
    JobBytes jb = job_bytes(jobs[j].npad, precision);
    need[j] = jb.a + jb.v + jb.x + jb.r + jb.piv;
  }
  int b = 0;
  int64_t acc = 0;
  for (int j = 0; j < n; ++j) {
    if (!single && j > b && (acc + need[j] > limit || j - b >= cap)) {
      int e = j;
      if (round > 1 && j - b > round && j - b < cap) e = b + (j - b) / round * round;
      int64_t bytes = 0;
      for (int q = b; q < e; ++q) bytes += need[q];
      waves.push_back({b, e, bytes});
      b = e;
      acc = 0;
      for (int q = b; q < j; ++q) acc += need[q];
    }
    acc += need[j];
  }
  waves.push_back({b, n, acc});
  return waves;
}

static std::vector<Wave> make_waves(std::vector<JobDesc>& jobs, int precision, int64_t limit, bool single,
                                    int round = 1) {
  std::vector<Wave> waves = make_waves_capped(jobs, precision, limit, single, round, 8192);
  const int nw = (int)waves.size();
  if (single || nw < 2) return waves;
  const int n = (int)jobs.size();
  int cap = (n + nw - 1) / nw;
  if (round > 1) cap = (cap + round - 1) / round * round;
  std::vector<Wave> even = make_waves_capped(jobs, precision, limit, single, round, std::min(cap, 8192));
  return even.size() <= waves.size() ? even : waves;
}

// Offsets (complex elements for matrices / blocks, int32 elements for pivots) of every
// job of a wave inside one allocation: [matrices | v | x | r | piv].  Split mode keeps no FP64
// copy of the matrices, only the packed FP64 contractions v of every pair of members, from
// which the refinement's residual forms M X.
static void layout_wave(std::vector<JobDesc>& jobs, const Wave& w, int precision, int64_t& bytes_a,
                        int64_t& bytes_v, int64_t& bytes_x, int64_t& bytes_r, int64_t& bytes_p) {
  bytes_a = bytes_v = bytes_x = bytes_r = bytes_p = 0;
  for (int j = w.b; j < w.e; ++j) {
    JobBytes jb = job_bytes(jobs[j].npad, precision);
    jobs[j].a_off = bytes_a / (precision == LSMS_SPLIT ? 8 : 16);
    bytes_a += jb.a;
    jobs[j].v_off = precision == LSMS_SPLIT ? bytes_v / 16 : -1;
    bytes_v += jb.v;
    jobs[j].x_off = bytes_x / 16;
    bytes_x += jb.x;
    jobs[j].r_off = precision == LSMS_SPLIT ? bytes_r / 16 : -1;
    bytes_r += jb.r;
    jobs[j].piv_off = bytes_p / 4;
    bytes_p += jb.piv;
  }
}

static void energies(double e_fermi, double eta, double2& kp, double2& km) {
  std::complex<double> z(e_fermi, eta);
  std::complex<double> k = std::sqrt(z);
  if (k.imag() < 0) k = -k;
  kp = make_double2(k.real(), k.imag());
  km = make_double2(-k.real(), k.imag());
}

// Refinement state per job: norms[j][0] = ||M||_inf, [1] = ||r||_inf, [2] = ||X||_inf, [3] = berr.
namespace lsms {
void launch_refine_step(const JobDesc* jobs, int njobs, double* norms, double tol, int32_t* done, int last,
                        int32_t* job_info, int32_t* pending, hipStream_t s);
void launch_zero_i32(int32_t* p, int n, hipStream_t s);
void launch_zero_pivot_to_fallback(int njobs, int32_t* job_info, hipStream_t s);
void launch_fallback_status(int nf, const JobDesc* fjobs, const int32_t* finfo, int32_t* job_info, double* norms,
                            hipStream_t s);
}  // namespace lsms

// ---------------------------------------------------------------------------------
// tau solve
// ---------------------------------------------------------------------------------
// Factorization + first solve of one wave: a fixed launch sequence whose arguments depend
// only on the wave's shape and buffers, so with graphs on it is captured once (on the
// context's own non-blocking stream, nothing runs during capture) and replayed on the
// caller's stream whenever the same shape and buffers come back.  Job descriptors, matrices
// and right-hand sides are read from device memory at replay, after the caller's stream has
// written them.
static int side_stream(lsms_ctx* ctx, const SideStream** out) {
  *out = nullptr;
  if (!ctx->lookahead) return LSMS_OK;
  if (!ctx->side.stream) {
    HIP_TRY(hipStreamCreateWithFlags(&ctx->side.stream, hipStreamNonBlocking));
    HIP_TRY(hipEventCreateWithFlags(&ctx->side.update_done, hipEventDisableTiming));
    HIP_TRY(hipEventCreateWithFlags(&ctx->side.panel_done, hipEventDisableTiming));
  }
  *out = &ctx->side;
  return LSMS_OK;
}

static int factor_and_solve(lsms_ctx* ctx, int precision, const JobDesc* jd, int nj, int npad_max, void* abuf,
                            int32_t* piv, int32_t* jinfo, double2* xbuf, GemmProfiler* prof, hipStream_t s,
                            bool sym = false) {
  const Tiling tiling = pick_tiling(ctx, precision, npad_max);
  const int variant = tiling.wide;
  TallScratch ts;
  int rc = tall_scratch(ctx, nj, npad_max, &ts, s);
  if (rc) return rc;
  if (sym) {
    rc = ensure_dev(ctx->ldlt, ldlt_scratch_bytes(nj), s);
    if (rc) return rc;
  }
  const SideStream* side = nullptr;
  const bool capture = ctx->graphs && !prof;
  if (!capture) {  // captured graphs keep the single-stream order
    rc = side_stream(ctx, &side);
    if (rc) return rc;
  }
  auto issue = [&](hipStream_t q, GemmProfiler* pr) {
    if (precision == LSMS_FP64) {
      lu_factor_f64(jd, nj, npad_max, (double2*)abuf, piv, jinfo, q, pr, tiling, ts, side);
      lu_solve_f64(jd, nj, npad_max, (const double2*)abuf, piv, xbuf, 0, 16, 0, tiling.group, q);
    } else {
      if (sym)
        ldlt_factor_f32(jd, nj, npad_max, (float2*)abuf, piv, jinfo, q, pr, variant, NB, ctx->ldlt.p);
      else
        lu_factor_f32(jd, nj, npad_max, (float2*)abuf, piv, jinfo, q, pr, tiling, ts, side);
      // the first solve in FP32 on a rounded copy of the right-hand side (refined below)
      launch_x32(jd, nj, npad_max, 0, xbuf, xbuf, nullptr, q);
      lu_solve_f32_single(jd, nj, npad_max, (const float2*)abuf, piv, xbuf, nullptr, tiling.group, q);
      launch_x32(jd, nj, npad_max, 1, nullptr, xbuf, nullptr, q);
    }
  };
  if (!ctx->graphs || prof) {
    issue(s, prof);
    HIP_TRY(hipGetLastError());
    return LSMS_OK;
  }
  const std::vector<intptr_t> key = {precision, nj, npad_max, variant, tiling.narrow, tiling.panel_small_rows,
                                     tiling.group,
                                     (intptr_t)jd, (intptr_t)abuf,
                                     (intptr_t)piv, (intptr_t)jinfo, (intptr_t)xbuf, ts.chunk,
                                     (intptr_t)ts.base, sym ? 1 : 0, (intptr_t)ctx->ldlt.p};
  auto it = ctx->graph_cache.find(key);
  if (it == ctx->graph_cache.end()) {
    if (!ctx->capture) HIP_TRY(hipStreamCreateWithFlags(&ctx->capture, hipStreamNonBlocking));
    HIP_TRY(hipStreamBeginCapture(ctx->capture, hipStreamCaptureModeThreadLocal));
    issue(ctx->capture, nullptr);
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(ctx->capture, &g);
    if (e != hipSuccess || !g) return fail(LSMS_E_DEVICE, "graph capture failed: %s", hipGetErrorString(e));
    hipGraphExec_t ex = nullptr;
    const hipError_t ei = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    hipGraphDestroy(g);
    if (ei != hipSuccess) return fail(LSMS_E_DEVICE, "graph instantiation failed: %s", hipGetErrorString(ei));
    it = ctx->graph_cache.emplace(key, ex).first;
  }
  HIP_TRY(hipGraphLaunch(it->second, s));
  return LSMS_OK;
}

extern "C" int lsms_tau_solve(lsms_ctx* ctx, int32_t n_atoms, const int64_t* liz_ptr, const int32_t* liz_atom,
                              const double* liz_pos, const double* phase, double e_fermi, double eta, int precision,
                              double refine_tol, int max_refine, void* tau_plus, void* tau_minus, int32_t* info,
                              double* berr, lsms_factors** keep, void* hip_stream) {
  if (!ctx) return fail(LSMS_E_ARG, "ctx is NULL");
  int rc = validate_liz_ptr(n_atoms, liz_ptr, keep == nullptr);
  if (rc) return rc;
  if (!liz_atom || !liz_pos || !phase || !tau_plus || !tau_minus || !info || !berr)
    return fail(LSMS_E_ARG, "NULL device pointer");
  if (!std::isfinite(e_fermi) || !(eta > 0.0) || !std::isfinite(eta))
    return fail(LSMS_E_ARG, "e_fermi must be finite and eta positive");
  if (precision != LSMS_FP64 && precision != LSMS_SPLIT) return fail(LSMS_E_ARG, "unknown precision %d", precision);
  if (precision == LSMS_SPLIT && (!(refine_tol > 0.0) || max_refine < 0 || max_refine > 100))
    return fail(LSMS_E_ARG, "refine_tol must be > 0 and 0 <= max_refine <= 100");
  if (keep && precision != LSMS_FP64) return fail(LSMS_E_ARG, "keep (factors for the adjoint) needs LSMS_FP64");
  if (keep) *keep = nullptr;
  hipStream_t s = (hipStream_t)hip_stream;
  HIP_TRY(hipSetDevice(ctx->device));

  // jobs, sorted by size (largest first) so each wave is nearly uniform; with the
  // conjugation symmetry (and no factors kept for the adjoint) only z+ is solved
  const bool mirror = ctx->conj_symmetry && keep == nullptr;
  std::vector<JobDesc> jobs;
  jobs.reserve(2 * (size_t)n_atoms);
  for (int a = 0; a < n_atoms; ++a) {
    const int nl = (int)(liz_ptr[a + 1] - liz_ptr[a]);
    if (nl == 0) continue;  // skipped atom
    for (int e = 0; e < (mirror ? 1 : 2); ++e) {
      JobDesc j{};
      j.liz_off = liz_ptr[a];
      j.atom = a;
      j.energy = e;
      j.nl = nl;
      j.n = NL * nl;
      j.npad = (int)align_up(j.n, PAD);
      jobs.push_back(j);
    }
  }
  std::stable_sort(jobs.begin(), jobs.end(), [](const JobDesc& x, const JobDesc& y) { return x.npad > y.npad; });
  if ((int64_t)jobs.size() < (mirror ? 1 : 2) * (int64_t)n_atoms) {  // skipped atoms report info 0, berr 0
    launch_zero_i32(info, 2 * n_atoms, s);
    launch_zero(berr, 2 * (int64_t)n_atoms, s);
    HIP_TRY(hipGetLastError());
  }
  if (jobs.empty()) return LSMS_OK;
  // the symmetric form (split mode, no kept factors)
  const bool sym = ctx->symmetric && precision == LSMS_SPLIT && keep == nullptr;
  const int64_t tpm_bytes = align_up((int64_t)n_atoms * 8 * 16, 256);
  const int64_t small_fixed = 2 * tpm_bytes;  // tpm | spm
  const int64_t limit = (int64_t)ctx->workspace_limit;
  // Pipelining: with two or more waves, waves alternate between the caller's stream and a
  // second one, each stream with its own half of the workspace, and the next wave's
  // assembly, factorization and first solve are issued before this wave's refinement loop
  // (whose host reads wait on its own stream only), so HBM-bound refinement overlaps
  // matrix-core factorization.  Waves on one stream run in order, which is what makes
  // reusing a half safe.  Not used where waves would share other context scratch (kept
  // factors, the symmetric form's tall-panel scratch, tournament panels, the look-ahead
  // stream) or with kernel profiling (its timings assume one stream).
  bool pipe = ctx->pipeline && keep == nullptr && !ctx->profiling && !sym && !ctx->lookahead &&
              jobs[0].npad <= 2 * std::max(ctx->tslu_chunk, NB);
  std::vector<Wave> waves;
  if (pipe) {
    waves = make_waves(jobs, precision, limit / 2, false, ctx->cu_count);
    int64_t mw = 0;
    for (auto& w : waves) mw = std::max(mw, w.bytes);
    if (waves.size() < 2 || mw > limit / 2) pipe = false;
  }
  if (!pipe) waves = make_waves(jobs, precision, limit, keep != nullptr, ctx->cu_count);
  int64_t max_wave = 0;
  for (auto& w : waves) max_wave = std::max(max_wave, w.bytes);
  max_wave = align_up(max_wave, 256);
  if (max_wave > (pipe ? limit / 2 : limit)) {
    return fail(LSMS_E_NOMEM, "a wave needs %lld bytes of workspace but the limit is %lld%s", (long long)max_wave,
                (long long)limit, keep ? " (keep requires every factor to stay resident)" : "");
  }
  double2 kp, km;
  energies(e_fermi, eta, kp, km);

  // small per-call device arrays: tpm | jobdesc (all jobs) | job_info | norms | done
  const int njobs_all = (int)jobs.size();
  const int64_t off_jobs = small_fixed;
  const int64_t off_info = off_jobs + align_up((int64_t)njobs_all * sizeof(JobDesc), 256);
  const int64_t off_norm = off_info + align_up((int64_t)njobs_all * 4, 256);
  const int64_t off_done = off_norm + align_up((int64_t)njobs_all * 8 * 8, 256);
  const int64_t off_pend = off_done + align_up((int64_t)njobs_all * 4, 256);
  const int64_t small_bytes = off_pend + 256;

  // lay out every wave now (offsets are relative to the wave's base)
  std::vector<int64_t> wave_sizes(waves.size() * 5);
  for (size_t w = 0; w < waves.size(); ++w)
    layout_wave(jobs, waves[w], precision, wave_sizes[5 * w], wave_sizes[5 * w + 1], wave_sizes[5 * w + 2],
                wave_sizes[5 * w + 3], wave_sizes[5 * w + 4]);

  rc = ensure_pinned(ctx, (size_t)njobs_all * sizeof(JobDesc), s);
  if (rc) return rc;
  std::memcpy(ctx->pinned, jobs.data(), (size_t)njobs_all * sizeof(JobDesc));

  // factors kept for the adjoint get their own allocation; otherwise the context's pool
  char* wbase = nullptr;
  char* sbase = nullptr;
  std::unique_ptr<lsms_factors> fac;
  if (keep) {
    fac.reset(new lsms_factors());
    fac->ctx = ctx;
    fac->precision = precision;
    fac->group = pick_tiling(ctx, precision, 0).group;
    fac->n_atoms = n_atoms;
    fac->kp = kp;
    fac->km = km;
    fac->work_bytes = (size_t)(max_wave + small_bytes);
    hipError_t e = hipMalloc(&fac->work, fac->work_bytes);
    if (e != hipSuccess) return fail(LSMS_E_NOMEM, "hipMalloc(%zu) for kept factors failed", fac->work_bytes);
    wbase = (char*)fac->work;
    sbase = wbase + max_wave;
  } else {
    const size_t need = (size_t)max_wave * (pipe ? 2 : 1);
    if (ctx->work.bytes < need) {
      // grow with slack, so alternating precisions or slightly larger waves do not
      // reallocate (and re-map) tens of GB on every call
      const size_t want = std::min((size_t)limit, std::max(need + (need >> 2), 2 * ctx->work.bytes));
      if (ctx->pipe) HIP_TRY(hipStreamSynchronize(ctx->pipe));  // a previous call's second stream
      rc = ensure_dev(ctx->work, std::max(want, need), s);
      if (rc) return rc;
    }
    rc = ensure_dev(ctx->small, (size_t)small_bytes, s);
    if (rc) return rc;
    wbase = (char*)ctx->work.p;
    sbase = (char*)ctx->small.p;
  }
  double2* tpm = (double2*)sbase;
  double2* spm = sym ? (double2*)(sbase + tpm_bytes) : nullptr;
  const double2* rhs_t = sym ? spm : tpm;  // diagonal of the right-hand side's first block
  JobDesc* jobs_dev = (JobDesc*)(sbase + off_jobs);
  int32_t* job_info = (int32_t*)(sbase + off_info);
  double* norms = (double*)(sbase + off_norm);
  int32_t* done = (int32_t*)(sbase + off_done);
  int32_t* pending = (int32_t*)(sbase + off_pend);
  HIP_TRY(hipMemcpyAsync(jobs_dev, ctx->pinned, (size_t)njobs_all * sizeof(JobDesc), hipMemcpyHostToDevice, s));
  launch_tmatrix(phase, n_atoms, kp, tpm, spm, s);

  if (pipe) {
    if (!ctx->pipe) {
      HIP_TRY(hipStreamCreateWithFlags(&ctx->pipe, hipStreamNonBlocking));
      HIP_TRY(hipEventCreateWithFlags(&ctx->pipe_start, hipEventDisableTiming));
      HIP_TRY(hipEventCreateWithFlags(&ctx->pipe_end, hipEventDisableTiming));
    }
    // the second stream starts after the uploads above
    HIP_TRY(hipEventRecord(ctx->pipe_start, s));
    HIP_TRY(hipStreamWaitEvent(ctx->pipe, ctx->pipe_start, 0));
  }
  hipStream_t const caller = s;
  struct WaveBufs {
    void* abuf;
    double2 *vtab, *xbuf, *rbuf;
    int32_t* piv;
  };
  auto bufs_of = [&](size_t w) {
    char* p = wbase + (pipe ? (int64_t)(w & 1) * max_wave : 0);
    WaveBufs b;
    b.abuf = p;
    p += wave_sizes[5 * w];
    b.vtab = (double2*)p;
    p += wave_sizes[5 * w + 1];
    b.xbuf = (double2*)p;
    p += wave_sizes[5 * w + 2];
    b.rbuf = (double2*)p;
    p += wave_sizes[5 * w + 3];
    b.piv = (int32_t*)p;
    return b;
  };
  // stage 1 of a wave: inputs, right-hand side, assembly, factorization, first solve (and,
  // in FP64 mode, the whole wave); nothing here waits on the host
  auto stage1 = [&](size_t w) -> int {
    hipStream_t s = (pipe && (w & 1)) ? ctx->pipe : caller;
    const Wave& wv = waves[w];
    const int nj = wv.e - wv.b;
    const int npad_max = jobs[wv.b].npad;
    const JobDesc* jd = jobs_dev + wv.b;
    int32_t* jinfo = job_info + wv.b;
    double* jnorm = norms + 8 * (size_t)wv.b;
    int32_t* jdone = done + wv.b;
    const WaveBufs wb = bufs_of(w);
    void* abuf = wb.abuf;
    double2* xbuf = wb.xbuf;
    int32_t* piv = wb.piv;
    int rc;
    GemmProfiler* prof = nullptr;
    if (ctx->profiling) {
      ctx->n_true.resize(nj);
      for (int j = 0; j < nj; ++j) ctx->n_true[j] = jobs[wv.b + j].n;
      ctx->prof.n_true = ctx->n_true.data();
      prof = &ctx->prof;
    }
    launch_check_inputs(jd, nj, liz_pos, liz_atom, phase, jinfo, s);
    launch_init_rhs(jd, nj, npad_max, liz_atom, rhs_t, xbuf, s);
    if (precision == LSMS_FP64) {
      launch_assemble_f64(jd, nj, npad_max, liz_pos, liz_atom, tpm, kp, km, (double2*)abuf, nullptr, s);
      rc = factor_and_solve(ctx, precision, jd, nj, npad_max, abuf, piv, jinfo, xbuf, prof, s);
      if (rc) return rc;
      launch_copy_tau(jd, nj, npad_max, xbuf, (double2*)tau_plus, (double2*)tau_minus, mirror, nullptr, liz_atom,
                      s);
      launch_write_status(jd, nj, jinfo, nullptr, info, berr, mirror, s);
    } else {
      launch_assemble_split(jd, nj, npad_max, liz_pos, liz_atom, tpm, kp, km, (float2*)abuf, wb.vtab, spm, s);
      rc = factor_and_solve(ctx, precision, jd, nj, npad_max, abuf, piv, jinfo, xbuf, prof, s, sym);
      if (rc) return rc;
      if (sym) launch_zero_pivot_to_fallback(nj, jinfo, s);
      launch_zero_i32(jdone, nj, s);
      launch_zero(jnorm, 8 * (int64_t)nj, s);
    }
    HIP_TRY(hipGetLastError());
    return LSMS_OK;
  };
  // stage 2 of a split-mode wave: refinement (host reads of its own stream only), FP64
  // fallback, tau blocks and status
  auto stage2 = [&](size_t w) -> int {
    if (precision == LSMS_FP64) return LSMS_OK;
    hipStream_t s = (pipe && (w & 1)) ? ctx->pipe : caller;
    const Wave& wv = waves[w];
    const int nj = wv.e - wv.b;
    const int npad_max = jobs[wv.b].npad;
    const JobDesc* jd = jobs_dev + wv.b;
    int32_t* jinfo = job_info + wv.b;
    double* jnorm = norms + 8 * (size_t)wv.b;
    int32_t* jdone = done + wv.b;
    const WaveBufs wb = bufs_of(w);
    void* abuf = wb.abuf;
    double2* xbuf = wb.xbuf;
    double2* rbuf = wb.rbuf;
    int32_t* piv = wb.piv;
    int rc;
    {
      int left = nj;
      for (int it = 0; it <= max_refine; ++it) {
        const int last = it == max_refine;
        launch_residual(jd, nj, npad_max, wb.vtab, liz_atom, tpm, spm, xbuf, rbuf, jnorm, jdone, it == 0, s);
        launch_zero_i32(pending, 1, s);
        launch_refine_step(jd, nj, jnorm, refine_tol, jdone, last, jinfo, pending, s);
        // read back how many jobs still miss the tolerance: stop as soon as none does
        HIP_TRY(hipMemcpyAsync(ctx->pinned_flag, pending, 4, hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        left = ctx->pinned_flag[0];
        if (last || left == 0) break;
        // correction: FP32 solve on the rounded residual, added to the FP64 solution
        launch_x32(jd, nj, npad_max, 0, rbuf, xbuf, jdone, s);
        lu_solve_f32_single(jd, nj, npad_max, (const float2*)abuf, piv, xbuf, jdone,
                            pick_tiling(ctx, LSMS_SPLIT, npad_max).group, s);
        launch_x32(jd, nj, npad_max, 2, nullptr, xbuf, jdone, s);
      }
      if (left > 0 || sym) {
        // Jobs whose refinement did not converge (info = NOCONV; in the symmetric form also
        // those that met a zero pivot) are recomputed in FP64: the matrix is assembled again in
        // FP64, factored with partial pivoting and solved directly.  The FP32 factors are done
        // with, so the wave's matrix area holds these FP64 matrices, as many at a time as fit
        // (a single job whose FP64 matrix does not fit there borrows a buffer of its own).
        std::vector<int32_t> hinfo(nj);
        HIP_TRY(hipMemcpyAsync(hinfo.data(), jinfo, nj * sizeof(int32_t), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        std::vector<JobDesc> fb;
        for (int j = 0; j < nj; ++j)
          if (hinfo[j] == LSMS_INFO_NOCONV) {
            JobDesc d = jobs[wv.b + j];
            d.info = j;
            fb.push_back(d);
          }
        if (!fb.empty()) {
          // jobs are sorted by size, largest first: every chunk's slots take the first job's size
          const int64_t slot = align_up((int64_t)fb[0].npad * fb[0].npad * 16, 256);
          int64_t cap = std::min<int64_t>(wave_sizes[5 * w] / slot, (int64_t)fb.size());
          char* fmat = (char*)abuf;
          if (cap < 1) {
            rc = ensure_dev(ctx->fallback_mat, (size_t)slot, s);
            if (rc) return rc;
            fmat = (char*)ctx->fallback_mat.p;
            cap = 1;
          }
          rc = ensure_dev(ctx->fallback, (size_t)(align_up(cap * (int64_t)sizeof(JobDesc), 256) + 4 * cap + 256), s);
          if (rc) return rc;
          JobDesc* fjd = (JobDesc*)ctx->fallback.p;
          int32_t* finfo = (int32_t*)((char*)ctx->fallback.p + align_up(cap * (int64_t)sizeof(JobDesc), 256));
          for (size_t c0 = 0; c0 < fb.size(); c0 += (size_t)cap) {
            const int nf = (int)std::min<int64_t>(cap, (int64_t)(fb.size() - c0));
            std::vector<JobDesc> part(fb.begin() + c0, fb.begin() + c0 + nf);
            for (int q = 0; q < nf; ++q) part[q].a_off = q * (slot / 16);
            const int fpad = part[0].npad;
            HIP_TRY(hipMemcpyAsync(fjd, part.data(), nf * sizeof(JobDesc), hipMemcpyHostToDevice, s));
            launch_zero_i32(finfo, nf, s);
            launch_init_rhs(fjd, nf, fpad, liz_atom, rhs_t, xbuf, s);
            launch_assemble_f64(fjd, nf, fpad, liz_pos, liz_atom, tpm, kp, km, (double2*)fmat, spm, s);
            TallScratch fts;
            rc = tall_scratch(ctx, nf, fpad, &fts, s);
            if (rc) return rc;
            const Tiling ft = pick_tiling(ctx, LSMS_FP64, fpad);
            lu_factor_f64(fjd, nf, fpad, (double2*)fmat, piv, finfo, s, nullptr, ft, fts);
            lu_solve_f64(fjd, nf, fpad, (const double2*)fmat, piv, xbuf, 0, 16, 0, ft.group, s);
            launch_fallback_status(nf, fjd, finfo, jinfo, jnorm, s);
            // the job list (and a borrowed matrix buffer) are context scratch: done before the
            // next chunk or another wave reuses them
            HIP_TRY(hipStreamSynchronize(s));
          }
        }
      }
      launch_copy_tau(jd, nj, npad_max, xbuf, (double2*)tau_plus, (double2*)tau_minus, mirror, spm, liz_atom, s);
      launch_write_status(jd, nj, jinfo, jnorm, info, berr, mirror, s);
    }
    HIP_TRY(hipGetLastError());
    return LSMS_OK;
  };
  if (!pipe) {
    for (size_t w = 0; w < waves.size(); ++w) {
      rc = stage1(w);
      if (rc) return rc;
      rc = stage2(w);
      if (rc) return rc;
    }
  } else {
    rc = stage1(0);
    if (rc) return rc;
    for (size_t w = 0; w < waves.size(); ++w) {
      if (w + 1 < waves.size()) {
        rc = stage1(w + 1);
        if (rc) return rc;
      }
      rc = stage2(w);
      if (rc) return rc;
    }
    // the caller's stream continues after the second stream's last wave
    HIP_TRY(hipEventRecord(ctx->pipe_end, ctx->pipe));
    HIP_TRY(hipStreamWaitEvent(caller, ctx->pipe_end, 0));
  }
  if (keep) {
    fac->jobs = jobs;
    fac->npad_max = jobs[0].npad;
    fac->jobs_dev = jobs_dev;
    fac->x_base = wave_sizes[0] + wave_sizes[1];
    fac->piv_base = wave_sizes[0] + wave_sizes[1] + wave_sizes[2] + wave_sizes[3];
    fac->liz_atom = liz_atom;
    fac->total_members = liz_ptr[n_atoms];
    *keep = fac.release();
  }
  return LSMS_OK;
}

// ---------------------------------------------------------------------------------
// Kubo-Greenwood sum
// ---------------------------------------------------------------------------------
static int kubo_sigma_common(lsms_ctx* ctx, int32_t n_atoms, const int64_t* liz_ptr, const int32_t* liz_atom,
                             const void* tau_plus, const void* tau_minus, const int32_t* species, int32_t n_species,
                             const void* J, double volume, double* sigma, void* sigma_tilde, void* per_atom,
                             bool tensor, void* hip_stream) {
  if (!ctx) return fail(LSMS_E_ARG, "ctx is NULL");
  int rc = validate_liz_ptr(n_atoms, liz_ptr, true);
  if (rc) return rc;
  if (!liz_atom || !tau_plus || !tau_minus || !species || !J || !sigma || !sigma_tilde)
    return fail(LSMS_E_ARG, "NULL device pointer");
  if (n_species <= 0) return fail(LSMS_E_ARG, "n_species must be positive");
  if (!(volume > 0.0) || !std::isfinite(volume)) return fail(LSMS_E_ARG, "volume must be positive");
  hipStream_t s = (hipStream_t)hip_stream;
  HIP_TRY(hipSetDevice(ctx->device));
  const int nq = tensor ? 36 : 12;
  const int64_t off_pa = align_up((int64_t)(n_atoms + 1) * 8, 256);
  const int64_t bytes = off_pa + align_up((int64_t)n_atoms * nq * 16, 256);
  rc = ensure_pinned(ctx, (size_t)(n_atoms + 1) * 8, s);
  if (rc) return rc;
  rc = ensure_dev(ctx->small, (size_t)bytes, s);
  if (rc) return rc;
  std::memcpy(ctx->pinned, liz_ptr, (size_t)(n_atoms + 1) * 8);
  int64_t* ptr_dev = (int64_t*)ctx->small.p;
  double2* pa = per_atom ? (double2*)per_atom : (double2*)((char*)ctx->small.p + off_pa);
  HIP_TRY(hipMemcpyAsync(ptr_dev, ctx->pinned, (size_t)(n_atoms + 1) * 8, hipMemcpyHostToDevice, s));
  launch_kubo_trace(n_atoms, ptr_dev, liz_atom, (const double2*)tau_plus, (const double2*)tau_minus, species,
                    n_species, (const double2*)J, pa, tensor, s);
  launch_kubo_reduce(n_atoms, pa, volume, sigma, (double2*)sigma_tilde, tensor, s);
  HIP_TRY(hipGetLastError());
  return LSMS_OK;
}

extern "C" int lsms_kubo_sigma(lsms_ctx* ctx, int32_t n_atoms, const int64_t* liz_ptr, const int32_t* liz_atom,
                               const void* tau_plus, const void* tau_minus, const int32_t* species, int32_t n_species,
                               const void* J, double volume, double* sigma, void* sigma_tilde, void* per_atom,
                               void* hip_stream) {
  return kubo_sigma_common(ctx, n_atoms, liz_ptr, liz_atom, tau_plus, tau_minus, species, n_species, J, volume,
                           sigma, sigma_tilde, per_atom, false, hip_stream);
}

extern "C" int lsms_kubo_sigma_tensor(lsms_ctx* ctx, int32_t n_atoms, const int64_t* liz_ptr,
                                      const int32_t* liz_atom, const void* tau_plus, const void* tau_minus,
                                      const int32_t* species, int32_t n_species, const void* J, double volume,
                                      double* sigma, void* sigma_tilde, void* per_atom, void* hip_stream) {
  return kubo_sigma_common(ctx, n_atoms, liz_ptr, liz_atom, tau_plus, tau_minus, species, n_species, J, volume,
                           sigma, sigma_tilde, per_atom, true, hip_stream);
}

extern "C" int lsms_kubo_sigma_noalloc(lsms_ctx* ctx, int32_t n_atoms, const int64_t* liz_ptr,
                                       const int32_t* liz_atom, const void* tau_plus, const void* tau_minus,
                                       const int32_t* species, int32_t n_species, const void* J, double volume,
                                       double* sigma, void* sigma_tilde, void* per_atom, void* hip_stream) {
  if (!ctx) return fail(LSMS_E_ARG, "ctx is NULL");
  if (n_atoms < 1 || n_atoms > LSMS_NOALLOC_MAX_ATOMS)
    return fail(LSMS_E_ARG, "n_atoms %d outside [1, %d] (the fixed scratch holds %d atoms)", n_atoms,
                LSMS_NOALLOC_MAX_ATOMS, LSMS_NOALLOC_MAX_ATOMS);
  if (!liz_ptr || !liz_atom || !tau_plus || !tau_minus || !species || !J || !sigma || !sigma_tilde)
    return fail(LSMS_E_ARG, "NULL device pointer");
  if (n_species <= 0) return fail(LSMS_E_ARG, "n_species must be positive");
  if (!(volume > 0.0) || !std::isfinite(volume)) return fail(LSMS_E_ARG, "volume must be positive");
  HIP_TRY(hipSetDevice(ctx->device));
  double2* pa = (double2*)per_atom;
  if (!pa) {
    pa = noalloc_scratch(ctx->device);
    if (!pa) return fail(LSMS_E_STATE, "no scratch address for device %d", ctx->device);
  }
  hipStream_t s = (hipStream_t)hip_stream;
  // every atom's 12 partial sums are written before the reduction reads them, so the scratch
  // needs no clearing between calls
  launch_kubo_trace(n_atoms, liz_ptr, liz_atom, (const double2*)tau_plus, (const double2*)tau_minus, species,
                    n_species, (const double2*)J, pa, false, s);
  launch_kubo_reduce(n_atoms, pa, volume, sigma, (double2*)sigma_tilde, false, s);
  HIP_TRY(hipGetLastError());
  return LSMS_OK;
}

extern "C" int lsms_set_tuning(lsms_ctx* ctx, int knob, int value) {
  if (!ctx) return fail(LSMS_E_ARG, "ctx is NULL");
  if (knob == LSMS_TUNE_LOOKAHEAD || knob == LSMS_TUNE_SYMMETRIC) {
    if (value != 0 && value != 1) return fail(LSMS_E_ARG, "knob %d takes 0 or 1 (got %d)", knob, value);
    (knob == LSMS_TUNE_LOOKAHEAD ? ctx->lookahead : ctx->symmetric) = value == 1;
    return LSMS_OK;
  }
  if (knob == LSMS_TUNE_TSLU_CHUNK) {
    if (value < NB || value > 2048 || value % NB != 0)
      return fail(LSMS_E_ARG, "tournament chunk %d must be a multiple of %d in [%d, 2048]", value, NB, NB);
    ctx->tslu_chunk = value;
    return LSMS_OK;
  }
  if (knob == LSMS_TUNE_GRAPHS || knob == LSMS_TUNE_CONJ_SYMMETRY || knob == LSMS_TUNE_PIPELINE) {
    if (value != 0 && value != 1) return fail(LSMS_E_ARG, "knob %d takes 0 or 1 (got %d)", knob, value);
    (knob == LSMS_TUNE_GRAPHS ? ctx->graphs : knob == LSMS_TUNE_PIPELINE ? ctx->pipeline : ctx->conj_symmetry) =
        value == 1;
    return LSMS_OK;
  }
  if (knob == LSMS_TUNE_GEMM_F32_NARROW || knob == LSMS_TUNE_GEMM_F64 || knob == LSMS_TUNE_GEMM_F64_NARROW) {
    const int nv = knob == LSMS_TUNE_GEMM_F32_NARROW ? gemm_f32_variants_all() : gemm_f64_variants();
    if (value < -1 || value >= nv) return fail(LSMS_E_ARG, "tiling %d outside [-1, %d) for knob %d", value, nv, knob);
    (knob == LSMS_TUNE_GEMM_F32_NARROW ? ctx->gemm_f32_narrow
     : knob == LSMS_TUNE_GEMM_F64      ? ctx->gemm_f64
                                       : ctx->gemm_f64_narrow) = value;
    return LSMS_OK;
  }
  if (knob == LSMS_TUNE_GROUP_F32 || knob == LSMS_TUNE_GROUP_F64) {
    if (value != -1 && (value < 2 || value > GROUP_MAX))
      return fail(LSMS_E_ARG, "panels per group %d outside [2, %d] (or -1)", value, GROUP_MAX);
    (knob == LSMS_TUNE_GROUP_F32 ? ctx->group_f32 : ctx->group_f64) = value;
    return LSMS_OK;
  }
  if (knob == LSMS_TUNE_PANEL_SMALL_ROWS) {
    if (value < -1 || value > PANEL_SMALL_MAX)
      return fail(LSMS_E_ARG, "panel height %d outside [-1, %d]", value, PANEL_SMALL_MAX);
    ctx->panel_small_rows = value;
    return LSMS_OK;
  }
  if (knob != LSMS_TUNE_GEMM_F32) return fail(LSMS_E_ARG, "unknown tuning knob %d", knob);
  if (value < -1 || value >= gemm_f32_variants_all())
    return fail(LSMS_E_ARG, "gemm_f32 tiling %d outside [-1, %d)", value, gemm_f32_variants_all());
  ctx->gemm_f32 = value;
  return LSMS_OK;
}

extern "C" int lsms_get_tuning(lsms_ctx* ctx, int knob, int* value) {
  if (!ctx || !value) return fail(LSMS_E_ARG, "NULL argument");
  if (knob == LSMS_TUNE_TSLU_CHUNK) {
    *value = ctx->tslu_chunk;
    return LSMS_OK;
  }
  if (knob == LSMS_TUNE_LOOKAHEAD || knob == LSMS_TUNE_SYMMETRIC) {
    *value = (knob == LSMS_TUNE_LOOKAHEAD ? ctx->lookahead : ctx->symmetric) ? 1 : 0;
    return LSMS_OK;
  }
  if (knob == LSMS_TUNE_GRAPHS || knob == LSMS_TUNE_CONJ_SYMMETRY || knob == LSMS_TUNE_PIPELINE) {
    *value = (knob == LSMS_TUNE_GRAPHS ? ctx->graphs : knob == LSMS_TUNE_PIPELINE ? ctx->pipeline : ctx->conj_symmetry)
                 ? 1
                 : 0;
    return LSMS_OK;
  }
  if (knob == LSMS_TUNE_GROUP_F32 || knob == LSMS_TUNE_GROUP_F64) {
    const int v = knob == LSMS_TUNE_GROUP_F32 ? ctx->group_f32 : ctx->group_f64;
    *value = v > 0 ? v : (knob == LSMS_TUNE_GROUP_F32 ? kDefaultGroupF32 : kDefaultGroupF64);
    return LSMS_OK;
  }
  if (knob == LSMS_TUNE_GEMM_F32_NARROW || knob == LSMS_TUNE_GEMM_F64 || knob == LSMS_TUNE_GEMM_F64_NARROW ||
      knob == LSMS_TUNE_PANEL_SMALL_ROWS) {
    *value = knob == LSMS_TUNE_GEMM_F32_NARROW ? ctx->gemm_f32_narrow
             : knob == LSMS_TUNE_GEMM_F64      ? ctx->gemm_f64
             : knob == LSMS_TUNE_GEMM_F64_NARROW ? ctx->gemm_f64_narrow
                                                 : ctx->panel_small_rows;
    return LSMS_OK;
  }
  if (knob != LSMS_TUNE_GEMM_F32) return fail(LSMS_E_ARG, "unknown tuning knob %d", knob);
  *value = gemm_f32_variant(ctx);
  return LSMS_OK;
}

extern "C" int lsms_autotune(lsms_ctx* ctx, int npad, int batch, int* best, float* ms, void* hip_stream) {
  if (!ctx || !best) return fail(LSMS_E_ARG, "NULL argument");
  if (npad % PAD != 0 || npad <= 2 * NB || npad > NL * LSMS_MAX_LIZ)
    return fail(LSMS_E_ARG, "npad %d must be a multiple of %d in (%d, %d]", npad, PAD, 2 * NB, NL * LSMS_MAX_LIZ);
  if (batch < 1 || batch > 65535) return fail(LSMS_E_ARG, "batch %d outside [1, 65535]", batch);
  HIP_TRY(hipSetDevice(ctx->device));
  float t[LSMS_GEMM_F32_VARIANTS];
  int b = -1;
  const int group = pick_tiling(ctx, LSMS_SPLIT, npad).group;
  if (npad <= group * NB)
    return fail(LSMS_E_ARG, "npad %d has no wide update with %d panels per group (needs > %d)", npad, group,
                group * NB);
  if (update_autotune(1, 1, npad, batch, group, (hipStream_t)hip_stream, t, &b) != 0 || b < 0)
    return fail(LSMS_E_NOMEM, "autotuning batch of %d systems of size %d could not run", batch, npad);
  if (t[kDefaultF32Wide] <= 1.01f * t[b]) b = kDefaultF32Wide;  // as lsms_autotune_kernel
  ctx->gemm_f32 = b;
  ctx->tuned[1][1][tune_bucket(npad)] = (int8_t)b;
  *best = b;
  if (ms)
    for (int v = 0; v < LSMS_GEMM_F32_VARIANTS; ++v) ms[v] = t[v];
  return LSMS_OK;
}

extern "C" int lsms_autotune_kernel(lsms_ctx* ctx, int what, int npad, int batch, int* best, float* ms,
                                    int ms_len, void* hip_stream) {
  if (!ctx || !best) return fail(LSMS_E_ARG, "NULL argument");
  if (batch < 1 || batch > 65535) return fail(LSMS_E_ARG, "batch %d outside [1, 65535]", batch);
  hipStream_t s = (hipStream_t)hip_stream;
  HIP_TRY(hipSetDevice(ctx->device));
  if (what == LSMS_AUTOTUNE_F32_PANEL) {
    // both variants at heights the small one can take; the threshold T (panels of at most
    // T rows take the small workgroups) minimises the summed time over the measured
    // heights, as an LU's panels cover every height below its size evenly (0: never)
    const int heights[LSMS_PANEL_HEIGHTS] = {256, 512, PANEL_SMALL_MAX};
    if (ms && ms_len < 2 * LSMS_PANEL_HEIGHTS)
      return fail(LSMS_E_ARG, "ms needs %d entries for the panel autotuner", 2 * LSMS_PANEL_HEIGHTS);
    float t[LSMS_PANEL_HEIGHTS][2];
    for (int h = 0; h < LSMS_PANEL_HEIGHTS; ++h) {
      if (panel_autotune(heights[h], batch, s, t[h]) != 0)
        return fail(LSMS_E_NOMEM, "panel autotuning batch of %d systems of height %d could not run", batch,
                    heights[h]);
      if (ms) {
        ms[2 * h] = t[h][0];
        ms[2 * h + 1] = t[h][1];
      }
    }
    int thr = 0;
    double best_sum = 0.0;
    for (int c = 0; c <= LSMS_PANEL_HEIGHTS; ++c) {  // c heights take the small variant
      double sum = 0.0;
      for (int h = 0; h < LSMS_PANEL_HEIGHTS; ++h) sum += t[h][h < c ? 0 : 1];
      if (c == 0 || sum < best_sum) {
        best_sum = sum;
        thr = c == 0 ? 0 : heights[c - 1];
      }
    }
    ctx->tuned_panel_rows = thr;
    *best = thr;
    return LSMS_OK;
  }
  if (what < LSMS_AUTOTUNE_F32_WIDE || what > LSMS_AUTOTUNE_F64_NARROW)
    return fail(LSMS_E_ARG, "unknown autotuner target %d", what);
  const int precision = (what == LSMS_AUTOTUNE_F32_WIDE || what == LSMS_AUTOTUNE_F32_NARROW) ? 1 : 0;
  const int kind = (what == LSMS_AUTOTUNE_F32_WIDE || what == LSMS_AUTOTUNE_F64_WIDE) ? 1 : 0;
  if (npad % PAD != 0 || npad <= 2 * NB || npad > NL * LSMS_MAX_LIZ)
    return fail(LSMS_E_ARG, "npad %d must be a multiple of %d in (%d, %d]", npad, PAD, 2 * NB, NL * LSMS_MAX_LIZ);
  const int nv = precision ? gemm_f32_variants_all() : gemm_f64_variants();
  if (ms && ms_len < nv) return fail(LSMS_E_ARG, "ms needs %d entries for this autotuner target", nv);
  std::vector<float> t(nv);
  int b = -1;
  const int group = pick_tiling(ctx, precision ? LSMS_SPLIT : LSMS_FP64, npad).group;
  if (npad <= group * NB)
    return fail(LSMS_E_ARG, "npad %d has no %s update with %d panels per group (needs > %d)", npad,
                kind ? "wide" : "narrow", group, group * NB);
  if (update_autotune(precision, kind, npad, batch, group, s, t.data(), &b) != 0 || b < 0)
    return fail(LSMS_E_NOMEM, "autotuning batch of %d systems of size %d could not run", batch, npad);
  // the default stays unless another tiling is faster by more than the spread of repeated
  // timings (1 %): near-ties are decided by noise, and the default's tile order is the one
  // that moves least HBM traffic
  const int def = precision ? (kind ? kDefaultF32Wide : kDefaultF32Narrow) : (kind ? kDefaultF64Wide : kDefaultF64Narrow);
  if (t[def] <= 1.01f * t[b]) b = def;
  ctx->tuned[precision][kind][tune_bucket(npad)] = (int8_t)b;
  *best = b;
  if (ms)
    for (int v = 0; v < nv; ++v) ms[v] = t[v];
  return LSMS_OK;
}

extern "C" int lsms_peak_probe(lsms_ctx* ctx, int what, double* value, void* hip_stream) {
  if (!ctx || !value) return fail(LSMS_E_ARG, "NULL argument");
  if (what < 0 || what > 6) return fail(LSMS_E_ARG, "unknown probe %d", what);
  HIP_TRY(hipSetDevice(ctx->device));
  if (peak_probe(what, ctx->cu_count, (hipStream_t)hip_stream, value) != 0)
    return fail(LSMS_E_DEVICE, "probe %d failed: %s", what, hipGetErrorString(hipGetLastError()));
  return LSMS_OK;
}

extern "C" int lsms_tuning_table(lsms_ctx* ctx, int what, int* out) {
  if (!ctx || !out) return fail(LSMS_E_ARG, "NULL argument");
  if (what == LSMS_AUTOTUNE_F32_PANEL) {
    out[0] = ctx->tuned_panel_rows;
    return LSMS_OK;
  }
  if (what < LSMS_AUTOTUNE_F32_WIDE || what > LSMS_AUTOTUNE_F64_NARROW)
    return fail(LSMS_E_ARG, "unknown autotuner target %d", what);
  const int precision = (what == LSMS_AUTOTUNE_F32_WIDE || what == LSMS_AUTOTUNE_F32_NARROW) ? 1 : 0;
  const int kind = (what == LSMS_AUTOTUNE_F32_WIDE || what == LSMS_AUTOTUNE_F64_WIDE) ? 1 : 0;
  for (int b = 0; b < LSMS_TUNE_BUCKETS; ++b) out[b] = ctx->tuned[precision][kind][b];
  return LSMS_OK;
}

// The cache identifies the device by its architecture name and compute-unit count.
static int device_tag(int device, char* tag, size_t len) {
  hipDeviceProp_t p;
  HIP_TRY(hipGetDeviceProperties(&p, device));
  std::snprintf(tag, len, "%s/%d", p.gcnArchName, p.multiProcessorCount);
  for (char* q = tag; *q; ++q)
    if (*q == ' ') *q = '_';
  return LSMS_OK;
}

extern "C" int lsms_tuning_save(lsms_ctx* ctx, const char* path) {
  if (!ctx || !path) return fail(LSMS_E_ARG, "NULL argument");
  char tag[256];
  int rc = device_tag(ctx->device, tag, sizeof(tag));
  if (rc) return rc;
  FILE* f = std::fopen(path, "w");
  if (!f) return fail(LSMS_E_ARG, "cannot write %s", path);
  std::fprintf(f, "lsms-tune 1 %s\n", tag);
  for (int p = 0; p < 2; ++p)
    for (int k = 0; k < 2; ++k)
      for (int b = 0; b < LSMS_TUNE_BUCKETS; ++b)
        if (ctx->tuned[p][k][b] >= 0) std::fprintf(f, "update %d %d %d %d\n", p, k, b, (int)ctx->tuned[p][k][b]);
  if (ctx->tuned_panel_rows >= 0) std::fprintf(f, "panel %d\n", ctx->tuned_panel_rows);
  // the panels per group the tilings were timed with (explicit settings only)
  if (ctx->group_f64 > 0) std::fprintf(f, "group 0 %d\n", ctx->group_f64);
  if (ctx->group_f32 > 0) std::fprintf(f, "group 1 %d\n", ctx->group_f32);
  const bool ok = std::ferror(f) == 0;
  std::fclose(f);
  return ok ? LSMS_OK : fail(LSMS_E_ARG, "writing %s failed", path);
}

extern "C" int lsms_tuning_load(lsms_ctx* ctx, const char* path) {
  if (!ctx || !path) return fail(LSMS_E_ARG, "NULL argument");
  char tag[256], ftag[256];
  int rc = device_tag(ctx->device, tag, sizeof(tag));
  if (rc) return rc;
  FILE* f = std::fopen(path, "r");
  if (!f) return fail(LSMS_E_ARG, "cannot read %s", path);
  int version = 0;
  if (std::fscanf(f, "lsms-tune %d %255s", &version, ftag) != 2 || version != 1) {
    std::fclose(f);
    return fail(LSMS_E_ARG, "%s is not a tuning cache", path);
  }
  if (std::strcmp(tag, ftag) != 0) {
    std::fclose(f);
    return fail(LSMS_E_STATE, "%s was tuned on %s, this device is %s", path, ftag, tag);
  }
  int8_t tuned[2][2][LSMS_TUNE_BUCKETS];
  std::memset(tuned, -1, sizeof(tuned));
  int panel = -1, group[2] = {-1, -1};
  char word[32];
  while (std::fscanf(f, "%31s", word) == 1) {
    int p, k, b, v;
    if (std::strcmp(word, "update") == 0 && std::fscanf(f, "%d %d %d %d", &p, &k, &b, &v) == 4 && p >= 0 && p < 2 &&
        k >= 0 && k < 2 && b >= 0 && b < LSMS_TUNE_BUCKETS && v >= 0 &&
        v < (p ? gemm_f32_variants_all() : gemm_f64_variants())) {
      tuned[p][k][b] = (int8_t)v;
    } else if (std::strcmp(word, "panel") == 0 && std::fscanf(f, "%d", &v) == 1 && v >= 0 && v <= PANEL_SMALL_MAX) {
      panel = v;
    } else if (std::strcmp(word, "group") == 0 && std::fscanf(f, "%d %d", &p, &v) == 2 && p >= 0 && p < 2 &&
               v >= 2 && v <= GROUP_MAX) {
      group[p] = v;
    } else {
      std::fclose(f);
      return fail(LSMS_E_ARG, "malformed entry in %s", path);
    }
  }
  std::fclose(f);
  std::memcpy(ctx->tuned, tuned, sizeof(tuned));
  ctx->tuned_panel_rows = panel;
  if (group[0] > 0) ctx->group_f64 = group[0];
  if (group[1] > 0) ctx->group_f32 = group[1];
  return LSMS_OK;
}

extern "C" int lsms_set_profiling(lsms_ctx* ctx, int on) {
  if (!ctx) return fail(LSMS_E_ARG, "ctx is NULL");
  HIP_TRY(hipSetDevice(ctx->device));
  HIP_TRY(hipDeviceSynchronize());
  ctx->profiling = on != 0;
  ctx->prof.reset();
  return LSMS_OK;
}

extern "C" int lsms_kernel_stats(lsms_ctx* ctx, int kind, double* total_ms, int64_t* launches, double* alg_flops,
                                 double* alg_bytes) {
  if (!ctx || !total_ms || !launches || !alg_flops || !alg_bytes) return fail(LSMS_E_ARG, "NULL argument");
  if (kind < -1 || kind > 1) return fail(LSMS_E_ARG, "kind %d is not -1, 0 or 1", kind);
  HIP_TRY(hipSetDevice(ctx->device));
  double ms = 0.0, fl = 0.0, by = 0.0;
  int64_t count = 0;
  const size_t n = ctx->prof.flops.size();
  for (size_t i = 0; i < n; ++i) {
    if (kind >= 0 && ctx->prof.kinds[i] != kind) continue;
    ++count;
    hipEvent_t a = ctx->prof.pool[2 * i], b = ctx->prof.pool[2 * i + 1];
    HIP_TRY(hipEventSynchronize(b));
    float e = 0.f;
    HIP_TRY(hipEventElapsedTime(&e, a, b));
    ms += e;
    fl += ctx->prof.flops[i];
    by += ctx->prof.bytes[i];
  }
  *total_ms = ms;
  *launches = count;
  *alg_flops = fl;
  *alg_bytes = by;
  return LSMS_OK;
}

extern "C" int lsms_factors_free(lsms_factors* f) {
  if (!f) return fail(LSMS_E_ARG, "factors is NULL");
  hipSetDevice(f->ctx->device);
  hipDeviceSynchronize();
  if (f->work) hipFree(f->work);
  delete f;
  return LSMS_OK;
}

extern "C" int lsms_kubo_sigma_grad(lsms_ctx* ctx, const lsms_factors* factors, int32_t n_atoms,
                                    const int64_t* liz_ptr, const int32_t* liz_atom, const double* phase,
                                    const void* tau_plus, const void* tau_minus, const int32_t* species,
                                    int32_t n_species, const void* J, double volume, const double* dsigma,
                                    double* dphase, void* hip_stream) {
  if (!ctx || !factors) return fail(LSMS_E_ARG, "ctx or factors is NULL");
  if (factors->ctx != ctx) return fail(LSMS_E_STATE, "factors belong to another context");
  int rc = validate_liz_ptr(n_atoms, liz_ptr);
  if (rc) return rc;
  if (n_atoms != factors->n_atoms || liz_ptr[n_atoms] != factors->total_members)
    return fail(LSMS_E_STATE, "inputs do not match the factored system");
  if (!liz_atom || !phase || !tau_plus || !tau_minus || !species || !J || !dsigma || !dphase)
    return fail(LSMS_E_ARG, "NULL device pointer");
  if (n_species <= 0) return fail(LSMS_E_ARG, "n_species must be positive");
  if (!(volume > 0.0) || !std::isfinite(volume)) return fail(LSMS_E_ARG, "volume must be positive");
  hipStream_t s = (hipStream_t)hip_stream;
  HIP_TRY(hipSetDevice(ctx->device));
  const int nj = (int)factors->jobs.size();
  char* base = (char*)factors->work;
  double2* abuf = (double2*)base;
  double2* xbuf = (double2*)(base + factors->x_base);
  int32_t* piv = (int32_t*)(base + factors->piv_base);
  launch_zero(dphase, (int64_t)n_atoms * 4, s);
  launch_adjoint_rhs(factors->jobs_dev, nj, factors->npad_max, liz_atom, (const double2*)tau_plus,
                     (const double2*)tau_minus, species, n_species, (const double2*)J, dsigma, volume, xbuf, s);
  lu_solve_f64(factors->jobs_dev, nj, factors->npad_max, abuf, piv, xbuf, 0, 32, 1, factors->group, s);
  launch_adjoint_contract(factors->jobs_dev, nj, factors->npad_max, liz_atom, phase, factors->kp, xbuf, dphase, s);
  HIP_TRY(hipGetLastError());
  return LSMS_OK;
}

// ---------------------------------------------------------------------------------
// diagnostic batched LU solve of caller matrices
// ---------------------------------------------------------------------------------
namespace lsms {
void launch_load_user(const JobDesc* jobs, int njobs, int npad_max, void* const* A_dev, void* const* B_dev, int nrhs,
                      int precision, void* work, double2* x, hipStream_t s);
void launch_store_user(const JobDesc* jobs, int njobs, int npad_max, void* const* B_dev, int nrhs, const double2* x,
                       hipStream_t s);
}  // namespace lsms

extern "C" int lsms_batched_lu_solve(lsms_ctx* ctx, int32_t batch, const int32_t* n, void* const* A, void* const* B,
                                     int32_t nrhs, int precision, int32_t* info, void* hip_stream) {
  if (!ctx) return fail(LSMS_E_ARG, "ctx is NULL");
  if (batch <= 0 || !n || !A || !B || !info) return fail(LSMS_E_ARG, "NULL argument or empty batch");
  if (nrhs < 1 || nrhs > 16) return fail(LSMS_E_ARG, "nrhs must be in [1, 16]");
  if (precision != LSMS_FP64 && precision != LSMS_SPLIT) return fail(LSMS_E_ARG, "unknown precision");
  for (int b = 0; b < batch; ++b) {
    if (n[b] < 1 || n[b] > NL * LSMS_MAX_LIZ) return fail(LSMS_E_ARG, "n[%d] = %d out of range", b, n[b]);
    if (!A[b] || !B[b]) return fail(LSMS_E_ARG, "NULL matrix pointer for system %d", b);
  }
  hipStream_t s = (hipStream_t)hip_stream;
  HIP_TRY(hipSetDevice(ctx->device));
  std::vector<JobDesc> jobs(batch);
  int npad_max = 0;
  for (int b = 0; b < batch; ++b) {
    JobDesc j{};
    j.atom = b;
    j.n = n[b];
    j.npad = (int)align_up(n[b], PAD);
    j.nl = (n[b] + NL - 1) / NL;
    npad_max = std::max(npad_max, j.npad);
    jobs[b] = j;
  }
  Wave w{0, batch, 0};
  int64_t ba, bv, bx, br, bp;
  const int prec = precision == LSMS_SPLIT ? LSMS_SPLIT : LSMS_FP64;
  layout_wave(jobs, w, prec, ba, bv, bx, br, bp);  // no refinement here: the table (bv) is not allocated
  const int64_t ptr_bytes = align_up((int64_t)batch * 16, 256);
  const int64_t jd_bytes = align_up((int64_t)batch * sizeof(JobDesc), 256);
  const int64_t total = ba + bx + bp + jd_bytes + 2 * ptr_bytes;
  if (total > (int64_t)ctx->workspace_limit) return fail(LSMS_E_NOMEM, "batch needs %lld bytes", (long long)total);
  int rc = ensure_dev(ctx->work, (size_t)total, s);
  if (rc) return rc;
  const size_t host_bytes = (size_t)jd_bytes + 2 * (size_t)ptr_bytes;
  rc = ensure_pinned(ctx, host_bytes, s);
  if (rc) return rc;
  char* base = (char*)ctx->work.p;
  void* abuf = base;
  double2* xbuf = (double2*)(base + ba);
  int32_t* piv = (int32_t*)(base + ba + bx);
  JobDesc* jd = (JobDesc*)(base + ba + bx + bp);
  void** aptr = (void**)(base + ba + bx + bp + jd_bytes);
  void** bptr = (void**)(base + ba + bx + bp + jd_bytes + ptr_bytes);
  char* hp = (char*)ctx->pinned;
  std::memcpy(hp, jobs.data(), batch * sizeof(JobDesc));
  std::memcpy(hp + jd_bytes, A, batch * sizeof(void*));
  std::memcpy(hp + jd_bytes + ptr_bytes, B, batch * sizeof(void*));
  HIP_TRY(hipMemcpyAsync(jd, hp, (size_t)host_bytes, hipMemcpyHostToDevice, s));
  TallScratch ts;
  rc = tall_scratch(ctx, batch, npad_max, &ts, s);
  if (rc) return rc;
  launch_zero_i32(info, batch, s);
  launch_load_user(jd, batch, npad_max, aptr, bptr, nrhs, prec, abuf, xbuf, s);
  if (prec == LSMS_FP64) {
    const Tiling tl = pick_tiling(ctx, prec, npad_max);
    lu_factor_f64(jd, batch, npad_max, (double2*)abuf, piv, info, s, nullptr, tl, ts);
    lu_solve_f64(jd, batch, npad_max, (const double2*)abuf, piv, xbuf, 0, 16, 0, tl.group, s);
  } else {
    const Tiling tl = pick_tiling(ctx, prec, npad_max);
    lu_factor_f32(jd, batch, npad_max, (float2*)abuf, piv, info, s, nullptr, tl, ts);
    lu_solve_f32(jd, batch, npad_max, (const float2*)abuf, piv, xbuf, 0, 16, 0, tl.group, s);
  }
  launch_store_user(jd, batch, npad_max, bptr, nrhs, xbuf, s);
  HIP_TRY(hipGetLastError());
  // the pinned staging buffer must outlive the upload
  HIP_TRY(hipStreamSynchronize(s));
  return LSMS_OK;
}
