// Host side of the mvpb C-ABI: argument validation, handles, device buffers,
// the k-independent plan build and the batched per-k solve.
#include <math.h>
#include <stdarg.h>
#include <stdlib.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/mvpb.h"
#include "common.h"
#include "kernels.h"
#include "prof.h"

using namespace mvpb;

namespace mvpb {
thread_local Profiler *t_prof = nullptr;
}

// ---------------------------------------------------------------------------
// error state
// ---------------------------------------------------------------------------
static thread_local std::string g_last_error;

static int set_err(int code, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return code;
}

#define HIP_TRY(expr)                                                                        \
  do {                                                                                       \
    hipError_t _e = (expr);                                                                  \
    if (_e != hipSuccess)                                                                    \
      return set_err(MVPB_E_DEVICE, "%s failed: %s (%s:%d)", #expr, hipGetErrorString(_e), __FILE__, \
                     __LINE__);                                                              \
  } while (0)

// Stream-ordered cache of device allocations, one per context.  Every use of
// a context's memory is ordered on the context stream, so a block given back
// by the host may be handed out again at once: the later work that reuses it
// runs after the earlier work that used it.  hipFree (which waits for the
// whole device) only runs when the context goes or an allocation fails.
struct Pool {
  std::multimap<size_t, void *> idle;   // size -> block
  std::map<void *, size_t> size_of;     // every block this pool owns
  ~Pool() { trim(); }
  static size_t round(size_t b) {
    const size_t g = b >= ((size_t)1 << 20) ? ((size_t)1 << 16) : 256;
    return (b + g - 1) / g * g;
  }
  hipError_t get(size_t b, void **out) {
    b = round(b);
    // an idle block of at least b and at most 2 b (or 1 MB for small requests)
    auto it = idle.lower_bound(b);
    if (it != idle.end() && it->first <= std::max(2 * b, (size_t)1 << 20)) {
      *out = it->second;
      idle.erase(it);
      return hipSuccess;
    }
    void *p = nullptr;
    hipError_t e = hipMalloc(&p, b);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      trim();
      e = hipMalloc(&p, b);
      if (e != hipSuccess) return e;
    }
    size_of[p] = b;
    *out = p;
    return hipSuccess;
  }
  void put(void *p) {
    auto it = size_of.find(p);
    if (it != size_of.end()) idle.emplace(it->second, p);
  }
  void trim() {
    for (auto &kv : idle) {
      (void)hipFree(kv.second);
      size_of.erase(kv.second);
    }
    idle.clear();
  }
};

// Device buffer owned by a host object; from the context's pool when one is
// given, else straight from hipMalloc.
struct DevBuf {
  void *p = nullptr;
  size_t bytes = 0;
  Pool *pool = nullptr;
  DevBuf() = default;
  explicit DevBuf(Pool *pl) : pool(pl) {}
  DevBuf(const DevBuf &) = delete;
  DevBuf &operator=(const DevBuf &) = delete;
  ~DevBuf() { release(); }
  void release() {
    if (p) {
      if (pool)
        pool->put(p);
      else
        (void)hipFree(p);
    }
    p = nullptr;
    bytes = 0;
  }
  hipError_t alloc(size_t b) {
    release();
    if (b == 0) return hipSuccess;
    hipError_t e = pool ? pool->get(b, &p) : hipMalloc(&p, b);
    if (e == hipSuccess)
      bytes = b;
    else
      p = nullptr;
    return e;
  }
  // grow-only
  hipError_t reserve(size_t b) {
    if (b <= bytes) return hipSuccess;
    return alloc(b);
  }
  template <typename T>
  T *as() const { return reinterpret_cast<T *>(p); }
};

// Side streams of a context (stage 1 of a solve runs in up to MAX_SIDE + 1
// independent parts, one stream each).
constexpr int MAX_SIDE = 3;

// Launch shape of the eigensolve for one size class of operators (chosen by
// mvpb_autotune or loaded from its cache; defaults otherwise).
struct TuneParams {
  int parts = 1;    // stage-1 parts (each on a stream and a look-ahead stream)
  int group = 0;    // bulge chasing: sweeps per workgroup group (0: 8)
  int wg_max = 0;   // bulge chasing: most workgroups per item (0: 4)
};
// Size class of an operator of order n (the key of the tuning table).
static int size_class(int n) { return (n + 127) / 128; }

struct mvpb_ctx_s {
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  // side streams (owned) for work that overlaps the main stream, and the
  // events of the fork from and the joins back to it
  hipStream_t side[MAX_SIDE] = {};
  hipEvent_t ev_fork = nullptr, ev_join[MAX_SIDE] = {};
  // look-ahead streams of stage 1 (one per part) and the events of a launch
  // sequence's steps (grow-only; a sequence never records one event twice)
  hipStream_t la[MAX_SIDE + 1] = {};
  std::vector<hipEvent_t> la_events;
  size_t cap = 0;
  Pool pool;          // declared before every buffer that returns to it
  DevBuf ws{&pool};      // per-solve workspace (grow-only)
  DevBuf items{&pool};   // item table
  DevBuf scratch{&pool}; // small host-visible results staging
  DevBuf accbuf{&pool};  // one double: largest error estimate of the bands of the current solve
  double acc_tol = 1e-5; // accuracy bar of solves with the FP32 reduction (0: no check)
  double last_acc = 0.0; // largest error estimate of the last synchronous solve
  // Captured launch sequences of the eigensolve, keyed by everything that
  // fixes their launch shapes (item orders, bands, precision, stage-1 parts;
  // see launch_signature).  The kernels find their matrices through the item
  // table, which is uploaded before every replay, so a graph never refers to
  // a plan.  At most MAX_GRAPHS are kept; the least recently used goes first.
  struct GraphEntry {
    hipGraphExec_t exec;
    unsigned long long last_use;
  };
  std::map<std::string, GraphEntry> graphs;
  unsigned long long graph_clock = 0;
  std::vector<EigItem> host_items;                // staging of the item table (kept alive for async copies)
  // mvpb_solve_cells: workspace (plain device allocation, grow-only), its
  // captured graphs (keyed by the call's shape, at most MAX_CELL_GRAPHS) and
  // the staging of the per-call tables
  DevBuf cws;
  std::map<std::string, GraphEntry> cell_graphs;
  std::vector<char> cell_stage;
  std::vector<hipEvent_t> cell_events;            // stage-1 fork/join events, MAX_SIDE + 1 per chunk
  std::map<int, TuneParams> tune;                 // launch shapes by size class
  long long spin_limit = 0;                       // bounded-wait polls of the bulge chasing (0: default)
  Profiler prof;
  int children = 0;     // live cells and plans
  bool closing = false; // mvpb_ctx_destroy called while children were alive
};

static void ctx_free(mvpb_ctx c) {
  (void)hipSetDevice(c->device);
  (void)hipStreamSynchronize(c->stream);
  for (auto &kv : c->graphs) (void)hipGraphExecDestroy(kv.second.exec);
  c->graphs.clear();
  for (auto &kv : c->cell_graphs) (void)hipGraphExecDestroy(kv.second.exec);
  c->cell_graphs.clear();
  for (hipEvent_t ev : c->cell_events) (void)hipEventDestroy(ev);
  c->cell_events.clear();
  c->cws.release();
  c->ws.release();
  c->items.release();
  c->scratch.release();
  c->accbuf.release();
  c->pool.trim();
  c->prof.reset();
  for (int q = 0; q < MAX_SIDE; ++q) {
    if (c->side[q]) {
      (void)hipStreamSynchronize(c->side[q]);
      (void)hipStreamDestroy(c->side[q]);
    }
    if (c->ev_join[q]) (void)hipEventDestroy(c->ev_join[q]);
  }
  for (int q = 0; q <= MAX_SIDE; ++q)
    if (c->la[q]) {
      (void)hipStreamSynchronize(c->la[q]);
      (void)hipStreamDestroy(c->la[q]);
    }
  for (hipEvent_t ev : c->la_events) (void)hipEventDestroy(ev);
  c->la_events.clear();
  if (c->ev_fork) (void)hipEventDestroy(c->ev_fork);
  if (c->own_stream) (void)hipStreamDestroy(c->stream);
  delete c;
}

// A cell or plan releases its hold on the context; the context goes once
// it has been destroyed by the caller and no child is left.
static void ctx_release(mvpb_ctx c) {
  if (--c->children == 0 && c->closing) ctx_free(c);
}

// Routes the kernel timers of the calling thread to a context for one call.
struct ProfBind {
  Profiler *old;
  explicit ProfBind(mvpb_ctx c) : old(t_prof) { t_prof = c ? &c->prof : nullptr; }
  ~ProfBind() { t_prof = old; }
};

struct mvpb_cell_s {
  mvpb_ctx ctx = nullptr;
  double lattice[4];
  double T[4];       // A^-1, row-major
  double area = 0.0;
  int nx = 0, ny = 0, n_phases = 0;
  DevBuf phase;      // int32 [nx*ny] (pixel cells)
  DevBuf wtab;       // double [n_phases][4]
  // polygon cells
  bool polygons = false;
  int n_edges = 0;
  DevBuf edges;      // double [n_edges][4]: midpoint, edge vector
  DevBuf ephase;     // int32 [n_edges]
  double f0[4] = {0.0, 0.0, 0.0, 0.0};   // weighted phase areas (dG = 0)
  // general compliance / spatial cells
  int dim = 2;          // 2: planar cell, 3: voxel cell
  int nz = 1;           // voxels along h3 (1 for planar cells)
  double T3[9] = {};    // A^-1 row-major, dim x dim packed (planar cells: = T)
  bool general = false; // compliance given as a full matrix or spatial cell: only the general plan applies
  int nf = 0;           // weight fields of the general structure factors
  DevBuf gwtab;         // double [n_phases][nf]: Voigt compliance (upper triangle), rho (pixel/voxel cells)
};

struct mvpb_plan_s {
  mvpb_ctx ctx = nullptr;
  int M1 = 0, M2 = 0, N = 0, prec = 0;
  double T[4];
  double area = 0.0;
  DevBuf coef;       // isotropic layout: 15 N x N; general layout: (dim+1)(dim+2)/2 of n x n
  DevBuf linvR;      // N x N, L_R^-1
  DevBuf linvSD;     // 2 N x N: L_Sigma^-1, L_Delta^-1 (stress modes, isotropic layout)
  int dim = 0;       // 0: isotropic planar layout; 2, 3: general layout (full Phi)
  int n = 0;         // displacement unknowns = order of the reduced operator
  int nsig = 0;      // stress unknowns
  int qdim = 2;      // components of a Bloch vector Q
  int M3 = 0;
  double T3[9] = {}; // A^-1 row-major, qdim x qdim packed
  DevBuf linvPhi;    // general layout: L_Phi^-1 (nsig x nsig)
  int gx = 0, gy = 0, gz = 0;   // pixel / voxel grid of the cell (0: polygon cell)
};

namespace mvpb {
int set_error(int code, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return code;
}
hipStream_t ctx_stream(mvpb_ctx c) { return c->stream; }
int ctx_device(mvpb_ctx c) { return c->device; }
bool ctx_closing(mvpb_ctx c) { return c->closing; }
void ctx_retain(mvpb_ctx c) { c->children++; }
void ctx_release_child(mvpb_ctx c) { ctx_release(c); }
}  // namespace mvpb

static hipError_t scratch_setup(int device);   // fixed scratch of the allocation-free call (below)

static int check_ctx(mvpb_ctx c) {
  if (!c) return set_err(MVPB_E_INVALID, "NULL context");
  if (c->closing) return set_err(MVPB_E_INVALID, "context has been destroyed");
  return MVPB_OK;
}

// ---------------------------------------------------------------------------
// basic calls
// ---------------------------------------------------------------------------
extern "C" const char *mvpb_last_error(void) { return g_last_error.c_str(); }

extern "C" const char *mvpb_version(void) { return "mvpb 0.1 (gfx950)"; }

extern "C" int mvpb_ctx_create(int device, void *hip_stream, size_t workspace_cap, mvpb_ctx *out) {
  if (!out) return set_err(MVPB_E_INVALID, "out is NULL");
  int ndev = 0;
  HIP_TRY(hipGetDeviceCount(&ndev));
  if (device < 0 || device >= ndev) return set_err(MVPB_E_INVALID, "device %d out of range [0,%d)", device, ndev);
  HIP_TRY(hipSetDevice(device));
  HIP_TRY(init_kernel_attributes());
  HIP_TRY(scratch_setup(device));
  mvpb_ctx c = new mvpb_ctx_s();
  c->device = device;
  c->cap = workspace_cap;
  if (hip_stream) {
    c->stream = (hipStream_t)hip_stream;
  } else {
    hipError_t e = hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking);
    if (e != hipSuccess) {
      delete c;
      return set_err(MVPB_E_DEVICE, "hipStreamCreate: %s", hipGetErrorString(e));
    }
    c->own_stream = true;
  }
  hipError_t e = hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming);
  for (int q = 0; q < MAX_SIDE && e == hipSuccess; ++q) {
    e = hipStreamCreateWithFlags(&c->side[q], hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&c->ev_join[q], hipEventDisableTiming);
  }
  for (int q = 0; q <= MAX_SIDE && e == hipSuccess; ++q) e = hipStreamCreateWithFlags(&c->la[q], hipStreamNonBlocking);
  // the running error estimate every eigensolve launch sequence updates
  if (e == hipSuccess) e = c->accbuf.reserve(sizeof(double));
  if (e == hipSuccess) e = hipMemsetAsync(c->accbuf.p, 0, sizeof(double), c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) {
    ctx_free(c);
    return set_err(MVPB_E_DEVICE, "context set-up: %s", hipGetErrorString(e));
  }
  *out = c;
  return MVPB_OK;
}

extern "C" int mvpb_ctx_destroy(mvpb_ctx c) {
  if (!c) return MVPB_OK;
  if (c->closing) return set_err(MVPB_E_INVALID, "context destroyed twice");
  if (c->children > 0) {
    c->closing = true;  // freed with its last cell or plan
    return MVPB_OK;
  }
  ctx_free(c);
  return MVPB_OK;
}

// ---------------------------------------------------------------------------
// cell
// ---------------------------------------------------------------------------
static bool lattice_ok(const double *L, double *T, double *area) {
  for (int i = 0; i < 4; ++i)
    if (!isfinite(L[i])) return false;
  const double det = L[0] * L[3] - L[1] * L[2];
  if (!(fabs(det) > 0.0) || !isfinite(det)) return false;
  // A = [[h1x, h1y], [h2x, h2y]]; T = A^-1
  T[0] = L[3] / det;
  T[1] = -L[1] / det;
  T[2] = -L[2] / det;
  T[3] = L[0] / det;
  *area = fabs(det);
  return true;
}

// Weights of the four structure-factor fields per phase (isotropic E, nu,
// rho rows): plane-strain compliances d11 + d12 = 1/(2(lam+mu)) =
// (1+nu)(1-2nu)/E and d11 - d12 = 1/(2 mu) = (1+nu)/E (the shear weight is
// d33 = 2 (d11 - d12)), the density, and 1 (the partition of unity).
static int phase_weight_table(int n_phases, const double *props, std::vector<double> &w) {
  w.assign((size_t)n_phases * 4, 0.0);
  for (int p = 0; p < n_phases; ++p) {
    const double E = props[3 * p], nu = props[3 * p + 1], rho = props[3 * p + 2];
    if (!(E > 0.0) || !isfinite(E)) return set_err(MVPB_E_INVALID, "phase %d: E must be positive", p);
    if (!(nu > -1.0 && nu < 0.5)) return set_err(MVPB_E_INVALID, "phase %d: nu must be in (-1, 0.5)", p);
    if (!(rho > 0.0) || !isfinite(rho)) return set_err(MVPB_E_INVALID, "phase %d: rho must be positive", p);
    w[4 * p + 0] = (1.0 + nu) * (1.0 - 2.0 * nu) / E;
    w[4 * p + 1] = (1.0 + nu) / E;
    w[4 * p + 2] = rho;
    w[4 * p + 3] = 1.0;
  }
  return MVPB_OK;
}

// Engineering-Voigt compliance matrix (the Phi weights c_s c_t D_jkmn of
// Sec. 4.1 eq. (ep), c = 1 on normal and 2 on shear components) of every phase,
// upper triangle row-major, then rho: the weight fields of the general plan.
// dim 2: stress order 11, 22, 12 (plane strain for isotropic rows);
// dim 3: 11, 22, 33, 23, 13, 12.  Rows of kind VOIGT_D_RHO hold the upper
// triangle and rho directly; the matrix must be positive definite.
static int general_weight_table(int dim, int n_phases, int prop_kind, const double *props, std::vector<double> &w,
                                int *nf_out) {
  const int ns = dim == 2 ? 3 : 6, nt = ns * (ns + 1) / 2, nf = nt + 1;
  w.assign((size_t)n_phases * nf, 0.0);
  for (int p = 0; p < n_phases; ++p) {
    double D[6][6] = {};
    double rho;
    if (prop_kind == MVPB_PROP_ISO_E_NU_RHO) {
      const double E = props[3 * p], nu = props[3 * p + 1];
      rho = props[3 * p + 2];
      if (!(E > 0.0) || !isfinite(E)) return set_err(MVPB_E_INVALID, "phase %d: E must be positive", p);
      if (!(nu > -1.0 && nu < 0.5)) return set_err(MVPB_E_INVALID, "phase %d: nu must be in (-1, 0.5)", p);
      if (dim == 2) {   // plane strain
        D[0][0] = D[1][1] = (1.0 + nu) * (1.0 - nu) / E;
        D[0][1] = D[1][0] = -nu * (1.0 + nu) / E;
        D[2][2] = 2.0 * (1.0 + nu) / E;
      } else {
        for (int a = 0; a < 3; ++a)
          for (int b = 0; b < 3; ++b) D[a][b] = (a == b) ? 1.0 / E : -nu / E;
        for (int a = 3; a < 6; ++a) D[a][a] = 2.0 * (1.0 + nu) / E;
      }
    } else {
      const double *r = props + (size_t)p * nf;
      int k = 0;
      for (int a = 0; a < ns; ++a)
        for (int b = a; b < ns; ++b) {
          if (!isfinite(r[k])) return set_err(MVPB_E_INVALID, "phase %d: non-finite compliance", p);
          D[a][b] = D[b][a] = r[k++];
        }
      rho = r[nt];
    }
    if (!(rho > 0.0) || !isfinite(rho)) return set_err(MVPB_E_INVALID, "phase %d: rho must be positive", p);
    // positive definite: Cholesky of the scaled matrix
    double L[6][6] = {};
    for (int j = 0; j < ns; ++j) {
      double dj = D[j][j];
      for (int k = 0; k < j; ++k) dj -= L[j][k] * L[j][k];
      if (!(dj > 1e-12 * D[j][j]) || !(D[j][j] > 0.0))
        return set_err(MVPB_E_INVALID, "phase %d: compliance matrix is not positive definite", p);
      L[j][j] = sqrt(dj);
      for (int i = j + 1; i < ns; ++i) {
        double v = D[i][j];
        for (int k = 0; k < j; ++k) v -= L[i][k] * L[j][k];
        L[i][j] = v / L[j][j];
      }
    }
    double *o = w.data() + (size_t)p * nf;
    int k = 0;
    for (int a = 0; a < ns; ++a)
      for (int b = a; b < ns; ++b) o[k++] = D[a][b];
    o[nt] = rho;
  }
  *nf_out = nf;
  return MVPB_OK;
}

static int prop_stride(int dim, int prop_kind) {
  if (prop_kind == MVPB_PROP_ISO_E_NU_RHO) return 3;
  return dim == 2 ? 7 : 22;
}

extern "C" int mvpb_cell_create_pixels(mvpb_ctx ctx, const double lattice[4], int nx, int ny,
                                       const int32_t *phase, int n_phases, int prop_kind, const double *props,
                                       mvpb_cell *out) {
  int rc = check_ctx(ctx);
  if (rc) return rc;
  if (!lattice || !phase || !props || !out) return set_err(MVPB_E_INVALID, "NULL argument");
  if (nx <= 0 || ny <= 0 || nx > 4096 || ny > 4096) return set_err(MVPB_E_INVALID, "bad grid %d x %d", nx, ny);
  if (n_phases <= 0) return set_err(MVPB_E_INVALID, "n_phases must be positive");
  if (prop_kind != MVPB_PROP_ISO_E_NU_RHO && prop_kind != MVPB_PROP_VOIGT_D_RHO)
    return set_err(MVPB_E_UNSUPPORTED, "property kind %d not supported", prop_kind);
  double T[4], area;
  if (!lattice_ok(lattice, T, &area)) return set_err(MVPB_E_INVALID, "degenerate or non-finite lattice");
  for (size_t i = 0; i < (size_t)nx * ny; ++i)
    if (phase[i] < 0 || phase[i] >= n_phases)
      return set_err(MVPB_E_INVALID, "phase id %d at pixel %zu out of range [0,%d)", phase[i], i, n_phases);
  const bool iso = prop_kind == MVPB_PROP_ISO_E_NU_RHO;
  std::vector<double> w, gw;
  if (iso) {
    rc = phase_weight_table(n_phases, props, w);
    if (rc) return rc;
  }
  int nf = 0;
  rc = general_weight_table(2, n_phases, prop_kind, props, gw, &nf);
  if (rc) return rc;
  HIP_TRY(hipSetDevice(ctx->device));
  mvpb_cell c = new mvpb_cell_s();
  c->ctx = ctx;
  memcpy(c->lattice, lattice, sizeof c->lattice);
  memcpy(c->T, T, sizeof T);
  memcpy(c->T3, T, sizeof T);
  c->area = area;
  c->nx = nx;
  c->ny = ny;
  c->n_phases = n_phases;
  c->general = !iso;
  c->nf = nf;
  c->phase.pool = &ctx->pool;
  c->wtab.pool = &ctx->pool;
  c->gwtab.pool = &ctx->pool;
  hipError_t e = c->phase.alloc(sizeof(int32_t) * nx * ny);
  if (e == hipSuccess && iso) e = c->wtab.alloc(sizeof(double) * w.size());
  if (e == hipSuccess) e = c->gwtab.alloc(sizeof(double) * gw.size());
  if (e == hipSuccess)
    e = hipMemcpyAsync(c->phase.p, phase, sizeof(int32_t) * nx * ny, hipMemcpyHostToDevice, ctx->stream);
  if (e == hipSuccess && iso)
    e = hipMemcpyAsync(c->wtab.p, w.data(), sizeof(double) * w.size(), hipMemcpyHostToDevice, ctx->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(c->gwtab.p, gw.data(), sizeof(double) * gw.size(), hipMemcpyHostToDevice, ctx->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
  if (e != hipSuccess) {
    delete c;
    return set_err(MVPB_E_NOMEM, "cell upload: %s", hipGetErrorString(e));
  }
  ctx->children++;
  *out = c;
  return MVPB_OK;
}

// A = rows h1, h2, h3; T = A^-1 (row-major), vol = |det A|.
static bool lattice3_ok(const double *L, double *T, double *vol) {
  for (int i = 0; i < 9; ++i)
    if (!isfinite(L[i])) return false;
  const double c00 = L[4] * L[8] - L[5] * L[7], c01 = L[5] * L[6] - L[3] * L[8], c02 = L[3] * L[7] - L[4] * L[6];
  const double det = L[0] * c00 + L[1] * c01 + L[2] * c02;
  if (!(fabs(det) > 0.0) || !isfinite(det)) return false;
  // inverse = adjugate / det (adjugate = transpose of the cofactor matrix)
  T[0] = c00 / det;
  T[3] = c01 / det;
  T[6] = c02 / det;
  T[1] = (L[2] * L[7] - L[1] * L[8]) / det;
  T[4] = (L[0] * L[8] - L[2] * L[6]) / det;
  T[7] = (L[1] * L[6] - L[0] * L[7]) / det;
  T[2] = (L[1] * L[5] - L[2] * L[4]) / det;
  T[5] = (L[2] * L[3] - L[0] * L[5]) / det;
  T[8] = (L[0] * L[4] - L[1] * L[3]) / det;
  *vol = fabs(det);
  return true;
}

extern "C" int mvpb_cell_create_voxels(mvpb_ctx ctx, const double lattice[9], int nx, int ny, int nz,
                                       const int32_t *phase, int n_phases, int prop_kind, const double *props,
                                       mvpb_cell *out) {
  int rc = check_ctx(ctx);
  if (rc) return rc;
  if (!lattice || !phase || !props || !out) return set_err(MVPB_E_INVALID, "NULL argument");
  if (nx <= 0 || ny <= 0 || nz <= 0 || nx > 1024 || ny > 1024 || nz > 1024 || (long)nx * ny * nz > (1L << 26))
    return set_err(MVPB_E_INVALID, "bad grid %d x %d x %d", nx, ny, nz);
  if (n_phases <= 0) return set_err(MVPB_E_INVALID, "n_phases must be positive");
  if (prop_kind != MVPB_PROP_ISO_E_NU_RHO && prop_kind != MVPB_PROP_VOIGT_D_RHO)
    return set_err(MVPB_E_UNSUPPORTED, "property kind %d not supported", prop_kind);
  double T[9], vol;
  if (!lattice3_ok(lattice, T, &vol)) return set_err(MVPB_E_INVALID, "degenerate or non-finite lattice");
  const size_t nvox = (size_t)nx * ny * nz;
  for (size_t i = 0; i < nvox; ++i)
    if (phase[i] < 0 || phase[i] >= n_phases)
      return set_err(MVPB_E_INVALID, "phase id %d at voxel %zu out of range [0,%d)", phase[i], i, n_phases);
  std::vector<double> gw;
  int nf = 0;
  rc = general_weight_table(3, n_phases, prop_kind, props, gw, &nf);
  if (rc) return rc;
  HIP_TRY(hipSetDevice(ctx->device));
  mvpb_cell c = new mvpb_cell_s();
  c->ctx = ctx;
  c->dim = 3;
  memcpy(c->T3, T, sizeof T);
  c->area = vol;
  c->nx = nx;
  c->ny = ny;
  c->nz = nz;
  c->n_phases = n_phases;
  c->general = true;
  c->nf = nf;
  c->phase.pool = &ctx->pool;
  c->gwtab.pool = &ctx->pool;
  hipError_t e = c->phase.alloc(sizeof(int32_t) * nvox);
  if (e == hipSuccess) e = c->gwtab.alloc(sizeof(double) * gw.size());
  if (e == hipSuccess) e = hipMemcpyAsync(c->phase.p, phase, sizeof(int32_t) * nvox, hipMemcpyHostToDevice, ctx->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(c->gwtab.p, gw.data(), sizeof(double) * gw.size(), hipMemcpyHostToDevice, ctx->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
  if (e != hipSuccess) {
    delete c;
    return set_err(MVPB_E_NOMEM, "cell upload: %s", hipGetErrorString(e));
  }
  ctx->children++;
  *out = c;
  return MVPB_OK;
}

extern "C" int mvpb_cell_create_polygons(mvpb_ctx ctx, const double lattice[4], int n_polys,
                                         const int32_t *poly_phase, const int32_t *vert_offset, const double *xy,
                                         int n_phases, int prop_kind, const double *props, mvpb_cell *out) {
  int rc = check_ctx(ctx);
  if (rc) return rc;
  if (!lattice || !poly_phase || !vert_offset || !xy || !props || !out)
    return set_err(MVPB_E_INVALID, "NULL argument");
  if (n_polys <= 0) return set_err(MVPB_E_INVALID, "n_polys must be positive");
  if (n_phases <= 0) return set_err(MVPB_E_INVALID, "n_phases must be positive");
  if (prop_kind != MVPB_PROP_ISO_E_NU_RHO)
    return set_err(MVPB_E_UNSUPPORTED, "property kind %d not supported", prop_kind);
  double T[4], area;
  if (!lattice_ok(lattice, T, &area)) return set_err(MVPB_E_INVALID, "degenerate or non-finite lattice");
  if (vert_offset[0] != 0) return set_err(MVPB_E_INVALID, "vert_offset[0] must be 0");
  std::vector<double> eg;
  std::vector<int32_t> ep;
  std::vector<double> aph((size_t)n_phases, 0.0);
  double total = 0.0;
  for (int i = 0; i < n_polys; ++i) {
    const int v0 = vert_offset[i], v1 = vert_offset[i + 1], nv = v1 - v0;
    if (nv < 3) return set_err(MVPB_E_INVALID, "polygon %d has %d vertices (at least 3)", i, nv);
    const int ph = poly_phase[i];
    if (ph < 0 || ph >= n_phases)
      return set_err(MVPB_E_INVALID, "polygon %d: phase id %d out of range [0,%d)", i, ph, n_phases);
    double a2 = 0.0;   // twice the signed area (shoelace)
    for (int k = 0; k < nv; ++k) {
      const double *pa = xy + 2 * (size_t)(v0 + k), *pb = xy + 2 * (size_t)(v0 + (k + 1) % nv);
      if (!isfinite(pa[0]) || !isfinite(pa[1])) return set_err(MVPB_E_INVALID, "polygon %d: non-finite vertex", i);
      a2 += pa[0] * pb[1] - pb[0] * pa[1];
      eg.push_back(0.5 * (pa[0] + pb[0]));
      eg.push_back(0.5 * (pa[1] + pb[1]));
      eg.push_back(pb[0] - pa[0]);
      eg.push_back(pb[1] - pa[1]);
      ep.push_back(ph);
    }
    aph[ph] += 0.5 * a2;
    total += 0.5 * a2;
  }
  // the phases partition the cell: signed areas add up to |Omega|, none negative
  const double tol = 1e-9 * area;
  if (fabs(total - area) > tol)
    return set_err(MVPB_E_INVALID, "polygons must tile the unit cell: signed area %.12g, cell area %.12g", total,
                   area);
  for (int p = 0; p < n_phases; ++p)
    if (aph[p] < -tol) return set_err(MVPB_E_INVALID, "phase %d has negative signed area %.6g", p, aph[p]);
  std::vector<double> w;
  rc = phase_weight_table(n_phases, props, w);
  if (rc) return rc;
  HIP_TRY(hipSetDevice(ctx->device));
  mvpb_cell c = new mvpb_cell_s();
  c->ctx = ctx;
  memcpy(c->lattice, lattice, sizeof c->lattice);
  memcpy(c->T, T, sizeof T);
  c->area = area;
  c->n_phases = n_phases;
  c->polygons = true;
  c->n_edges = (int)ep.size();
  for (int k = 0; k < 4; ++k) {
    double f = 0.0;
    for (int p = 0; p < n_phases; ++p) f += w[4 * p + k] * aph[p];
    c->f0[k] = f;
  }
  c->wtab.pool = &ctx->pool;
  c->edges.pool = &ctx->pool;
  c->ephase.pool = &ctx->pool;
  hipError_t e = c->wtab.alloc(sizeof(double) * w.size());
  if (e == hipSuccess) e = c->edges.alloc(sizeof(double) * eg.size());
  if (e == hipSuccess) e = c->ephase.alloc(sizeof(int32_t) * ep.size());
  if (e == hipSuccess)
    e = hipMemcpyAsync(c->wtab.p, w.data(), sizeof(double) * w.size(), hipMemcpyHostToDevice, ctx->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(c->edges.p, eg.data(), sizeof(double) * eg.size(), hipMemcpyHostToDevice, ctx->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(c->ephase.p, ep.data(), sizeof(int32_t) * ep.size(), hipMemcpyHostToDevice, ctx->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
  if (e != hipSuccess) {
    delete c;
    return set_err(MVPB_E_NOMEM, "cell upload: %s", hipGetErrorString(e));
  }
  ctx->children++;
  *out = c;
  return MVPB_OK;
}

extern "C" int mvpb_cell_destroy(mvpb_cell c) {
  if (!c) return MVPB_OK;
  mvpb_ctx ctx = c->ctx;
  (void)hipSetDevice(ctx->device);
  (void)hipStreamSynchronize(ctx->stream);
  delete c;
  ctx_release(ctx);
  return MVPB_OK;
}

// ---------------------------------------------------------------------------
// structure factors
// ---------------------------------------------------------------------------
static int run_structure_factors(mvpb_cell c, int M1, int M2, int precision, DevBuf &X, DevBuf &F) {
  const int nm = 4 * M1 + 1, nq = 4 * M2 + 1;
  const size_t plain = sizeof(cd) * 4 * (size_t)std::max(c->nx, c->ny) * std::max(nm, nq);
  const size_t mfma = sizeof(double) * 8 * (size_t)c->nx * nq;
  HIP_TRY(X.reserve(std::max(plain, mfma)));
  HIP_TRY(F.reserve(sizeof(cd) * 4 * (size_t)nm * nq));
  hipStream_t st = c->ctx->stream;
  if (c->polygons) {
    // closed-form edge sums in FP64 for every precision setting
    HIP_TRY(X.reserve(sf_poly_scratch_bytes(c->n_edges, M1, M2)));
    HIP_TRY(launch_structure_factors_poly(c->edges.as<double>(), c->ephase.as<int32_t>(), c->wtab.as<double>(),
                                          c->n_edges, c->T, c->f0, M1, M2, X.as<cd>(), F.as<cd>(), st));
  } else if (precision & MVPB_PREC_SF_PLAIN64) {
    HIP_TRY(launch_structure_factors_f64(c->phase.as<int32_t>(), c->wtab.as<double>(), c->nx, c->ny, M1, M2,
                                         c->area, X.as<cd>(), F.as<cd>(), st));
  } else {
    const int sf = precision & 3;  // 0: FP64, 1: FP32, 2: BF16, 3: split-BF16 matrix-core contraction
    HIP_TRY(launch_structure_factors_mfma(sf, c->phase.as<int32_t>(), c->wtab.as<double>(), c->nx, c->ny, M1, M2,
                                          c->area, X.as<double>(), F.as<cd>(), st));
  }
  return MVPB_OK;
}

static int check_precision(int precision) {
  const int sf = precision & 3;
  if ((precision & ~31) || ((precision & MVPB_PREC_SF_PLAIN64) && sf))
    return set_err(MVPB_E_INVALID, "bad precision flags %d", precision);
  return MVPB_OK;
}

static int check_cutoff(int M1, int M2) {
  if (M1 < 0 || M2 < 0) return set_err(MVPB_E_INVALID, "cutoffs must be non-negative");
  const long N = (long)(2 * M1 + 1) * (2 * M2 + 1);
  if (2 * N > MAX_N) return set_err(MVPB_E_UNSUPPORTED, "2N = %ld exceeds %d", 2 * N, MAX_N);
  return MVPB_OK;
}

extern "C" int mvpb_structure_factors(mvpb_cell c, int M1, int M2, int precision, double *F) {
  if (!c || !F) return set_err(MVPB_E_INVALID, "NULL argument");
  if (c->general)
    return set_err(MVPB_E_UNSUPPORTED, "cell has a general compliance or is spatial: use mvpb_structure_factors_general");
  int rc = check_cutoff(M1, M2);
  if (rc) return rc;
  rc = check_precision(precision);
  if (rc) return rc;
  HIP_TRY(hipSetDevice(c->ctx->device));
  ProfBind pb(c->ctx);
  DevBuf X(&c->ctx->pool), Fd(&c->ctx->pool);
  rc = run_structure_factors(c, M1, M2, precision, X, Fd);
  if (rc) return rc;
  const size_t cnt = 4 * (size_t)(4 * M1 + 1) * (4 * M2 + 1);
  HIP_TRY(hipMemcpyAsync(F, Fd.p, sizeof(cd) * cnt, hipMemcpyDeviceToHost, c->ctx->stream));
  HIP_TRY(hipStreamSynchronize(c->ctx->stream));
  return MVPB_OK;
}

static int check_cutoff3(const mvpb_cell c, int M1, int M2, int M3) {
  if (M1 < 0 || M2 < 0 || M3 < 0) return set_err(MVPB_E_INVALID, "cutoffs must be non-negative");
  if (c->dim == 2 && M3 != 0) return set_err(MVPB_E_INVALID, "a planar cell takes M3 = 0");
  const long N = (long)(2 * M1 + 1) * (2 * M2 + 1) * (2 * M3 + 1);
  if (c->dim * N > MAX_N) return set_err(MVPB_E_UNSUPPORTED, "%d N = %ld exceeds %d", c->dim, c->dim * N, MAX_N);
  return MVPB_OK;
}

// Weight fields of the general plan on the difference grid (pixel and voxel cells).
static int run_structure_factors_general(mvpb_cell c, int M1, int M2, int M3, DevBuf &X1, DevBuf &X2, DevBuf &F) {
  if (c->polygons) return set_err(MVPB_E_UNSUPPORTED, "general compliance is not available for polygon cells");
  const size_t nm = 4 * M1 + 1, nq = 4 * M2 + 1, nr = 4 * M3 + 1, nf = c->nf;
  HIP_TRY(X1.reserve(sizeof(cd) * nf * c->nx * c->ny * nr));
  HIP_TRY(X2.reserve(sizeof(cd) * nf * c->nx * nq * nr));
  HIP_TRY(F.reserve(sizeof(cd) * nf * nm * nq * nr));
  HIP_TRY(launch_structure_factors_general(c->phase.as<int32_t>(), c->gwtab.as<double>(), c->nf, c->nx, c->ny, c->nz,
                                           M1, M2, M3, c->area, X1.as<cd>(), X2.as<cd>(), F.as<cd>(), c->ctx->stream));
  return MVPB_OK;
}

extern "C" int mvpb_structure_factors_general(mvpb_cell c, int M1, int M2, int M3, double *F) {
  if (!c || !F) return set_err(MVPB_E_INVALID, "NULL argument");
  int rc = check_cutoff3(c, M1, M2, M3);
  if (rc) return rc;
  HIP_TRY(hipSetDevice(c->ctx->device));
  ProfBind pb(c->ctx);
  DevBuf X1(&c->ctx->pool), X2(&c->ctx->pool), Fd(&c->ctx->pool);
  rc = run_structure_factors_general(c, M1, M2, M3, X1, X2, Fd);
  if (rc) return rc;
  const size_t cnt = (size_t)c->nf * (4 * M1 + 1) * (4 * M2 + 1) * (4 * M3 + 1);
  HIP_TRY(hipMemcpyAsync(F, Fd.p, sizeof(cd) * cnt, hipMemcpyDeviceToHost, c->ctx->stream));
  HIP_TRY(hipStreamSynchronize(c->ctx->stream));
  return MVPB_OK;
}

// ---------------------------------------------------------------------------
// Structure factors without allocation: the scratch of the two DFT passes
// lives in a fixed file-scope device array; each device holds its own copy,
// whose address is looked up once per device when a context is created there.
// ---------------------------------------------------------------------------
constexpr size_t SF_SCRATCH_BYTES = (size_t)16 << 20;
static __device__ __align__(256) char scratch[SF_SCRATCH_BYTES];
constexpr int SCRATCH_DEVICES = 64;
static void *g_scratch_ptr[SCRATCH_DEVICES];   // device address of `scratch` per device (NULL: not looked up)
static std::mutex g_scratch_mu;

// With `device` current: record the device address of its scratch array.
static hipError_t scratch_setup(int device) {
  if (device < 0 || device >= SCRATCH_DEVICES) return hipSuccess;   // the allocation-free call then refuses
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_ptr[device]) return hipSuccess;
  void *ptr = nullptr;
  hipError_t e = hipGetSymbolAddress((void **)&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  g_scratch_ptr[device] = ptr;
  return hipSuccess;
}

// Bytes of pass scratch the structure factors of cell c at (M1, M2) need.
static size_t sf_scratch_need(mvpb_cell c, int M1, int M2, int precision) {
  const size_t nq = (size_t)(4 * M2 + 1);
  if (c->polygons) return sf_poly_scratch_bytes(c->n_edges, M1, M2);
  if (precision & MVPB_PREC_SF_PLAIN64) return sizeof(cd) * 4 * (size_t)c->nx * nq;
  return sizeof(double) * 8 * (size_t)c->nx * nq;
}

extern "C" int mvpb_structure_factors_noalloc(mvpb_cell c, int M1, int M2, int precision, double *F,
                                              unsigned flags) {
  if (!c || !F) return set_err(MVPB_E_INVALID, "NULL argument");
  if (c->general) return set_err(MVPB_E_UNSUPPORTED, "cell has a general compliance or is spatial");
  int rc = check_cutoff(M1, M2);
  if (rc) return rc;
  rc = check_precision(precision);
  if (rc) return rc;
  mvpb_ctx ctx = c->ctx;
  if (ctx->device < 0 || ctx->device >= SCRATCH_DEVICES || !g_scratch_ptr[ctx->device])
    return set_err(MVPB_E_UNSUPPORTED, "no fixed scratch on device %d", ctx->device);
  const size_t need = sf_scratch_need(c, M1, M2, precision);
  if (need > SF_SCRATCH_BYTES)
    return set_err(MVPB_E_NOMEM, "structure factors at M = (%d, %d) need %zu bytes of scratch; the fixed scratch holds %zu",
                   M1, M2, need, SF_SCRATCH_BYTES);
  HIP_TRY(hipSetDevice(ctx->device));
  ProfBind pb(nullptr);   // no timer events (they are created on demand)
  void *ptr = g_scratch_ptr[ctx->device];
  hipStream_t st = ctx->stream;
  if (c->polygons) {
    HIP_TRY(launch_structure_factors_poly(c->edges.as<double>(), c->ephase.as<int32_t>(), c->wtab.as<double>(),
                                          c->n_edges, c->T, c->f0, M1, M2, (cd *)ptr, (cd *)F, st));
  } else if (precision & MVPB_PREC_SF_PLAIN64) {
    HIP_TRY(launch_structure_factors_f64(c->phase.as<int32_t>(), c->wtab.as<double>(), c->nx, c->ny, M1, M2,
                                         c->area, (cd *)ptr, (cd *)F, st));
  } else {
    HIP_TRY(launch_structure_factors_mfma(precision & 3, c->phase.as<int32_t>(), c->wtab.as<double>(), c->nx, c->ny,
                                          M1, M2, c->area, (double *)ptr, (cd *)F, st));
  }
  if (!(flags & MVPB_F_ASYNC)) HIP_TRY(hipStreamSynchronize(st));
  return MVPB_OK;
}

// ---------------------------------------------------------------------------
// plan
// ---------------------------------------------------------------------------
// Build the plans of g cells that share the cutoff (M1, M2): structure
// factors and Toeplitz scatter per cell, then one factorisation launch for
// all 3g matrices and two batched GEMM launches.  On error every plan built
// here is released and none is returned.
static int build_plan_group(mvpb_ctx ctx, const mvpb_cell *cells, int g, int M1, int M2, int precision,
                            mvpb_plan *out, int index_base) {
  hipStream_t st = ctx->stream;
  const int N = (2 * M1 + 1) * (2 * M2 + 1);
  const size_t NN = (size_t)N * N;
  const int nm = 4 * M1 + 1, nq = 4 * M2 + 1;
  const size_t fsz = (size_t)4 * nm * nq;

  Pool *pool = &ctx->pool;
  DevBuf X(pool), F1(pool), F(pool), mats(pool), linv(pool), stat(pool), ptrs(pool), gvec(pool), P(pool), Xp(pool);
  HIP_TRY(F.alloc(sizeof(cd) * fsz * g));
  HIP_TRY(mats.alloc(sizeof(cd) * 3 * NN * g));
  HIP_TRY(linv.alloc(sizeof(cd) * 3 * NN * g));
  HIP_TRY(stat.alloc(sizeof(int) * 3 * g));
  HIP_TRY(P.alloc(sizeof(cd) * 6 * NN * g));
  HIP_TRY(Xp.alloc(sizeof(cd) * 18 * NN * g));
  cd *Tm = mats.as<cd>(), *Li = linv.as<cd>(), *Pm = P.as<cd>(), *Xm = Xp.as<cd>();
  // structure factors: runs of pixel cells on one grid in one launch pair on
  // the matrix cores, other cells one by one
  {
    DevBuf tabs(pool);
    int c = 0;
    while (c < g) {
      const mvpb_cell c0 = cells[c];
      int c1 = c + 1;
      const bool batchable = !c0->polygons && !(precision & MVPB_PREC_SF_PLAIN64);
      while (batchable && c1 < g && !cells[c1]->polygons && cells[c1]->nx == c0->nx && cells[c1]->ny == c0->ny) ++c1;
      if (batchable && c1 - c > 1) {
        const int cnt = c1 - c;
        std::vector<const void *> tb;
        for (int k = c; k < c1; ++k) tb.push_back(cells[k]->phase.p);
        for (int k = c; k < c1; ++k) tb.push_back(cells[k]->wtab.p);
        std::vector<double> areas(cnt);
        for (int k = 0; k < cnt; ++k) areas[k] = cells[c + k]->area;
        const size_t tbytes = sizeof(void *) * tb.size();
        HIP_TRY(tabs.reserve(tbytes + sizeof(double) * cnt));
        HIP_TRY(hipMemcpyAsync(tabs.p, tb.data(), tbytes, hipMemcpyHostToDevice, st));
        HIP_TRY(hipMemcpyAsync(tabs.as<char>() + tbytes, areas.data(), sizeof(double) * cnt, hipMemcpyHostToDevice,
                               st));
        HIP_TRY(X.reserve(sizeof(double) * 8 * (size_t)c0->nx * (4 * M2 + 1) * cnt));
        void **tp = tabs.as<void *>();
        HIP_TRY(launch_structure_factors_mfma_batch(precision & 3, (const int32_t *const *)tp,
                                                    (const double *const *)(tp + cnt),
                                                    (const double *)(tabs.as<char>() + tbytes), cnt, c0->nx, c0->ny,
                                                    M1, M2, X.as<double>(), F.as<cd>() + c * fsz, st));
      } else {
        for (int k = c; k < c1; ++k) {
          int rc = run_structure_factors(cells[k], M1, M2, precision, X, F1);
          if (rc) return rc;
          HIP_TRY(hipMemcpyAsync(F.as<cd>() + k * fsz, F1.p, sizeof(cd) * fsz, hipMemcpyDeviceToDevice, st));
        }
      }
      c = c1;
    }
  }
  // Sigma = T(d11+d12), Delta = T(d11-d12), R = T(rho) of every cell in one launch
  HIP_TRY(launch_toeplitz_scatter(F.as<cd>(), M1, M2, N, Tm, g, st));
  // G_l vectors per cell: G_0 = 1, G_l = 2 pi (T n)_l at Q = 0
  std::vector<double> gv(3 * (size_t)N * g);
  for (int c = 0; c < g; ++c)
    for (int a = -M1; a <= M1; ++a)
      for (int b = -M2; b <= M2; ++b) {
        const int r = (a + M1) * (2 * M2 + 1) + (b + M2);
        double *gc = gv.data() + 3 * (size_t)N * c;
        gc[r] = 1.0;
        gc[N + r] = 2.0 * M_PI * (cells[c]->T[0] * a + cells[c]->T[1] * b);
        gc[2 * N + r] = 2.0 * M_PI * (cells[c]->T[2] * a + cells[c]->T[3] * b);
      }
  HIP_TRY(gvec.alloc(sizeof(double) * gv.size()));
  HIP_TRY(hipMemcpyAsync(gvec.p, gv.data(), sizeof(double) * gv.size(), hipMemcpyHostToDevice, st));
  // pointer tables
  std::vector<void *> hp;
  for (int c = 0; c < g; ++c)
    for (int i = 0; i < 3; ++i) hp.push_back(Tm + (3 * c + i) * NN);
  const size_t o_inv = hp.size();
  for (int c = 0; c < g; ++c)
    for (int i = 0; i < 3; ++i) hp.push_back(Li + (3 * c + i) * NN);
  // P_{x,l} = L_R^-1 diag(G_l) L_x^-H   (x = 0: Sigma, 1: Delta)
  const size_t o_pA = hp.size();
  for (int c = 0; c < g; ++c)
    for (int x = 0; x < 2; ++x)
      for (int l = 0; l < 3; ++l) hp.push_back(Li + (3 * c + 2) * NN);
  const size_t o_pB = hp.size();
  for (int c = 0; c < g; ++c)
    for (int x = 0; x < 2; ++x)
      for (int l = 0; l < 3; ++l) hp.push_back(Li + (3 * c + x) * NN);
  const size_t o_pC = hp.size();
  for (int c = 0; c < g; ++c)
    for (int x = 0; x < 2; ++x)
      for (int l = 0; l < 3; ++l) hp.push_back(Pm + (6 * c + x * 3 + l) * NN);
  const size_t o_pS = hp.size();
  for (int c = 0; c < g; ++c)
    for (int x = 0; x < 2; ++x)
      for (int l = 0; l < 3; ++l) hp.push_back(gvec.as<double>() + 3 * (size_t)N * c + l * N);
  // X_{x,l,m} = P_{x,l} P_{x,m}^H
  const size_t o_xA = hp.size();
  for (int c = 0; c < g; ++c)
    for (int x = 0; x < 2; ++x)
      for (int l = 0; l < 3; ++l)
        for (int m = 0; m < 3; ++m) hp.push_back(Pm + (6 * c + x * 3 + l) * NN);
  const size_t o_xB = hp.size();
  for (int c = 0; c < g; ++c)
    for (int x = 0; x < 2; ++x)
      for (int l = 0; l < 3; ++l)
        for (int m = 0; m < 3; ++m) hp.push_back(Pm + (6 * c + x * 3 + m) * NN);
  const size_t o_xC = hp.size();
  for (int c = 0; c < g; ++c)
    for (int x = 0; x < 2; ++x)
      for (int l = 0; l < 3; ++l)
        for (int m = 0; m < 3; ++m) hp.push_back(Xm + (18 * c + x * 9 + l * 3 + m) * NN);
  HIP_TRY(ptrs.alloc(sizeof(void *) * hp.size()));
  HIP_TRY(hipMemcpyAsync(ptrs.p, hp.data(), sizeof(void *) * hp.size(), hipMemcpyHostToDevice, st));
  void **dp = ptrs.as<void *>();

  HIP_TRY(launch_potrf_trtri((cd *const *)dp, (cd *const *)(dp + o_inv), stat.as<int>(), 3 * g, N, st));
  std::vector<int> hstat(3 * g, 0);
  HIP_TRY(hipMemcpyAsync(hstat.data(), stat.p, sizeof(int) * 3 * g, hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  const char *names[3] = {"compliance block Phi(d11+d12)", "compliance block Phi(d11-d12)", "density matrix Omega"};
  for (int i = 0; i < 3 * g; ++i)
    if (hstat[i])
      return set_err(MVPB_E_NOT_PD, "cell %d: %s is not positive definite (pivot %d)", index_base + i / 3,
                     names[i % 3], hstat[i] - 1);
  {
    GemmBatch bt{(const cd *const *)(dp + o_pA), (const cd *const *)(dp + o_pB), (cd *const *)(dp + o_pC),
                 (const double *const *)(dp + o_pS), N, N, N};
    HIP_TRY(launch_zgemm(OP_N, OP_C, N, N, N, mk(1.0, 0.0), bt, mk(0.0, 0.0), 6 * g, st));
  }
  {
    GemmBatch bt{(const cd *const *)(dp + o_xA), (const cd *const *)(dp + o_xB), (cd *const *)(dp + o_xC),
                 nullptr, N, N, N};
    HIP_TRY(launch_zgemm(OP_N, OP_C, N, N, N, mk(1.0, 0.0), bt, mk(0.0, 0.0), 18 * g, st));
  }
  std::vector<mvpb_plan> made;
  hipError_t e = hipSuccess;
  for (int c = 0; c < g && e == hipSuccess; ++c) {
    mvpb_plan pl = new mvpb_plan_s();
    pl->ctx = ctx;
    pl->M1 = M1;
    pl->M2 = M2;
    pl->N = N;
    pl->n = 2 * N;
    pl->nsig = 3 * N;
    if (!cells[c]->polygons) {
      pl->gx = cells[c]->nx;
      pl->gy = cells[c]->ny;
      pl->gz = 1;
    }
    pl->prec = precision;
    memcpy(pl->T, cells[c]->T, sizeof pl->T);
    memcpy(pl->T3, cells[c]->T, sizeof pl->T);
    pl->area = cells[c]->area;
    pl->coef.pool = &ctx->pool;
    pl->linvR.pool = &ctx->pool;
    pl->linvSD.pool = &ctx->pool;
    made.push_back(pl);
    e = pl->coef.alloc(sizeof(cd) * 15 * NN);
    if (e == hipSuccess) e = pl->linvR.alloc(sizeof(cd) * NN);
    if (e == hipSuccess) e = pl->linvSD.alloc(sizeof(cd) * 2 * NN);
    if (e == hipSuccess)
      e = hipMemcpyAsync(pl->linvSD.p, Li + (3 * c + 0) * NN, sizeof(cd) * 2 * NN, hipMemcpyDeviceToDevice, st);
    if (e == hipSuccess) e = launch_combine(Xm + 18 * NN * c, N, 0.5 * pl->area * pl->area, pl->coef.as<cd>(), st);
    if (e == hipSuccess)
      e = hipMemcpyAsync(pl->linvR.p, Li + (3 * c + 2) * NN, sizeof(cd) * NN, hipMemcpyDeviceToDevice, st);
  }
  if (e != hipSuccess) {
    (void)hipStreamSynchronize(st);
    for (mvpb_plan pl : made) delete pl;
    return set_err(MVPB_E_NOMEM, "plan build: %s", hipGetErrorString(e));
  }
  for (int c = 0; c < g; ++c) {
    ctx->children++;
    out[c] = made[c];
  }
  return MVPB_OK;
}

// Voigt index of the stress component (a, b) (planar: 11, 22, 12; spatial:
// 11, 22, 33, 23, 13, 12).
static int voigt_index(int dim, int a, int b) {
  if (a == b) return a;
  if (dim == 2) return 2;
  const int lo = std::min(a, b), hi = std::max(a, b);
  return lo == 1 ? 3 : (hi == 2 ? 4 : 5);   // (1,2) -> 3, (0,2) -> 4, (0,1) -> 5
}

// Plan of the general layout for one pixel or voxel cell: weight fields on the
// difference grid, the full Phi (n_s N square) and R = T(rho) by block-Toeplitz
// scatter, their Cholesky factors and inverse factors, the matrices
// Z_l = (I (x) L_R^-1) H'_l L_P^-H (l = 0: the G part of K, l >= 1: the unit
// Bloch part along axis l), and the coefficients |Omega|^2 (Z_l Z_m^H + ...)
// of C(k) (see general.hip).
static int build_plan_general(mvpb_cell c, int M1, int M2, int M3, int precision, mvpb_plan *out) {
  mvpb_ctx ctx = c->ctx;
  hipStream_t st = ctx->stream;
  const int d = c->dim, ns = d == 2 ? 3 : 6;
  const int N = (2 * M1 + 1) * (2 * M2 + 1) * (2 * M3 + 1), n = d * N, nsig = ns * N;
  const int nc = (d + 1) * (d + 2) / 2;
  const size_t NN = (size_t)N * N, SS = (size_t)nsig * nsig, nn = (size_t)n * n;
  Pool *pool = &ctx->pool;
  DevBuf X1(pool), X2(pool), F(pool), Phi(pool), R(pool), stat(pool), gvec(pool), Z(pool), ptrs(pool);
  int rc = run_structure_factors_general(c, M1, M2, M3, X1, X2, F);
  if (rc) return rc;
  std::unique_ptr<mvpb_plan_s> pl(new mvpb_plan_s());
  pl->ctx = ctx;
  pl->coef.pool = pl->linvR.pool = pl->linvSD.pool = pl->linvPhi.pool = pool;
  HIP_TRY(Phi.alloc(sizeof(cd) * SS));
  HIP_TRY(pl->linvPhi.alloc(sizeof(cd) * SS));
  HIP_TRY(R.alloc(sizeof(cd) * NN));
  HIP_TRY(pl->linvR.alloc(sizeof(cd) * NN));
  HIP_TRY(stat.alloc(sizeof(int) * 2));
  HIP_TRY(Z.alloc(sizeof(cd) * (d + 1) * (size_t)n * nsig));
  HIP_TRY(pl->coef.alloc(sizeof(cd) * nc * nn));
  // Phi block (s, t) from field f(min, max) (upper-triangle packing), R from rho
  int fmap[36];
  for (int a = 0; a < ns; ++a)
    for (int b = 0; b < ns; ++b) {
      const int lo = std::min(a, b), hi = std::max(a, b);
      fmap[a * ns + b] = lo * ns - lo * (lo - 1) / 2 + (hi - lo);
    }
  const int frho = c->nf - 1;
  HIP_TRY(launch_toeplitz_blocks(F.as<cd>(), M1, M2, M3, N, ns, fmap, Phi.as<cd>(), st));
  HIP_TRY(launch_toeplitz_blocks(F.as<cd>(), M1, M2, M3, N, 1, &frho, R.as<cd>(), st));
  // G_l vectors (signed plane-wave indices): G_l[i] = 2 pi (T n_i)_l
  std::vector<double> gv((size_t)d * N);
  for (int a = -M1; a <= M1; ++a)
    for (int b = -M2; b <= M2; ++b)
      for (int e = -M3; e <= M3; ++e) {
        const int i = ((a + M1) * (2 * M2 + 1) + (b + M2)) * (2 * M3 + 1) + (e + M3);
        const double nv[3] = {(double)a, (double)b, (double)e};
        for (int l = 0; l < d; ++l) {
          double acc = 0.0;
          for (int j = 0; j < d; ++j) acc += c->T3[l * d + j] * nv[j];
          gv[(size_t)l * N + i] = 2.0 * M_PI * acc;
        }
      }
  HIP_TRY(gvec.alloc(sizeof(double) * gv.size()));
  HIP_TRY(hipMemcpyAsync(gvec.p, gv.data(), sizeof(double) * gv.size(), hipMemcpyHostToDevice, st));
  cd *P = Phi.as<cd>(), *LP = pl->linvPhi.as<cd>(), *Rm = R.as<cd>(), *LR = pl->linvR.as<cd>(), *Zm = Z.as<cd>();
  cd *coef = pl->coef.as<cd>();
  const double *gd = gvec.as<double>();
  // Device pointer table: consecutive lists per batched launch.
  std::vector<const void *> tab = {P, LP, Rm, LR};
  auto list = [&](std::vector<const void *> v) {
    const size_t o = tab.size();
    tab.insert(tab.end(), v.begin(), v.end());
    return o;
  };
  // B_s = (columns s N .. (s+1) N - 1 of L_P^-1)^H (N x nsig)
  auto Bs = [&](int s_) { return (const void *)(LP + (size_t)s_ * N * nsig); };
  // Z_0 block a = sum_b L_R^-1 diag(G_b) B_{voigt(a,b)}: one launch per b over a
  size_t z0[3][4];
  for (int b = 0; b < d; ++b) {
    std::vector<const void *> A, B, C, S;
    for (int a = 0; a < d; ++a) {
      A.push_back(LR);
      B.push_back(Bs(voigt_index(d, a, b)));
      C.push_back(Zm + (size_t)a * N);
      S.push_back(gd + (size_t)b * N);
    }
    z0[b][0] = list(A);
    z0[b][1] = list(B);
    z0[b][2] = list(C);
    z0[b][3] = list(S);
  }
  // Z_l block a = L_R^-1 B_{voigt(a, l-1)}, l = 1 .. d: one launch
  size_t zl[3];
  {
    std::vector<const void *> A, B, C;
    for (int l = 1; l <= d; ++l)
      for (int a = 0; a < d; ++a) {
        A.push_back(LR);
        B.push_back(Bs(voigt_index(d, a, l - 1)));
        C.push_back(Zm + (size_t)l * n * nsig + (size_t)a * N);
      }
    zl[0] = list(A);
    zl[1] = list(B);
    zl[2] = list(C);
  }
  // coefficients |Omega|^2 Z_l Z_m^H for l <= m, then + |Omega|^2 Z_m Z_l^H for l < m
  size_t c1[3], c2[3];
  int n2 = 0;
  {
    std::vector<const void *> A1, B1, C1, A2, B2, C2;
    int q = 0;
    for (int l = 0; l <= d; ++l)
      for (int m = l; m <= d; ++m, ++q) {
        A1.push_back(Zm + (size_t)l * n * nsig);
        B1.push_back(Zm + (size_t)m * n * nsig);
        C1.push_back(coef + (size_t)q * nn);
        if (l < m) {
          A2.push_back(Zm + (size_t)m * n * nsig);
          B2.push_back(Zm + (size_t)l * n * nsig);
          C2.push_back(coef + (size_t)q * nn);
        }
      }
    n2 = (int)A2.size();
    c1[0] = list(A1); c1[1] = list(B1); c1[2] = list(C1);
    c2[0] = list(A2); c2[1] = list(B2); c2[2] = list(C2);
  }
  HIP_TRY(ptrs.alloc(sizeof(void *) * tab.size()));
  HIP_TRY(hipMemcpyAsync(ptrs.p, tab.data(), sizeof(void *) * tab.size(), hipMemcpyHostToDevice, st));
  void **dp = ptrs.as<void *>();
  auto cp = [&](size_t o) { return (const cd *const *)(dp + o); };
  HIP_TRY(launch_potrf_trtri((cd *const *)dp, (cd *const *)(dp + 1), stat.as<int>(), 1, nsig, st));
  HIP_TRY(launch_potrf_trtri((cd *const *)(dp + 2), (cd *const *)(dp + 3), stat.as<int>() + 1, 1, N, st));
  int hstat[2] = {0, 0};
  HIP_TRY(hipMemcpyAsync(hstat, stat.p, sizeof hstat, hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  if (hstat[0] || hstat[1])
    return set_err(MVPB_E_NOT_PD, "%s is not positive definite (pivot %d)",
                   hstat[0] ? "compliance matrix Phi" : "density matrix Omega", (hstat[0] ? hstat[0] : hstat[1]) - 1);
  for (int b = 0; b < d; ++b) {
    GemmBatch bt{cp(z0[b][0]), cp(z0[b][1]), (cd *const *)(dp + z0[b][2]), (const double *const *)(dp + z0[b][3]),
                 N, nsig, n};
    HIP_TRY(launch_zgemm(OP_N, OP_C, N, nsig, N, mk(1.0, 0.0), bt, mk(b == 0 ? 0.0 : 1.0, 0.0), d, st));
  }
  {
    GemmBatch bt{cp(zl[0]), cp(zl[1]), (cd *const *)(dp + zl[2]), nullptr, N, nsig, n};
    HIP_TRY(launch_zgemm(OP_N, OP_C, N, nsig, N, mk(1.0, 0.0), bt, mk(0.0, 0.0), d * d, st));
  }
  const double v2 = c->area * c->area;
  {
    GemmBatch bt{cp(c1[0]), cp(c1[1]), (cd *const *)(dp + c1[2]), nullptr, n, n, n};
    HIP_TRY(launch_zgemm(OP_N, OP_C, n, n, nsig, mk(v2, 0.0), bt, mk(0.0, 0.0), nc, st));
  }
  {
    GemmBatch bt{cp(c2[0]), cp(c2[1]), (cd *const *)(dp + c2[2]), nullptr, n, n, n};
    HIP_TRY(launch_zgemm(OP_N, OP_C, n, n, nsig, mk(v2, 0.0), bt, mk(1.0, 0.0), n2, st));
  }
  pl->M1 = M1;
  pl->M2 = M2;
  pl->M3 = M3;
  pl->N = N;
  pl->prec = precision;
  pl->dim = d;
  pl->n = n;
  pl->nsig = nsig;
  pl->qdim = d;
  pl->area = c->area;
  pl->gx = c->nx;
  pl->gy = c->ny;
  pl->gz = c->nz;
  memcpy(pl->T, c->T, sizeof pl->T);
  memcpy(pl->T3, c->T3, sizeof pl->T3);
  ctx->children++;
  *out = pl.release();
  return MVPB_OK;
}

extern "C" int mvpb_plan_create(mvpb_cell c, int M1, int M2, int precision, mvpb_plan *out) {
  if (!c || !out) return set_err(MVPB_E_INVALID, "NULL argument");
  int rc = check_cutoff(M1, M2);
  if (rc) return rc;
  rc = check_precision(precision);
  if (rc) return rc;
  mvpb_ctx ctx = c->ctx;
  if (ctx->closing) return set_err(MVPB_E_INVALID, "context has been destroyed");
  if (c->dim != 2) return set_err(MVPB_E_INVALID, "a voxel cell needs mvpb_plan_create3");
  HIP_TRY(hipSetDevice(ctx->device));
  ProfBind pb(ctx);
  mvpb_plan pl = nullptr;
  if (c->general || (precision & MVPB_PREC_GENERAL))
    rc = build_plan_general(c, M1, M2, 0, precision, &pl);
  else
    rc = build_plan_group(ctx, &c, 1, M1, M2, precision, &pl, 0);
  if (rc) return rc;
  *out = pl;
  return MVPB_OK;
}

extern "C" int mvpb_plan_create3(mvpb_cell c, int M1, int M2, int M3, int precision, mvpb_plan *out) {
  if (!c || !out) return set_err(MVPB_E_INVALID, "NULL argument");
  int rc = check_cutoff3(c, M1, M2, M3);
  if (rc) return rc;
  rc = check_precision(precision);
  if (rc) return rc;
  if (c->dim == 2) return mvpb_plan_create(c, M1, M2, precision, out);
  mvpb_ctx ctx = c->ctx;
  if (ctx->closing) return set_err(MVPB_E_INVALID, "context has been destroyed");
  HIP_TRY(hipSetDevice(ctx->device));
  ProfBind pb(ctx);
  mvpb_plan pl = nullptr;
  rc = build_plan_general(c, M1, M2, M3, precision, &pl);
  if (rc) return rc;
  *out = pl;
  return MVPB_OK;
}

extern "C" int mvpb_plan_create_batch(mvpb_ctx ctx, int n, const mvpb_cell *cells, const int *M1, const int *M2,
                                      int precision, mvpb_plan *out) {
  int rc = check_ctx(ctx);
  if (rc) return rc;
  if (n < 0 || (n > 0 && (!cells || !M1 || !M2 || !out))) return set_err(MVPB_E_INVALID, "NULL argument");
  rc = check_precision(precision);
  if (rc) return rc;
  bool general = (precision & MVPB_PREC_GENERAL) != 0;
  for (int i = 0; i < n; ++i) {
    if (!cells[i] || cells[i]->ctx != ctx) return set_err(MVPB_E_INVALID, "cell %d missing or from another context", i);
    if (cells[i]->dim != 2) return set_err(MVPB_E_INVALID, "cell %d is a voxel cell: use mvpb_plan_create3", i);
    rc = check_cutoff(M1[i], M2[i]);
    if (rc) return rc;
    general = general || cells[i]->general;
  }
  HIP_TRY(hipSetDevice(ctx->device));
  ProfBind pb(ctx);
  if (general) {
    // general layout: one build per cell
    std::vector<mvpb_plan> res(n, nullptr);
    for (int i = 0; i < n; ++i) {
      rc = (cells[i]->general || (precision & MVPB_PREC_GENERAL))
               ? build_plan_general(cells[i], M1[i], M2[i], 0, precision, &res[i])
               : build_plan_group(ctx, &cells[i], 1, M1[i], M2[i], precision, &res[i], i);
      if (rc) {
        for (mvpb_plan p : res)
          if (p) mvpb_plan_destroy(p);
        return rc;
      }
    }
    for (int i = 0; i < n; ++i) out[i] = res[i];
    return MVPB_OK;
  }
  // group by cutoff, keep each group's temporaries under ~8 GB
  std::vector<int> order(n);
  for (int i = 0; i < n; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
    return M1[a] != M1[b] ? M1[a] < M1[b] : M2[a] < M2[b];
  });
  std::vector<mvpb_plan> res(n, nullptr);
  auto release = [&]() {
    for (mvpb_plan p : res)
      if (p) mvpb_plan_destroy(p);
  };
  size_t i0 = 0;
  while (i0 < (size_t)n) {
    size_t i1 = i0;
    while (i1 < (size_t)n && M1[order[i1]] == M1[order[i0]] && M2[order[i1]] == M2[order[i0]]) ++i1;
    const size_t N = (size_t)(2 * M1[order[i0]] + 1) * (2 * M2[order[i0]] + 1);
    const size_t per = 30 * N * N * sizeof(cd) + 64 * N * sizeof(cd);
    const size_t gmax = std::max<size_t>(1, ((size_t)8 << 30) / per);
    for (size_t s = i0; s < i1; s += gmax) {
      const size_t g = std::min(gmax, i1 - s);
      std::vector<mvpb_cell> cs(g);
      std::vector<mvpb_plan> ps(g, nullptr);
      for (size_t k = 0; k < g; ++k) cs[k] = cells[order[s + k]];
      rc = build_plan_group(ctx, cs.data(), (int)g, M1[order[s]], M2[order[s]], precision, ps.data(), (int)s);
      if (rc) {
        release();
        return rc;
      }
      for (size_t k = 0; k < g; ++k) res[order[s + k]] = ps[k];
    }
    i0 = i1;
  }
  for (int i = 0; i < n; ++i) out[i] = res[i];
  return MVPB_OK;
}

extern "C" int mvpb_plan_dofs(mvpb_plan p, int *n_u, int *n_s) {
  if (!p) return set_err(MVPB_E_INVALID, "NULL plan");
  if (n_u) *n_u = p->n;
  if (n_s) *n_s = p->nsig;
  return MVPB_OK;
}

extern "C" int mvpb_plan_destroy(mvpb_plan p) {
  if (!p) return MVPB_OK;
  mvpb_ctx ctx = p->ctx;
  (void)hipSetDevice(ctx->device);
  delete p;   // its buffers return to the stream-ordered pool
  ctx_release(ctx);
  return MVPB_OK;
}

// ---------------------------------------------------------------------------
// per-item workspace layout
// ---------------------------------------------------------------------------
static size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

// Sizes of the per-item buffers, in carving order.
static void item_layout(int n, int nb, bool fp32, size_t *sz, int *count) {
  const size_t es = fp32 ? sizeof(cf) : sizeof(cd);
  const size_t nrb = (size_t)(n + 63) / 64, npan = (size_t)(n + HB - 1) / HB;
  const size_t nrefl = (size_t)refl_total(n);
  int k = 0;
  sz[k++] = es * (size_t)n * n;                  // A
  sz[k++] = sizeof(cd) * (size_t)n * n;          // Ak
  sz[k++] = es * (size_t)n * HB;                 // X0
  sz[k++] = es * (size_t)n * HB;                 // Wm
  sz[k++] = es * nrb * HB * HB;                  // M0p
  sz[k++] = es * npan * HB * HB;                 // T1
  sz[k++] = es * ((size_t)n + WB_PAD_COLS) * (2 * HB + 1);  // WB (zero columns after the last)
  sz[k++] = es * nrefl * HB;                     // V2
  sz[k++] = es * nrefl;                          // tau2
  sz[k++] = sizeof(double) * n;                  // d
  sz[k++] = sizeof(double) * n;                  // e
  sz[k++] = sizeof(int) * ((size_t)n + 2);       // flag: error, abort, progress of each sweep
  sz[k++] = sizeof(double) * (size_t)n * nb;     // X
  sz[k++] = sizeof(double) * (size_t)5 * n * nb; // lu
  sz[k++] = sizeof(double) * nb;                 // lam_t
  sz[k++] = sizeof(double) * nb;                 // lam
  sz[k++] = sizeof(double) * nb;                 // omega
  sz[k++] = sizeof(cd) * (size_t)n * nb;         // Y
  sz[k++] = sizeof(cd) * (size_t)n * nb;         // Z
  const bool rr = nb <= RR_MAX_BANDS;            // the Rayleigh-Ritz step runs
  sz[k++] = rr ? sizeof(cd) * ((size_t)(n + 63) / 64) * 2 * nb * nb : 0;  // Gp
  sz[k++] = rr ? sizeof(cd) * (size_t)nb * nb : 0;                      // Lr
  sz[k++] = fp32 ? sizeof(cf) * (size_t)n * nb : 0;  // Yb (FP32 path only)
  sz[k++] = sizeof(double);                      // acc
  *count = k;
}

static size_t item_bytes(int n, int nb, bool fp32) {
  size_t sz[32];
  int cnt = 0;
  item_layout(n, nb, fp32, sz, &cnt);
  size_t s = 0;
  for (int i = 0; i < cnt; ++i) s += align256(sz[i]);
  return s;
}

// Bulge-chasing control words of a launch sequence over n items (placed
// after the items in the workspace).
static size_t ctl_bytes(size_t n_items) { return align256(sizeof(int) * hb2st_ctl_ints((int)n_items)); }
// Workspace of a launch sequence over n items of per bytes each.
static size_t solve_bytes(size_t n_items, size_t per) { return n_items * per + ctl_bytes(n_items); }

static EigItem carve_item(char *base, int n, int nb, bool fp32) {
  size_t sz[32];
  int cnt = 0;
  item_layout(n, nb, fp32, sz, &cnt);
  EigItem it{};
  size_t o = 0;
  int k = 0;
  auto take = [&]() {
    char *p = base + o;
    o += align256(sz[k++]);
    return p;
  };
  it.A = take();
  it.Ak = (cd *)take();
  it.X0 = take();
  it.Wm = take();
  it.M0p = take();
  it.T1 = take();
  it.WB = take();
  it.V2 = take();
  it.tau2 = take();
  it.d = (double *)take();
  it.e = (double *)take();
  it.flag = (int *)take();
  it.X = (double *)take();
  it.lu = (double *)take();
  it.lam_t = (double *)take();
  it.lam = (double *)take();
  it.omega = (double *)take();
  it.Y = (cd *)take();
  it.Z = (cd *)take();
  it.Gp = (cd *)take();
  it.Lr = (cd *)take();
  char *yb = take();
  it.Yb = fp32 ? (void *)yb : (void *)it.Y;
  it.acc = (double *)take();
  return it;
}

// Normalise each eigenvector (length len, complex) so that its
// largest-modulus entry (lowest index on ties) is real and positive.
__global__ void normalize_phase(cd *U, int len, int count) {
  __shared__ double bv[256];
  __shared__ int bi[256];
  const int v = blockIdx.x;
  if (v >= count) return;
  cd *u = U + (size_t)v * len;
  double best = -1.0;
  int idx = 0;
  for (int r = threadIdx.x; r < len; r += blockDim.x) {
    const double a = abs2(u[r]);
    if (a > best) { best = a; idx = r; }
  }
  bv[threadIdx.x] = best;
  bi[threadIdx.x] = idx;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) {
      const double o = bv[threadIdx.x + s];
      const int oi = bi[threadIdx.x + s];
      if (o > bv[threadIdx.x] || (o == bv[threadIdx.x] && oi < bi[threadIdx.x])) {
        bv[threadIdx.x] = o;
        bi[threadIdx.x] = oi;
      }
    }
    __syncthreads();
  }
  const cd piv = u[bi[0]];
  const double a = sqrt(abs2(piv));
  if (a == 0.0) return;
  const cd ph = mk(piv.re / a, -piv.im / a);
  for (int r = threadIdx.x; r < len; r += blockDim.x) u[r] = u[r] * ph;
}

// Frequencies of every item to its row of the caller's output; an item whose
// bulge chasing gave up gets NaN.
__global__ void gather_omega(const EigItem *items, int n_items, int nb, double *out) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n_items * nb) return;
  const int i = t / nb, b = t % nb;
  const EigItem &it = items[i];
  const double v = __hip_atomic_load(it.flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) ? NAN : it.omega[b];
  out[(size_t)it.slot * nb + b] = v;
}

__global__ void set_double(double *p, double v) { *p = v; }

// Largest error estimate of the items' refined bands into *out (running max
// over the launch sequences of one solve).
__global__ void __launch_bounds__(256) max_acc(const EigItem *items, int n_items, double *out) {
  __shared__ double red[4];
  double v = 0.0;
  for (int i = threadIdx.x; i < n_items; i += 256) v = fmax(v, *items[i].acc);
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) *out = fmax(fmax(fmax(*out, red[0]), fmax(red[1], red[2])), red[3]);
}

// Start of a solve: clear the running error estimate.
static int acc_begin(mvpb_ctx ctx) {
  HIP_TRY(ctx->accbuf.reserve(sizeof(double)));
  hipLaunchKernelGGL(set_double, dim3(1), dim3(1), 0, ctx->stream, ctx->accbuf.as<double>(), 0.0);
  HIP_TRY(hipGetLastError());
  return MVPB_OK;
}

// End of a synchronous solve (stream drained): record the estimate and apply
// the accuracy bar to solves with the FP32 reduction.
static int acc_finish(mvpb_ctx ctx, bool fp32) {
  double v = 0.0;
  HIP_TRY(hipMemcpy(&v, ctx->accbuf.p, sizeof v, hipMemcpyDeviceToHost));
  ctx->last_acc = v;
  if (fp32 && ctx->acc_tol > 0.0 && !(v <= ctx->acc_tol))
    return set_err(MVPB_E_ACCURACY, "estimated relative frequency error %.3g exceeds the bar %.3g", v,
                   ctx->acc_tol);
  return MVPB_OK;
}

// One batch of work items that share a workspace allocation.
struct Job {
  mvpb_plan plan;
  double Q1, Q2, Q3;   // Bloch vector in the reciprocal basis (Q3 = 0 for planar plans)
  int out_index;       // position in the caller's flattened output
};

constexpr size_t MAX_GRAPHS = 16;

// Everything the launch shapes of one eigensolve sequence depend on: the
// order 2N of every item in table order (which fixes the workspace carving,
// the stage-1 parts' size ranges and the grids), the bands, the reduction
// precision and the number of stage-1 parts.
static std::string launch_signature(const std::vector<Job> &jobs, int nb, bool fp32, int parts,
                                    const Stage2Shape &sh) {
  std::string k;
  k.reserve(32 + 8 * jobs.size());
  auto put = [&](int v) { k.append(reinterpret_cast<const char *>(&v), sizeof v); };
  put(nb);
  put(fp32 ? 1 : 0);
  put(parts);
  put(sh.group);
  put(sh.wg_max);
  put((int)(sh.spin_limit & 0x7fffffff));
  put((int)(sh.spin_limit >> 31));
  put((int)jobs.size());
  for (const Job &j : jobs) {
    put(j.plan->n);
    put(j.plan->dim);
  }
  return k;
}

// Events of one eigensolve launch sequence over items of order at most n_max
// in `parts` parts: two per stage-1 step and part, then the fork and join of
// the tridiagonal eigenvectors.
static size_t la_events_needed(int n_max, int parts) { return (size_t)2 * parts * stage1_steps(n_max) + 2; }

// Grow the context's step-event pool to at least `count` events (outside any
// capture).
static hipError_t reserve_la_events(mvpb_ctx ctx, size_t count) {
  while (ctx->la_events.size() < count) {
    hipEvent_t ev;
    hipError_t e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
    if (e != hipSuccess) return e;
    ctx->la_events.push_back(ev);
  }
  return hipSuccess;
}

// The eigensolve launch sequence over the items of a device table whose
// operator orders are `orders` (table order): operator formation, stage 1 in
// independent parts on the context's streams, bulge chasing, tridiagonal
// eigenpairs, back-transform, Rayleigh-Ritz (or the tridiagonal results
// beyond RR_MAX_BANDS).  ctl: the bulge-chasing control words.
static hipError_t enqueue_eigensolve(mvpb_ctx ctx, const EigItem *d_items, const std::vector<int> &orders,
                                     bool any_iso, bool any_general, int nb, bool fp32, int parts_wanted,
                                     const Stage2Shape &sh, int *ctl, hipStream_t st, hipEvent_t ev_fork,
                                     const hipEvent_t *ev_join, const hipEvent_t *la_ev) {
  const int n_items = (int)orders.size();
  int n_max = 0, n_min = 1 << 30;
  for (int n : orders) {
    n_max = std::max(n_max, n);
    n_min = std::min(n_min, n);
  }
  hipError_t e = hipSuccess;
  if (any_iso) e = launch_form_operator(d_items, n_items, n_max, fp32, st);
  if (e == hipSuccess && any_general) e = launch_form_operator_general(d_items, n_items, n_max, fp32, st);
  // stage 1 in independent parts of the items, one per stream
  ItemPart parts[MAX_SIDE + 1];
  const int n_parts = std::max(1, std::min(parts_wanted, n_items));
  for (int q = 0; q < n_parts; ++q) {
    const int i0 = (int)((long long)n_items * q / n_parts), i1 = (int)((long long)n_items * (q + 1) / n_parts);
    ItemPart &pt = parts[q];
    pt.items = d_items + i0;
    pt.n_items = i1 - i0;
    pt.n_min = 1 << 30;
    pt.n_max = 0;
    for (int i = i0; i < i1; ++i) {
      pt.n_min = std::min(pt.n_min, orders[i]);
      pt.n_max = std::max(pt.n_max, orders[i]);
    }
    pt.stream = q == 0 ? st : ctx->side[q - 1];
    pt.aside = ctx->la[q];
    pt.ev = la_ev + (size_t)q * 2 * stage1_steps(n_max);
  }
  if (e == hipSuccess && n_parts > 1) {
    e = hipEventRecord(ev_fork, st);
    for (int q = 1; q < n_parts && e == hipSuccess; ++q) e = hipStreamWaitEvent(parts[q].stream, ev_fork, 0);
  }
  if (e == hipSuccess) e = launch_stage1(parts, n_parts, fp32);
  for (int q = 1; q < n_parts && e == hipSuccess; ++q) {
    e = hipEventRecord(ev_join[q - 1], parts[q].stream);
    if (e == hipSuccess) e = hipStreamWaitEvent(st, ev_join[q - 1], 0);
  }
  if (e == hipSuccess) e = launch_stage2(d_items, n_items, n_max, fp32, ctl, sh, st);
  if (e == hipSuccess) {
    const hipEvent_t *tev = la_ev + (size_t)2 * std::max(1, parts_wanted) * stage1_steps(n_max);
    e = launch_tridiag_eig(d_items, n_items, n_max, nb, st, ctx->la[0], tev[0], tev[1]);
  }
  if (e == hipSuccess) e = launch_backtransform(d_items, n_items, n_min, n_max, nb, fp32, st);
  if (e == hipSuccess)
    e = nb <= RR_MAX_BANDS ? launch_rayleigh_ritz(d_items, n_items, n_max, nb, fp32, st)
                           : launch_tridiag_results(d_items, n_items, nb, st);
  return e;
}

static int run_items(mvpb_ctx ctx, const std::vector<Job> &jobs, int nb, double *omega_dev, double *U_dev,
                     bool use_graph) {
  // the reduction precision is shared by every item of one launch sequence
  const bool fp32 = jobs.empty() ? false : (jobs[0].plan->prec & MVPB_PREC_EIG_FP32_RR64) != 0;
  hipStream_t st = ctx->stream;
  const int n_items = (int)jobs.size();
  if (n_items == 0) return MVPB_OK;
  // the sequence ends with a write of the running error estimate
  if (!ctx->accbuf.p || ctx->accbuf.bytes < sizeof(double))
    return set_err(MVPB_E_DEVICE, "context has no error-estimate buffer");
  size_t total = 0;
  int n_max = 0, n_min = 1 << 30;
  bool any_iso = false, any_general = false;
  for (const Job &j : jobs) {
    const int n = j.plan->n;
    any_iso = any_iso || j.plan->dim == 0;
    any_general = any_general || j.plan->dim != 0;
    total += item_bytes(n, nb, fp32);
    n_max = std::max(n_max, n);
    n_min = std::min(n_min, n);
  }
  const size_t ctl_off = total;   // bulge-chasing launch control words after the items
  // launch shape of this size class
  TuneParams tp;
  {
    auto f = ctx->tune.find(size_class(n_max));
    if (f != ctx->tune.end()) tp = f->second;
  }
  const int parts_wanted = std::max(1, std::min(tp.parts, MAX_SIDE + 1));
  Stage2Shape sh;
  sh.group = tp.group;
  sh.wg_max = tp.wg_max;
  sh.spin_limit = ctx->spin_limit;
  total += ctl_bytes(n_items);
  if (ctx->cap && total > ctx->cap)
    return set_err(MVPB_E_NOMEM, "workspace %zu bytes exceeds the cap of %zu bytes", total, ctx->cap);
  const bool realloc = total > ctx->ws.bytes || sizeof(EigItem) * n_items > ctx->items.bytes;
  if (realloc) {
    // captured graphs point into the old buffers
    HIP_TRY(hipStreamSynchronize(st));
    for (auto &kv : ctx->graphs) (void)hipGraphExecDestroy(kv.second.exec);
    ctx->graphs.clear();
  }
  HIP_TRY(ctx->ws.reserve(total));
  HIP_TRY(ctx->items.reserve(sizeof(EigItem) * n_items));
  // the staging vector may still feed an earlier asynchronous copy
  HIP_TRY(hipStreamSynchronize(st));
  std::vector<EigItem> &items = ctx->host_items;
  items.assign(n_items, EigItem{});
  size_t off = 0;
  for (int i = 0; i < n_items; ++i) {
    const Job &j = jobs[i];
    const int n = j.plan->n;
    EigItem it = carve_item(ctx->ws.as<char>() + off, n, nb, fp32);
    off += item_bytes(n, nb, fp32);
    it.coef = j.plan->coef.as<cd>();
    it.N = j.plan->N;
    it.n = n;
    it.dim = j.plan->dim;
    it.check = fp32 ? 1 : 0;
    it.nb = nb;
    it.slot = j.out_index;
    // kappa = 2 pi T Q (Cartesian Bloch vector)
    const int qd = j.plan->qdim;
    const double *T = j.plan->T3;
    const double q[3] = {j.Q1, j.Q2, j.Q3};
    double kap[3] = {0.0, 0.0, 0.0};
    for (int l = 0; l < qd; ++l)
      for (int m = 0; m < qd; ++m) kap[l] += 2.0 * M_PI * T[l * qd + m] * q[m];
    it.kap1 = kap[0];
    it.kap2 = kap[1];
    it.kap3 = kap[2];
    items[i] = it;
  }
  HIP_TRY(hipMemcpyAsync(ctx->items.p, items.data(), sizeof(EigItem) * n_items, hipMemcpyHostToDevice, st));
  const EigItem *d_items = ctx->items.as<EigItem>();

  std::vector<int> orders(n_items);
  for (int i = 0; i < n_items; ++i) orders[i] = jobs[i].plan->n;
  int *ctl = reinterpret_cast<int *>(ctx->ws.as<char>() + ctl_off);
  HIP_TRY(reserve_la_events(ctx, la_events_needed(n_max, parts_wanted)));
  auto enqueue = [&]() -> hipError_t {
    return enqueue_eigensolve(ctx, d_items, orders, any_iso, any_general, nb, fp32, parts_wanted, sh, ctl, st,
                              ctx->ev_fork, ctx->ev_join, ctx->la_events.data());
  };
  if (use_graph) {
    const std::string graph_key = launch_signature(jobs, nb, fp32, parts_wanted, sh);
    auto found = ctx->graphs.find(graph_key);
    hipGraphExec_t exec = nullptr;
    if (found == ctx->graphs.end()) {
      if (ctx->graphs.size() >= MAX_GRAPHS) {
        auto lru = ctx->graphs.begin();
        for (auto it = ctx->graphs.begin(); it != ctx->graphs.end(); ++it)
          if (it->second.last_use < lru->second.last_use) lru = it;
        HIP_TRY(hipStreamSynchronize(st));
        (void)hipGraphExecDestroy(lru->second.exec);
        ctx->graphs.erase(lru);
      }
      hipGraph_t g;
      HIP_TRY(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
      Profiler *saved = t_prof;
      t_prof = nullptr;  // no event records inside the captured graph
      hipError_t e = enqueue();
      t_prof = saved;
      hipError_t e2 = hipStreamEndCapture(st, &g);
      if (e != hipSuccess) return set_err(MVPB_E_DEVICE, "graph capture: %s", hipGetErrorString(e));
      if (e2 != hipSuccess) return set_err(MVPB_E_DEVICE, "graph capture end: %s", hipGetErrorString(e2));
      e = hipGraphInstantiate(&exec, g, nullptr, nullptr, 0);
      (void)hipGraphDestroy(g);
      if (e != hipSuccess) return set_err(MVPB_E_DEVICE, "graph instantiate: %s", hipGetErrorString(e));
      ctx->graphs[graph_key] = mvpb_ctx_s::GraphEntry{exec, ++ctx->graph_clock};
    } else {
      exec = found->second.exec;
      found->second.last_use = ++ctx->graph_clock;
    }
    HIP_TRY(hipGraphLaunch(exec, st));
  } else {
    HIP_TRY(enqueue());
  }
  // frequencies to the caller's order (jobs may be sorted)
  hipLaunchKernelGGL(gather_omega, dim3((n_items * nb + 255) / 256), dim3(256), 0, st, d_items, n_items, nb,
                     omega_dev);
  HIP_TRY(hipGetLastError());
  hipLaunchKernelGGL(max_acc, dim3(1), dim3(256), 0, st, d_items, n_items, ctx->accbuf.as<double>());
  HIP_TRY(hipGetLastError());
  if (U_dev) {
    // U_t block c = L_R^-H Z_t(c N : (c+1) N, :) for the d displacement
    // components (d = n / N), written in caller order
    std::vector<const void *> hp;
    int dmax = 0;
    for (int i = 0; i < n_items; ++i) dmax = std::max(dmax, jobs[i].plan->n / jobs[i].plan->N);
    // table per component c: [A: n_items][B: n_items][C: n_items]
    for (int c = 0; c < dmax; ++c) {
      for (int i = 0; i < n_items; ++i) hp.push_back(jobs[i].plan->linvR.p);
      for (int i = 0; i < n_items; ++i)   // refined vectors (Z) or, beyond RR_MAX_BANDS, the back-transformed ones (Y)
        hp.push_back((nb <= RR_MAX_BANDS ? items[i].Z : items[i].Y) +
                     (size_t)std::min(c, jobs[i].plan->n / jobs[i].plan->N - 1) * jobs[i].plan->N);
      for (int i = 0; i < n_items; ++i) {
        const Job &jb = jobs[i];
        const int dd = jb.plan->n / jb.plan->N;
        hp.push_back(U_dev + ((size_t)jb.out_index * nb * jb.plan->n + (size_t)std::min(c, dd - 1) * jb.plan->N) * 2);
      }
    }
    DevBuf ptrs(&ctx->pool);
    HIP_TRY(ptrs.alloc(sizeof(void *) * hp.size()));
    HIP_TRY(hipMemcpyAsync(ptrs.p, hp.data(), sizeof(void *) * hp.size(), hipMemcpyHostToDevice, st));
    void **dp = ptrs.as<void *>();
    auto at = [&](int c, int part, int i) { return dp + (size_t)c * 3 * n_items + (size_t)part * n_items + i; };
    // items of one operator (every mvpb_solve call): d batched products and one
    // normalisation over all of them; otherwise item by item
    bool same_n = true;
    for (int i = 1; i < n_items; ++i)
      same_n = same_n && jobs[i].plan->N == jobs[0].plan->N && jobs[i].plan->n == jobs[0].plan->n;
    const int groups = same_n ? 1 : n_items;
    for (int g = 0; g < groups; ++g) {
      const int i0 = same_n ? 0 : g, cnt = same_n ? n_items : 1;
      const int N = jobs[i0].plan->N, n = jobs[i0].plan->n, dd = n / N;
      for (int c = 0; c < dd; ++c) {
        GemmBatch bt{(const cd *const *)at(c, 0, i0), (const cd *const *)at(c, 1, i0), (cd *const *)at(c, 2, i0),
                     nullptr, N, n, n};
        HIP_TRY(launch_zgemm(OP_C, OP_N, N, nb, N, mk(1.0, 0.0), bt, mk(0.0, 0.0), cnt, st));
      }
      cd *u0 = (cd *)(U_dev + (same_n ? 0 : (size_t)jobs[i0].out_index * nb * n * 2));
      hipLaunchKernelGGL(normalize_phase, dim3(cnt * nb), dim3(256), 0, st, u0, n, cnt * nb);
      HIP_TRY(hipGetLastError());
    }
    HIP_TRY(hipStreamSynchronize(st));
  }
  return MVPB_OK;
}

static bool q_ok(const double *Q, int count);

extern "C" int mvpb_stress_modes(mvpb_plan p, int n_k, const double *Q, int n_bands, const double *U, double *S,
                                 unsigned flags);

extern "C" int mvpb_band_sensitivities(mvpb_plan p, int n_k, const double *Q, int n_bands, const double *omega,
                                       const double *U, double *G, unsigned flags) {
  if (!p || !Q || !omega || !U || !G) return set_err(MVPB_E_INVALID, "NULL argument");
  if (n_k < 0) return set_err(MVPB_E_INVALID, "n_k must be non-negative");
  if (n_k == 0) return MVPB_OK;
  if (n_bands < 1 || n_bands > p->n) return set_err(MVPB_E_INVALID, "n_bands = %d outside [1, n_u]", n_bands);
  if (!q_ok(Q, p->qdim * n_k)) return set_err(MVPB_E_INVALID, "non-finite Bloch vector");
  if (p->gx <= 0) return set_err(MVPB_E_UNSUPPORTED, "sensitivities need a pixel or voxel cell");
  mvpb_ctx ctx = p->ctx;
  HIP_TRY(hipSetDevice(ctx->device));
  ProfBind pb(ctx);
  hipStream_t st = ctx->stream;
  const bool dev = flags & MVPB_F_DEVICE_PTRS;
  const int d = p->dim == 0 ? 2 : p->dim, ns = d == 2 ? 3 : 6, nf = ns * (ns + 1) / 2 + 1;
  const int n = p->n, nsig = p->nsig;
  const size_t items = (size_t)n_k * n_bands, cells = (size_t)p->gx * p->gy * p->gz;
  const size_t q1 = 4 * p->M1 + 1, q2 = 4 * p->M2 + 1, q3 = 4 * p->M3 + 1;
  DevBuf ud(&ctx->pool), od(&ctx->pool), Sd(&ctx->pool), Cw(&ctx->pool), Y1(&ctx->pool), Y2(&ctx->pool),
      Gd(&ctx->pool);
  const cd *u = (const cd *)U;
  const double *om = omega;
  if (!dev) {
    HIP_TRY(ud.alloc(sizeof(cd) * items * n));
    HIP_TRY(hipMemcpyAsync(ud.p, U, sizeof(cd) * items * n, hipMemcpyHostToDevice, st));
    u = ud.as<cd>();
    HIP_TRY(od.alloc(sizeof(double) * items));
    HIP_TRY(hipMemcpyAsync(od.p, omega, sizeof(double) * items, hipMemcpyHostToDevice, st));
    om = od.as<double>();
  }
  HIP_TRY(Sd.alloc(sizeof(cd) * items * nsig));
  int rc = mvpb_stress_modes(p, n_k, Q, n_bands, (const double *)u, Sd.as<double>(),
                             MVPB_F_DEVICE_PTRS | MVPB_F_ASYNC);
  if (rc) return rc;
  // chunks of items whose correlation and pass buffers stay within 2 GiB
  const size_t per = sizeof(cd) * nf * (q1 * q2 * q3 + p->gx * q2 * q3 + p->gx * p->gy * q3) +
                     (dev ? 0 : sizeof(double) * nf * cells);
  const size_t chunk = std::max<size_t>(1, std::min(items, ((size_t)2 << 30) / per));
  HIP_TRY(Cw.alloc(sizeof(cd) * chunk * nf * q1 * q2 * q3));
  HIP_TRY(Y1.alloc(sizeof(cd) * chunk * nf * p->gx * q2 * q3));
  HIP_TRY(Y2.alloc(sizeof(cd) * chunk * nf * p->gx * p->gy * q3));
  if (!dev) HIP_TRY(Gd.alloc(sizeof(double) * chunk * nf * cells));
  for (size_t i0 = 0; i0 < items; i0 += chunk) {
    const size_t cnt = std::min(chunk, items - i0);
    double *g = dev ? G + i0 * nf * cells : Gd.as<double>();
    HIP_TRY(launch_sensitivities(u + i0 * n, Sd.as<cd>() + i0 * nsig, om + i0, (int)cnt, d, p->M1, p->M2, p->M3,
                                 p->gx, p->gy, p->gz, p->area, Cw.as<cd>(), Y1.as<cd>(), Y2.as<cd>(), g, st));
    if (!dev)
      HIP_TRY(hipMemcpyAsync(G + i0 * nf * cells, g, sizeof(double) * cnt * nf * cells, hipMemcpyDeviceToHost, st));
  }
  if (!dev || !(flags & MVPB_F_ASYNC)) HIP_TRY(hipStreamSynchronize(st));
  return MVPB_OK;
}

extern "C" int mvpb_stress_modes(mvpb_plan p, int n_k, const double *Q, int n_bands, const double *U, double *S,
                                 unsigned flags) {
  if (!p || !Q || !U || !S) return set_err(MVPB_E_INVALID, "NULL argument");
  if (n_k < 0) return set_err(MVPB_E_INVALID, "n_k must be non-negative");
  if (n_k == 0) return MVPB_OK;
  if (n_bands < 1 || n_bands > p->n) return set_err(MVPB_E_INVALID, "n_bands = %d outside [1, n_u]", n_bands);
  if (!q_ok(Q, p->qdim * n_k)) return set_err(MVPB_E_INVALID, "non-finite Bloch vector");
  mvpb_ctx ctx = p->ctx;
  HIP_TRY(hipSetDevice(ctx->device));
  ProfBind pb(ctx);
  hipStream_t st = ctx->stream;
  const bool dev = flags & MVPB_F_DEVICE_PTRS;
  if (p->dim != 0) {
    // general layout: X = H* U, then S = -L_P^-H (L_P^-1 X) with the plan's inverse factor
    const int nb = n_bands, n = p->n, ns = p->nsig, qd = p->qdim;
    const size_t u_bytes = sizeof(cd) * (size_t)n_k * nb * n, s_bytes = sizeof(cd) * (size_t)n_k * nb * ns;
    DevBuf qd_(&ctx->pool), ud(&ctx->pool), sd(&ctx->pool), X(&ctx->pool), Y(&ctx->pool), ptrs(&ctx->pool);
    HIP_TRY(qd_.alloc(sizeof(double) * qd * (size_t)n_k));
    HIP_TRY(hipMemcpyAsync(qd_.p, Q, sizeof(double) * qd * (size_t)n_k, hipMemcpyHostToDevice, st));
    const cd *u_in = (const cd *)U;
    cd *s_out = (cd *)S;
    if (!dev) {
      HIP_TRY(ud.alloc(u_bytes));
      HIP_TRY(hipMemcpyAsync(ud.p, U, u_bytes, hipMemcpyHostToDevice, st));
      u_in = ud.as<cd>();
      HIP_TRY(sd.alloc(s_bytes));
      s_out = sd.as<cd>();
    }
    HIP_TRY(X.alloc(s_bytes));
    HIP_TRY(Y.alloc(s_bytes));
    HIP_TRY(launch_stress_rhs_general(u_in, qd_.as<double>(), n_k, nb, p->dim, p->M1, p->M2, p->M3, p->T3, p->area,
                                      X.as<cd>(), st));
    std::vector<const void *> hp;
    for (int t = 0; t < n_k; ++t) hp.push_back(p->linvPhi.p);
    for (int t = 0; t < n_k; ++t) hp.push_back(X.as<cd>() + (size_t)t * nb * ns);
    for (int t = 0; t < n_k; ++t) hp.push_back(Y.as<cd>() + (size_t)t * nb * ns);
    for (int t = 0; t < n_k; ++t) hp.push_back(s_out + (size_t)t * nb * ns);
    HIP_TRY(ptrs.alloc(sizeof(void *) * hp.size()));
    HIP_TRY(hipMemcpyAsync(ptrs.p, hp.data(), sizeof(void *) * hp.size(), hipMemcpyHostToDevice, st));
    void **dp = ptrs.as<void *>();
    GemmBatch b1{(const cd *const *)dp, (const cd *const *)(dp + n_k), (cd *const *)(dp + 2 * n_k), nullptr, ns, ns,
                 ns};
    HIP_TRY(launch_zgemm(OP_N, OP_N, ns, nb, ns, mk(1.0, 0.0), b1, mk(0.0, 0.0), n_k, st));
    GemmBatch b2{(const cd *const *)dp, (const cd *const *)(dp + 2 * n_k), (cd *const *)(dp + 3 * n_k), nullptr, ns,
                 ns, ns};
    HIP_TRY(launch_zgemm(OP_C, OP_N, ns, nb, ns, mk(-1.0, 0.0), b2, mk(0.0, 0.0), n_k, st));
    if (!dev) HIP_TRY(hipMemcpyAsync(S, s_out, s_bytes, hipMemcpyDeviceToHost, st));
    if (!(flags & MVPB_F_ASYNC) || !dev) HIP_TRY(hipStreamSynchronize(st));
    return MVPB_OK;
  }
  const int N = p->N, nb = n_bands;
  const size_t NN = (size_t)N * N, blk = (size_t)3 * N * nb;   // one k: three N x nb blocks
  const size_t u_bytes = sizeof(cd) * (size_t)n_k * nb * 2 * N, s_bytes = sizeof(cd) * (size_t)n_k * blk;
  DevBuf qd(&ctx->pool), ud(&ctx->pool), sd(&ctx->pool), X(&ctx->pool), Y(&ctx->pool), ptrs(&ctx->pool);
  HIP_TRY(qd.alloc(sizeof(double) * 2 * (size_t)n_k));
  HIP_TRY(hipMemcpyAsync(qd.p, Q, sizeof(double) * 2 * (size_t)n_k, hipMemcpyHostToDevice, st));
  const cd *u_in = (const cd *)U;
  cd *s_out = (cd *)S;
  if (!dev) {
    HIP_TRY(ud.alloc(u_bytes));
    HIP_TRY(hipMemcpyAsync(ud.p, U, u_bytes, hipMemcpyHostToDevice, st));
    u_in = ud.as<cd>();
    HIP_TRY(sd.alloc(s_bytes));
    s_out = sd.as<cd>();
  }
  HIP_TRY(X.alloc(s_bytes));
  HIP_TRY(Y.alloc(s_bytes));
  HIP_TRY(launch_stress_rhs(u_in, qd.as<double>(), n_k, nb, p->M1, p->M2, p->T, p->area, X.as<cd>(), st));
  // Y = L^-1 X, then X = L^-H Y: Sigma^-1 on block 0, Delta^-1 on blocks 1, 2
  std::vector<const void *> hp;
  for (int j = 0; j < 3; ++j)
    for (int t = 0; t < n_k; ++t) hp.push_back(p->linvSD.as<cd>() + (j == 0 ? 0 : NN));
  for (int j = 0; j < 3; ++j)
    for (int t = 0; t < n_k; ++t) hp.push_back(X.as<cd>() + (size_t)t * blk + (size_t)j * N * nb);
  for (int j = 0; j < 3; ++j)
    for (int t = 0; t < n_k; ++t) hp.push_back(Y.as<cd>() + (size_t)t * blk + (size_t)j * N * nb);
  const size_t m = (size_t)3 * n_k;
  HIP_TRY(ptrs.alloc(sizeof(void *) * hp.size()));
  HIP_TRY(hipMemcpyAsync(ptrs.p, hp.data(), sizeof(void *) * hp.size(), hipMemcpyHostToDevice, st));
  void **dp = ptrs.as<void *>();
  GemmBatch b1{(const cd *const *)dp, (const cd *const *)(dp + m), (cd *const *)(dp + 2 * m), nullptr, N, N, N};
  HIP_TRY(launch_zgemm(OP_N, OP_N, N, nb, N, mk(1.0, 0.0), b1, mk(0.0, 0.0), (int)m, st));
  GemmBatch b2{(const cd *const *)dp, (const cd *const *)(dp + 2 * m), (cd *const *)(dp + m), nullptr, N, N, N};
  HIP_TRY(launch_zgemm(OP_C, OP_N, N, nb, N, mk(1.0, 0.0), b2, mk(0.0, 0.0), (int)m, st));
  HIP_TRY(launch_stress_combine(X.as<cd>(), n_k, nb, N, s_out, st));
  if (!dev) HIP_TRY(hipMemcpyAsync(S, s_out, s_bytes, hipMemcpyDeviceToHost, st));
  if (!(flags & MVPB_F_ASYNC) || !dev) HIP_TRY(hipStreamSynchronize(st));
  return MVPB_OK;
}

// Host-side check of returned frequencies: NaN marks an item whose bulge
// chasing gave up (a hand-over that never came, or a workgroup placement the
// hand-over does not support).
static int check_failed_items(const double *om, size_t count, int nb) {
  size_t bad = 0;
  for (size_t i = 0; i < count; ++i)
    if (isnan(om[i])) ++bad;
  if (bad)
    return set_err(MVPB_E_DEVICE, "the reduction to tridiagonal form gave up on %zu k-point(s)",
                   (bad + nb - 1) / nb);
  return MVPB_OK;
}

// count doubles of Bloch-vector components, all finite
static bool q_ok(const double *Q, int count) {
  for (int i = 0; i < count; ++i)
    if (!isfinite(Q[i])) return false;
  return true;
}

extern "C" int mvpb_solve(mvpb_plan p, int n_k, const double *Q, int n_bands, double *omega, double *U,
                          unsigned flags) {
  if (!p || !Q || !omega) return set_err(MVPB_E_INVALID, "NULL argument");
  if (n_k < 0) return set_err(MVPB_E_INVALID, "n_k must be non-negative");
  if (n_k == 0) return MVPB_OK;
  const int bmax = (p->prec & MVPB_PREC_EIG_FP32_RR64) ? RR_MAX_BANDS : MAX_BANDS;
  if (n_bands < 1 || n_bands > p->n || n_bands > bmax)
    return set_err(MVPB_E_INVALID, "n_bands = %d outside [1, min(n_u=%d, %d)]", n_bands, p->n, bmax);
  const int qd = p->qdim;
  if (!q_ok(Q, qd * n_k)) return set_err(MVPB_E_INVALID, "non-finite Bloch vector");
  mvpb_ctx ctx = p->ctx;
  HIP_TRY(hipSetDevice(ctx->device));
  ProfBind pb(ctx);
  hipStream_t st = ctx->stream;
  const bool dev = flags & MVPB_F_DEVICE_PTRS;
  const int n = p->n;
  // chunk the k list so that the workspace (items and the bulge-chasing
  // control words) stays within the cap
  const size_t per = item_bytes(n, n_bands, (p->prec & MVPB_PREC_EIG_FP32_RR64) != 0);
  const size_t budget = ctx->cap ? ctx->cap : (size_t)32 << 30;
  if (solve_bytes(1, per) > budget)
    return set_err(MVPB_E_NOMEM, "one item needs %zu bytes, cap is %zu", solve_bytes(1, per), budget);
  int chunk = (int)std::min<size_t>((size_t)n_k, budget / per);
  while (chunk > 1 && solve_bytes(chunk, per) > budget) --chunk;
  const bool graph = !(ctx->prof.on);
  const bool fp32 = (p->prec & MVPB_PREC_EIG_FP32_RR64) != 0;
  int rc = acc_begin(ctx);
  if (rc) return rc;
  DevBuf om_dev(&ctx->pool), u_dev(&ctx->pool);
  double *om_out = omega;
  double *u_out = U;
  if (!dev) {
    HIP_TRY(om_dev.alloc(sizeof(double) * (size_t)n_k * n_bands));
    om_out = om_dev.as<double>();
    if (U) {
      HIP_TRY(u_dev.alloc(sizeof(double) * 2 * (size_t)n_k * n_bands * n));
      u_out = u_dev.as<double>();
    }
  }
  for (int k0 = 0; k0 < n_k; k0 += chunk) {
    const int kc = std::min(chunk, n_k - k0);
    std::vector<Job> jobs(kc);
    for (int t = 0; t < kc; ++t) {
      const double *q = Q + (size_t)qd * (k0 + t);
      jobs[t] = Job{p, q[0], q[1], qd == 3 ? q[2] : 0.0, t};
    }
    rc = run_items(ctx, jobs, n_bands, om_out + (size_t)k0 * n_bands,
                   u_out ? u_out + 2 * (size_t)k0 * n_bands * n : nullptr, graph);
    if (rc) return rc;
  }
  if (!dev) {
    HIP_TRY(hipMemcpyAsync(omega, om_out, sizeof(double) * (size_t)n_k * n_bands, hipMemcpyDeviceToHost, st));
    if (U)
      HIP_TRY(hipMemcpyAsync(U, u_out, sizeof(double) * 2 * (size_t)n_k * n_bands * n, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    rc = check_failed_items(omega, (size_t)n_k * n_bands, n_bands);
    return rc ? rc : acc_finish(ctx, fp32);
  } else if (!(flags & MVPB_F_ASYNC)) {
    HIP_TRY(hipStreamSynchronize(st));
    return acc_finish(ctx, fp32);
  }
  return MVPB_OK;
}

extern "C" int mvpb_solve_batch(mvpb_ctx ctx, int n_plans, const mvpb_plan *plans, const int *n_k,
                                const double *const *Q, int n_bands, double *const *omega, unsigned flags) {
  int rc = check_ctx(ctx);
  if (rc) return rc;
  if (n_plans < 0 || (n_plans > 0 && (!plans || !n_k || !Q || !omega)))
    return set_err(MVPB_E_INVALID, "NULL argument");
  if (n_bands < 1 || n_bands > MAX_BANDS) return set_err(MVPB_E_INVALID, "n_bands = %d out of range", n_bands);
  std::vector<Job> jobs;
  std::vector<size_t> base(n_plans + 1, 0);
  for (int i = 0; i < n_plans; ++i) {
    if (!plans[i] || plans[i]->ctx != ctx) return set_err(MVPB_E_INVALID, "plan %d missing or from another context", i);
    if (n_k[i] < 0 || (n_k[i] > 0 && (!Q[i] || !omega[i]))) return set_err(MVPB_E_INVALID, "plan %d: bad k list", i);
    if (plans[i]->n < n_bands) return set_err(MVPB_E_INVALID, "plan %d: n_bands > n_u", i);
    if ((plans[i]->prec & MVPB_PREC_EIG_FP32_RR64) != (plans[0]->prec & MVPB_PREC_EIG_FP32_RR64))
      return set_err(MVPB_E_INVALID, "plan %d: all plans of a batch need the same eigensolver precision", i);
    if ((plans[i]->prec & MVPB_PREC_EIG_FP32_RR64) && n_bands > RR_MAX_BANDS)
      return set_err(MVPB_E_INVALID, "the FP32 reduction takes at most %d bands", RR_MAX_BANDS);
    const int qd = plans[i]->qdim;
    if (!q_ok(Q[i], qd * n_k[i])) return set_err(MVPB_E_INVALID, "plan %d: non-finite Bloch vector", i);
    base[i + 1] = base[i] + n_k[i];
    for (int t = 0; t < n_k[i]; ++t) {
      const double *q = Q[i] + (size_t)qd * t;
      jobs.push_back(Job{plans[i], q[0], q[1], qd == 3 ? q[2] : 0.0, (int)(base[i] + t)});
    }
  }
  if (jobs.empty()) return MVPB_OK;
  HIP_TRY(hipSetDevice(ctx->device));
  hipStream_t st = ctx->stream;
  // largest items first so the longest work starts earliest; chunks of
  // similar size share one launch sequence (captured once, replayed)
  std::stable_sort(jobs.begin(), jobs.end(), [](const Job &a, const Job &b) { return a.plan->n > b.plan->n; });
  const bool fp32 = (jobs[0].plan->prec & MVPB_PREC_EIG_FP32_RR64) != 0;
  const size_t budget = ctx->cap ? ctx->cap : (size_t)24 << 30;
  rc = acc_begin(ctx);
  if (rc) return rc;
  DevBuf om(&ctx->pool);
  HIP_TRY(om.alloc(sizeof(double) * base[n_plans] * n_bands));
  size_t j0 = 0;
  while (j0 < jobs.size()) {
    size_t j1 = j0, bytes = 0;
    const int n0 = jobs[j0].plan->n;
    while (j1 < jobs.size()) {
      const size_t b = item_bytes(jobs[j1].plan->n, n_bands, fp32);
      // keep items of one chunk within a factor ~1.5 in order so that the
      // launch sequence sized for the largest wastes little on the rest
      if (j1 > j0 && (bytes + b + ctl_bytes(j1 - j0 + 1) > budget || 3 * jobs[j1].plan->n < 2 * n0)) break;
      bytes += b;
      ++j1;
    }
    if (bytes + ctl_bytes(j1 - j0) > budget)
      return set_err(MVPB_E_NOMEM, "one item needs %zu bytes, cap is %zu", bytes + ctl_bytes(j1 - j0), budget);
    std::vector<Job> part(jobs.begin() + j0, jobs.begin() + j1);
    rc = run_items(ctx, part, n_bands, om.as<double>(), nullptr, true);
    if (rc) return rc;
    j0 = j1;
  }
  const bool dev = flags & MVPB_F_DEVICE_PTRS;
  for (int i = 0; i < n_plans; ++i) {
    if (n_k[i] == 0) continue;
    HIP_TRY(hipMemcpyAsync(omega[i], om.as<double>() + base[i] * n_bands, sizeof(double) * n_k[i] * n_bands,
                           dev ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, st));
  }
  if (!dev || !(flags & MVPB_F_ASYNC)) HIP_TRY(hipStreamSynchronize(st));
  if (!dev)
    for (int i = 0; i < n_plans; ++i) {
      rc = check_failed_items(omega[i], (size_t)n_k[i] * n_bands, n_bands);
      if (rc) return rc;
    }
  if (!dev || !(flags & MVPB_F_ASYNC)) return acc_finish(ctx, fp32);
  return MVPB_OK;
}

// ---------------------------------------------------------------------------
// Many pixel cells: plan build and eigensolve in one captured graph
// ---------------------------------------------------------------------------
constexpr size_t MAX_CELL_GRAPHS = 4;

namespace {
// Cells of one cutoff at sorted positions [c0, c1), with their offsets in
// the workspace (o_*) and in the per-call table region (t_*, bytes).
struct CellGroup {
  int M1, M2, N, c0, c1;
  size_t o_coef;                      // coefficient matrices of cell c0
  size_t t_ptrs;                      // pointer table of the factorisations and GEMMs
  size_t n_ptrs, o_inv, o_pA, o_pB, o_pC, o_pS, o_xA, o_xB, o_xC;   // entries in it
  size_t t_gvec, t_scale;             // G vectors (3 N per cell), combine scales
  struct Run {                        // structure-factor launch: cells of one grid
    int k0, cnt;
    size_t t_tab;                     // phase pointers, weight-table pointers, areas
  };
  std::vector<Run> runs;
};
struct CellChunk {                    // eigensolve launch sequence over sorted jobs [j0, j1)
  size_t j0, j1;
  size_t t_items;                     // item table
  TuneParams tp;
};
}  // namespace

extern "C" int mvpb_solve_cells(mvpb_ctx ctx, int n_cells, const mvpb_cell *cells, const int *M1, const int *M2,
                                int precision, const int *n_k, const double *const *Q, int n_bands,
                                double *const *omega, unsigned flags) {
  int rc = check_ctx(ctx);
  if (rc) return rc;
  if (n_cells < 0 || (n_cells > 0 && (!cells || !M1 || !M2 || !n_k || !Q || !omega)))
    return set_err(MVPB_E_INVALID, "NULL argument");
  rc = check_precision(precision);
  if (rc) return rc;
  if (precision & (MVPB_PREC_SF_PLAIN64 | MVPB_PREC_GENERAL))
    return set_err(MVPB_E_UNSUPPORTED, "mvpb_solve_cells takes the matrix-core structure factors and the isotropic layout");
  const bool fp32 = (precision & MVPB_PREC_EIG_FP32_RR64) != 0;
  const int bmax = fp32 ? RR_MAX_BANDS : MAX_BANDS;
  if (n_bands < 1 || n_bands > bmax) return set_err(MVPB_E_INVALID, "n_bands = %d out of range 1..%d", n_bands, bmax);
  std::vector<size_t> base(n_cells + 1, 0);
  for (int i = 0; i < n_cells; ++i) {
    const mvpb_cell c = cells[i];
    if (!c || c->ctx != ctx) return set_err(MVPB_E_INVALID, "cell %d missing or from another context", i);
    if (c->polygons || c->dim != 2 || c->general)
      return set_err(MVPB_E_UNSUPPORTED, "cell %d: mvpb_solve_cells takes isotropic pixel cells", i);
    rc = check_cutoff(M1[i], M2[i]);
    if (rc) return rc;
    if (2 * (2 * M1[i] + 1) * (2 * M2[i] + 1) < n_bands) return set_err(MVPB_E_INVALID, "cell %d: n_bands > n_u", i);
    if (n_k[i] < 0 || (n_k[i] > 0 && (!Q[i] || !omega[i]))) return set_err(MVPB_E_INVALID, "cell %d: bad k list", i);
    if (!q_ok(Q[i], 2 * n_k[i])) return set_err(MVPB_E_INVALID, "cell %d: non-finite Bloch vector", i);
    base[i + 1] = base[i] + n_k[i];
  }
  if (n_cells == 0) return MVPB_OK;
  HIP_TRY(hipSetDevice(ctx->device));
  hipStream_t st = ctx->stream;
  const int sfp = precision & 3;

  // cells sorted by cutoff, then grid: groups of one cutoff, runs of one grid
  std::vector<int> ord(n_cells);
  for (int i = 0; i < n_cells; ++i) ord[i] = i;
  std::stable_sort(ord.begin(), ord.end(), [&](int a, int b) {
    if (M1[a] != M1[b]) return M1[a] < M1[b];
    if (M2[a] != M2[b]) return M2[a] < M2[b];
    if (cells[a]->nx != cells[b]->nx) return cells[a]->nx < cells[b]->nx;
    return cells[a]->ny < cells[b]->ny;
  });
  std::vector<int> pos(n_cells);   // sorted position of caller cell i
  for (int s = 0; s < n_cells; ++s) pos[ord[s]] = s;
  size_t tab = 0;   // table region bytes
  auto take_tab = [&](size_t b) {
    const size_t o = tab;
    tab += align256(b);
    return o;
  };
  std::vector<CellGroup> groups;
  size_t coef_bytes = 0, temp_bytes = 0;
  for (int s = 0; s < n_cells;) {
    CellGroup g{};
    g.M1 = M1[ord[s]];
    g.M2 = M2[ord[s]];
    g.N = (2 * g.M1 + 1) * (2 * g.M2 + 1);
    g.c0 = s;
    // at most ~8 GB of temporaries and 2048 cells (GEMM grid depth 18 per cell) per group
    const size_t per = 30 * (size_t)g.N * g.N * sizeof(cd) + 64 * (size_t)g.N * sizeof(cd);
    const int gmax = (int)std::max<size_t>(1, std::min<size_t>(2048, ((size_t)8 << 30) / per));
    while (s < n_cells && M1[ord[s]] == g.M1 && M2[ord[s]] == g.M2 && s - g.c0 < gmax) ++s;
    g.c1 = s;
    const size_t cnt = g.c1 - g.c0, NN = (size_t)g.N * g.N;
    const int nm = 4 * g.M1 + 1, nq = 4 * g.M2 + 1;
    g.o_coef = coef_bytes;
    coef_bytes += align256(sizeof(cd) * 15 * NN * cnt);
    size_t xmax = 0;
    for (int k = g.c0; k < g.c1;) {
      CellGroup::Run r{k, 0, 0};
      const mvpb_cell c0 = cells[ord[k]];
      while (k < g.c1 && cells[ord[k]]->nx == c0->nx && cells[ord[k]]->ny == c0->ny) ++k;
      r.cnt = k - r.k0;
      r.t_tab = take_tab((2 * sizeof(void *) + sizeof(double)) * r.cnt);
      xmax = std::max(xmax, sizeof(double) * 8 * (size_t)c0->nx * nq * r.cnt);
      g.runs.push_back(r);
    }
    // temporaries of the group: F, X, Toeplitz matrices, inverse factors, P, products
    const size_t t = align256(sizeof(cd) * 4 * (size_t)nm * nq * cnt) + align256(xmax) +
                     4 * align256(sizeof(cd) * 3 * NN * cnt) /* mats, linv: 3 NN each; P: 6 NN */ +
                     align256(sizeof(cd) * 18 * NN * cnt);
    temp_bytes = std::max(temp_bytes, t);
    g.n_ptrs = 6 * cnt + 4 * 6 * cnt + 3 * 18 * cnt;
    g.t_ptrs = take_tab(sizeof(void *) * g.n_ptrs);
    g.t_gvec = take_tab(sizeof(double) * 3 * (size_t)g.N * cnt);
    g.t_scale = take_tab(sizeof(double) * cnt);
    groups.push_back(std::move(g));
  }
  // jobs, largest operators first; chunks as in mvpb_solve_batch
  struct CJob {
    int s;         // sorted cell position
    int t;         // k index
  };
  std::vector<CJob> jobs;
  for (int s = 0; s < n_cells; ++s)
    for (int t = 0; t < n_k[ord[s]]; ++t) jobs.push_back(CJob{s, t});
  auto order_of = [&](const CJob &j) { return 2 * (2 * M1[ord[j.s]] + 1) * (2 * M2[ord[j.s]] + 1); };
  std::stable_sort(jobs.begin(), jobs.end(), [&](const CJob &a, const CJob &b) { return order_of(a) > order_of(b); });
  const size_t stat_bytes = align256(sizeof(int) * 3 * n_cells);
  const size_t om_bytes = align256(sizeof(double) * base[n_cells] * n_bands);
  const size_t fixed = coef_bytes + temp_bytes + stat_bytes + om_bytes;
  size_t budget = (size_t)24 << 30;
  if (ctx->cap) {
    if (fixed + tab >= ctx->cap)
      return set_err(MVPB_E_NOMEM, "plan build of %d cells needs %zu bytes, cap is %zu", n_cells, fixed + tab, ctx->cap);
    budget = std::min(budget, ctx->cap - fixed - tab);
  }
  std::vector<CellChunk> chunks;
  size_t item_region = 0;
  for (size_t j0 = 0; j0 < jobs.size();) {
    size_t j1 = j0, bytes = 0;
    const int n0 = order_of(jobs[j0]);
    while (j1 < jobs.size()) {
      const size_t b = item_bytes(order_of(jobs[j1]), n_bands, fp32);
      if (j1 > j0 && (bytes + b + ctl_bytes(j1 - j0 + 1) > budget || 3 * order_of(jobs[j1]) < 2 * n0)) break;
      bytes += b;
      ++j1;
    }
    bytes += ctl_bytes(j1 - j0);
    if (bytes > budget) return set_err(MVPB_E_NOMEM, "one item needs %zu bytes, the budget is %zu", bytes, budget);
    CellChunk ch{j0, j1, take_tab(sizeof(EigItem) * (j1 - j0)), TuneParams{}};
    auto f = ctx->tune.find(size_class(n0));
    if (f != ctx->tune.end()) ch.tp = f->second;
    chunks.push_back(ch);
    item_region = std::max(item_region, bytes);
    j0 = j1;
  }
  // workspace: tables | coefficients | status | temporaries | frequencies | items
  const size_t o_coef = align256(tab), o_stat = o_coef + coef_bytes, o_temp = o_stat + stat_bytes,
               o_om = o_temp + temp_bytes, o_items = o_om + om_bytes, total = o_items + item_region;
  if (ctx->cap && total > ctx->cap)
    return set_err(MVPB_E_NOMEM, "workspace %zu bytes exceeds the cap of %zu bytes", total, ctx->cap);
  // the staging may still feed an earlier copy; graphs point into the workspace
  HIP_TRY(hipStreamSynchronize(st));
  if (total > ctx->cws.bytes) {
    for (auto &kv : ctx->cell_graphs) (void)hipGraphExecDestroy(kv.second.exec);
    ctx->cell_graphs.clear();
    ctx->cws.pool = nullptr;
    HIP_TRY(ctx->cws.alloc(total));
  }
  char *W = ctx->cws.as<char>();
  int *stat = reinterpret_cast<int *>(W + o_stat);
  double *om = reinterpret_cast<double *>(W + o_om);

  // per-call tables
  std::vector<char> &stage = ctx->cell_stage;
  stage.assign(tab, 0);
  auto put_ptr = [&](size_t off, size_t i, const void *p) { memcpy(stage.data() + off + i * sizeof(void *), &p, sizeof p); };
  auto put_dbl = [&](size_t off, size_t i, double v) { memcpy(stage.data() + off + i * sizeof(double), &v, sizeof v); };
  for (CellGroup &g : groups) {
    const size_t cnt = g.c1 - g.c0, NN = (size_t)g.N * g.N;
    const int nm = 4 * g.M1 + 1, nq = 4 * g.M2 + 1;
    for (const CellGroup::Run &r : g.runs)
      for (int k = 0; k < r.cnt; ++k) {
        const mvpb_cell c = cells[ord[r.k0 + k]];
        put_ptr(r.t_tab, k, c->phase.p);
        put_ptr(r.t_tab, r.cnt + k, c->wtab.p);
        put_dbl(r.t_tab + 2 * sizeof(void *) * r.cnt, k, c->area);
      }
    char *tp = W + o_temp;
    cd *F = reinterpret_cast<cd *>(tp);
    tp += align256(sizeof(cd) * 4 * (size_t)nm * nq * cnt);
    (void)F;
    size_t xmax = 0;
    for (const CellGroup::Run &r : g.runs)
      xmax = std::max(xmax, sizeof(double) * 8 * (size_t)cells[ord[r.k0]]->nx * nq * r.cnt);
    tp += align256(xmax);
    cd *Tm = reinterpret_cast<cd *>(tp);
    tp += align256(sizeof(cd) * 3 * NN * cnt);
    cd *Li = reinterpret_cast<cd *>(tp);
    tp += align256(sizeof(cd) * 3 * NN * cnt);
    cd *Pm = reinterpret_cast<cd *>(tp);
    tp += 2 * align256(sizeof(cd) * 3 * NN * cnt);
    cd *Xm = reinterpret_cast<cd *>(tp);
    const double *gvd = reinterpret_cast<const double *>(W + g.t_gvec);
    // the pointer table of build_plan_group's factorisation and GEMMs
    size_t e = 0;
    auto push = [&](const void *p) { put_ptr(g.t_ptrs, e++, p); };
    for (size_t c = 0; c < cnt; ++c)
      for (int i = 0; i < 3; ++i) push(Tm + (3 * c + i) * NN);
    g.o_inv = e;
    for (size_t c = 0; c < cnt; ++c)
      for (int i = 0; i < 3; ++i) push(Li + (3 * c + i) * NN);
    g.o_pA = e;
    for (size_t c = 0; c < cnt; ++c)
      for (int x = 0; x < 2; ++x)
        for (int l = 0; l < 3; ++l) push(Li + (3 * c + 2) * NN);
    g.o_pB = e;
    for (size_t c = 0; c < cnt; ++c)
      for (int x = 0; x < 2; ++x)
        for (int l = 0; l < 3; ++l) push(Li + (3 * c + x) * NN);
    g.o_pC = e;
    for (size_t c = 0; c < cnt; ++c)
      for (int x = 0; x < 2; ++x)
        for (int l = 0; l < 3; ++l) push(Pm + (6 * c + x * 3 + l) * NN);
    g.o_pS = e;
    for (size_t c = 0; c < cnt; ++c)
      for (int x = 0; x < 2; ++x)
        for (int l = 0; l < 3; ++l) push(gvd + 3 * (size_t)g.N * c + l * g.N);
    g.o_xA = e;
    for (size_t c = 0; c < cnt; ++c)
      for (int x = 0; x < 2; ++x)
        for (int l = 0; l < 3; ++l)
          for (int m = 0; m < 3; ++m) push(Pm + (6 * c + x * 3 + l) * NN);
    g.o_xB = e;
    for (size_t c = 0; c < cnt; ++c)
      for (int x = 0; x < 2; ++x)
        for (int l = 0; l < 3; ++l)
          for (int m = 0; m < 3; ++m) push(Pm + (6 * c + x * 3 + m) * NN);
    g.o_xC = e;
    for (size_t c = 0; c < cnt; ++c)
      for (int x = 0; x < 2; ++x)
        for (int l = 0; l < 3; ++l)
          for (int m = 0; m < 3; ++m) push(Xm + (18 * c + x * 9 + l * 3 + m) * NN);
    if (e != g.n_ptrs) return set_err(MVPB_E_DEVICE, "internal: pointer table of %zu entries, expected %zu", e, g.n_ptrs);
    // G_l vectors at Q = 0 and the coefficient scales |Omega|^2 / 2
    for (size_t c = 0; c < cnt; ++c) {
      const mvpb_cell cl = cells[ord[g.c0 + c]];
      for (int a = -g.M1; a <= g.M1; ++a)
        for (int b = -g.M2; b <= g.M2; ++b) {
          const size_t r = (size_t)(a + g.M1) * (2 * g.M2 + 1) + (b + g.M2);
          const size_t o = 3 * (size_t)g.N * c;
          put_dbl(g.t_gvec, o + r, 1.0);
          put_dbl(g.t_gvec, o + g.N + r, 2.0 * M_PI * (cl->T[0] * a + cl->T[1] * b));
          put_dbl(g.t_gvec, o + 2 * g.N + r, 2.0 * M_PI * (cl->T[2] * a + cl->T[3] * b));
        }
      put_dbl(g.t_scale, c, 0.5 * cl->area * cl->area);
    }
  }
  // item tables: each chunk carves its items from the start of the item region
  std::vector<size_t> grp_of(n_cells);
  for (size_t gi = 0; gi < groups.size(); ++gi)
    for (int s = groups[gi].c0; s < groups[gi].c1; ++s) grp_of[s] = gi;
  for (const CellChunk &ch : chunks) {
    size_t off = 0;
    for (size_t j = ch.j0; j < ch.j1; ++j) {
      const CJob &jb = jobs[j];
      const int ci = ord[jb.s];
      const CellGroup &g = groups[grp_of[jb.s]];
      const int n = 2 * g.N;
      EigItem it = carve_item(W + o_items + off, n, n_bands, fp32);
      off += item_bytes(n, n_bands, fp32);
      it.coef = reinterpret_cast<cd *>(W + o_coef + g.o_coef) + (size_t)(jb.s - g.c0) * 15 * g.N * g.N;
      it.N = g.N;
      it.n = n;
      it.dim = 0;
      it.check = fp32 ? 1 : 0;
      it.nb = n_bands;
      it.slot = (int)(base[ci] + jb.t);
      const double *q = Q[ci] + 2 * (size_t)jb.t;
      const double *T = cells[ci]->T;
      it.kap1 = 2.0 * M_PI * (T[0] * q[0] + T[1] * q[1]);
      it.kap2 = 2.0 * M_PI * (T[2] * q[0] + T[3] * q[1]);
      it.kap3 = 0.0;
      memcpy(stage.data() + ch.t_items + (j - ch.j0) * sizeof(EigItem), &it, sizeof it);
    }
  }
  // fork/join events of every chunk's stage 1 (one set per chunk, so that the
  // captured dependencies of one chunk never alias another's)
  while (ctx->cell_events.size() < chunks.size() * (MAX_SIDE + 1)) {
    hipEvent_t ev;
    HIP_TRY(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
    ctx->cell_events.push_back(ev);
  }
  // step events of the chunks' stage 1, one range per chunk
  std::vector<size_t> la_base(chunks.size() + 1, 0);
  for (size_t c = 0; c < chunks.size(); ++c)
    la_base[c + 1] = la_base[c] + la_events_needed(order_of(jobs[chunks[c].j0]), MAX_SIDE + 1);
  HIP_TRY(reserve_la_events(ctx, la_base[chunks.size()]));
  rc = acc_begin(ctx);
  if (rc) return rc;
  HIP_TRY(hipMemcpyAsync(W, stage.data(), tab, hipMemcpyHostToDevice, st));

  // the launch sequence: every group's plan build, then every chunk's eigensolve
  auto enqueue = [&]() -> hipError_t {
    hipError_t e = hipSuccess;
    int *gstat = stat;
    for (const CellGroup &g : groups) {
      const int cnt = g.c1 - g.c0;
      const size_t NN = (size_t)g.N * g.N;
      const int nm = 4 * g.M1 + 1, nq = 4 * g.M2 + 1;
      const size_t fsz = (size_t)4 * nm * nq;
      char *tp = W + o_temp;
      cd *F = reinterpret_cast<cd *>(tp);
      tp += align256(sizeof(cd) * fsz * cnt);
      double *X = reinterpret_cast<double *>(tp);
      for (const CellGroup::Run &r : g.runs) {
        void **tb = reinterpret_cast<void **>(W + r.t_tab);
        const mvpb_cell c0 = cells[ord[r.k0]];
        if (e == hipSuccess)
          e = launch_structure_factors_mfma_batch(sfp, (const int32_t *const *)tb, (const double *const *)(tb + r.cnt),
                                                  reinterpret_cast<const double *>(tb + 2 * r.cnt), r.cnt, c0->nx,
                                                  c0->ny, g.M1, g.M2, X, F + (size_t)(r.k0 - g.c0) * fsz, st);
      }
      size_t xmax = 0;
      for (const CellGroup::Run &r : g.runs)
        xmax = std::max(xmax, sizeof(double) * 8 * (size_t)cells[ord[r.k0]]->nx * nq * r.cnt);
      tp += align256(xmax);
      cd *Tm = reinterpret_cast<cd *>(tp);
      tp += align256(sizeof(cd) * 3 * NN * cnt);
      tp += align256(sizeof(cd) * 3 * NN * cnt);   // inverse factors
      tp += 2 * align256(sizeof(cd) * 3 * NN * cnt);   // P
      cd *Xm = reinterpret_cast<cd *>(tp);
      void **dp = reinterpret_cast<void **>(W + g.t_ptrs);
      if (e == hipSuccess) e = launch_toeplitz_scatter(F, g.M1, g.M2, g.N, Tm, cnt, st);
      if (e == hipSuccess) e = launch_potrf_trtri((cd *const *)dp, (cd *const *)(dp + g.o_inv), gstat, 3 * cnt, g.N, st);
      if (e == hipSuccess) e = launch_identity_if_failed((cd *const *)(dp + g.o_inv), gstat, 3 * cnt, g.N, st);
      if (e == hipSuccess) {
        GemmBatch bt{(const cd *const *)(dp + g.o_pA), (const cd *const *)(dp + g.o_pB), (cd *const *)(dp + g.o_pC),
                     (const double *const *)(dp + g.o_pS), g.N, g.N, g.N};
        e = launch_zgemm(OP_N, OP_C, g.N, g.N, g.N, mk(1.0, 0.0), bt, mk(0.0, 0.0), 6 * cnt, st);
      }
      if (e == hipSuccess) {
        GemmBatch bt{(const cd *const *)(dp + g.o_xA), (const cd *const *)(dp + g.o_xB), (cd *const *)(dp + g.o_xC),
                     nullptr, g.N, g.N, g.N};
        e = launch_zgemm(OP_N, OP_C, g.N, g.N, g.N, mk(1.0, 0.0), bt, mk(0.0, 0.0), 18 * cnt, st);
      }
      if (e == hipSuccess)
        e = launch_combine_batch(Xm, g.N, reinterpret_cast<const double *>(W + g.t_scale),
                                 reinterpret_cast<cd *>(W + o_coef + g.o_coef), cnt, st);
      gstat += 3 * cnt;
    }
    int *ctl = nullptr;
    for (const CellChunk &ch : chunks) {
      const int cnt = (int)(ch.j1 - ch.j0);
      std::vector<int> orders(cnt);
      for (int i = 0; i < cnt; ++i) orders[i] = order_of(jobs[ch.j0 + i]);
      size_t item_sum = 0;
      for (int n : orders) item_sum += item_bytes(n, n_bands, fp32);
      ctl = reinterpret_cast<int *>(W + o_items + item_sum);
      const EigItem *d_items = reinterpret_cast<const EigItem *>(W + ch.t_items);
      Stage2Shape sh;
      sh.group = ch.tp.group;
      sh.wg_max = ch.tp.wg_max;
      sh.spin_limit = ctx->spin_limit;
      const int parts = std::max(1, std::min(ch.tp.parts, MAX_SIDE + 1));
      const hipEvent_t *ev = ctx->cell_events.data() + (size_t)(&ch - chunks.data()) * (MAX_SIDE + 1);
      if (e == hipSuccess)
        e = enqueue_eigensolve(ctx, d_items, orders, true, false, n_bands, fp32, parts, sh, ctl, st, ev[0], ev + 1,
                               ctx->la_events.data() + la_base[&ch - chunks.data()]);
      if (e == hipSuccess) {
        hipLaunchKernelGGL(gather_omega, dim3((cnt * n_bands + 255) / 256), dim3(256), 0, st, d_items, cnt, n_bands, om);
        hipLaunchKernelGGL(max_acc, dim3(1), dim3(256), 0, st, d_items, cnt, ctx->accbuf.as<double>());
        e = hipGetLastError();
      }
    }
    return e;
  };
  // the graph of this shape (captured on first use)
  std::string key;
  {
    auto put = [&](long long v) { key.append(reinterpret_cast<const char *>(&v), sizeof v); };
    put(precision);
    put(n_bands);
    put(ctx->spin_limit);
    put((long long)budget);
    put(n_cells);
    for (int s = 0; s < n_cells; ++s) {
      const int i = ord[s];
      put(M1[i]);
      put(M2[i]);
      put(cells[i]->nx);
      put(cells[i]->ny);
      put(n_k[i]);
    }
    for (const CellChunk &ch : chunks) {
      put(ch.tp.parts);
      put(ch.tp.group);
      put(ch.tp.wg_max);
    }
  }
  hipGraphExec_t exec = nullptr;
  auto found = ctx->cell_graphs.find(key);
  if (found == ctx->cell_graphs.end()) {
    if (ctx->cell_graphs.size() >= MAX_CELL_GRAPHS) {
      auto lru = ctx->cell_graphs.begin();
      for (auto it = ctx->cell_graphs.begin(); it != ctx->cell_graphs.end(); ++it)
        if (it->second.last_use < lru->second.last_use) lru = it;
      HIP_TRY(hipStreamSynchronize(st));
      (void)hipGraphExecDestroy(lru->second.exec);
      ctx->cell_graphs.erase(lru);
    }
    hipGraph_t gr;
    HIP_TRY(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
    Profiler *saved = t_prof;
    t_prof = nullptr;  // no event records inside the captured graph
    hipError_t e = enqueue();
    t_prof = saved;
    hipError_t e2 = hipStreamEndCapture(st, &gr);
    if (e != hipSuccess) return set_err(MVPB_E_DEVICE, "graph capture: %s", hipGetErrorString(e));
    if (e2 != hipSuccess) return set_err(MVPB_E_DEVICE, "graph capture end: %s", hipGetErrorString(e2));
    e = hipGraphInstantiate(&exec, gr, nullptr, nullptr, 0);
    (void)hipGraphDestroy(gr);
    if (e != hipSuccess) return set_err(MVPB_E_DEVICE, "graph instantiate: %s", hipGetErrorString(e));
    ctx->cell_graphs[key] = mvpb_ctx_s::GraphEntry{exec, ++ctx->graph_clock};
  } else {
    exec = found->second.exec;
    found->second.last_use = ++ctx->graph_clock;
  }
  HIP_TRY(hipGraphLaunch(exec, st));
  // results, then the factorisation status of every cell
  const bool dev = flags & MVPB_F_DEVICE_PTRS;
  for (int i = 0; i < n_cells; ++i) {
    if (n_k[i] == 0) continue;
    HIP_TRY(hipMemcpyAsync(omega[i], om + base[i] * n_bands, sizeof(double) * n_k[i] * n_bands,
                           dev ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, st));
  }
  std::vector<int> hstat(3 * (size_t)n_cells, 0);
  HIP_TRY(hipMemcpyAsync(hstat.data(), stat, sizeof(int) * 3 * n_cells, hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  const char *names[3] = {"compliance block Phi(d11+d12)", "compliance block Phi(d11-d12)", "density matrix Omega"};
  for (int i = 0; i < n_cells; ++i)
    for (int m = 0; m < 3; ++m)
      if (hstat[3 * (size_t)pos[i] + m])
        return set_err(MVPB_E_NOT_PD, "cell %d: %s is not positive definite (pivot %d)", i, names[m],
                       hstat[3 * (size_t)pos[i] + m] - 1);
  if (!dev)
    for (int i = 0; i < n_cells; ++i) {
      rc = check_failed_items(omega[i], (size_t)n_k[i] * n_bands, n_bands);
      if (rc) return rc;
    }
  return acc_finish(ctx, fp32);
}

extern "C" int mvpb_ctx_set_accuracy(mvpb_ctx ctx, double tol) {
  int rc = check_ctx(ctx);
  if (rc) return rc;
  if (!(tol >= 0.0) || !isfinite(tol)) return set_err(MVPB_E_INVALID, "tolerance must be finite and >= 0");
  ctx->acc_tol = tol;
  return MVPB_OK;
}

extern "C" int mvpb_ctx_last_accuracy(mvpb_ctx ctx, double *estimate) {
  int rc = check_ctx(ctx);
  if (rc) return rc;
  if (!estimate) return set_err(MVPB_E_INVALID, "NULL argument");
  *estimate = ctx->last_acc;
  return MVPB_OK;
}

// ---------------------------------------------------------------------------
// Autotuning of the eigensolve's launch shape
// ---------------------------------------------------------------------------
static std::string device_key(int device) {
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) != hipSuccess) return "unknown";
  std::string k = std::string(prop.gcnArchName) + " " + prop.name;
  for (char &c : k)
    if (c == '"' || c == '\\' || c == '\n') c = ' ';
  return k;
}

// Number after "key": in line (NAN if absent).
static double json_number(const std::string &line, const char *key) {
  const std::string pat = std::string("\"") + key + "\":";
  const size_t at = line.find(pat);
  if (at == std::string::npos) return NAN;
  return strtod(line.c_str() + at + pat.size(), nullptr);
}

static std::string json_string(const std::string &line, const char *key) {
  const std::string pat = std::string("\"") + key + "\": \"";
  const size_t at = line.find(pat);
  if (at == std::string::npos) return "";
  const size_t b = at + pat.size(), e = line.find('"', b);
  return e == std::string::npos ? "" : line.substr(b, e - b);
}

// Entries of a tuning cache: one JSON object per line inside "entries".
static std::vector<std::string> read_entries(const char *path) {
  std::vector<std::string> out;
  FILE *f = fopen(path, "r");
  if (!f) return out;
  char buf[1024];
  while (fgets(buf, sizeof buf, f)) {
    std::string line(buf);
    if (line.find("\"device\"") != std::string::npos) {
      while (!line.empty() && (line.back() == '\n' || line.back() == ',' || line.back() == ' ')) line.pop_back();
      out.push_back(line);
    }
  }
  fclose(f);
  return out;
}

extern "C" int mvpb_ctx_load_tuning(mvpb_ctx ctx, const char *path, int *n_loaded) {
  int rc = check_ctx(ctx);
  if (rc) return rc;
  if (!path) return set_err(MVPB_E_INVALID, "NULL path");
  FILE *f = fopen(path, "r");
  if (!f) return set_err(MVPB_E_INVALID, "cannot open %s", path);
  fclose(f);
  const std::string dev = device_key(ctx->device);
  int n = 0;
  for (const std::string &line : read_entries(path)) {
    if (json_string(line, "device") != dev) continue;
    const double cls = json_number(line, "n_class"), parts = json_number(line, "parts"),
                 group = json_number(line, "hb2st_group"), wg = json_number(line, "hb2st_wg");
    if (!(cls >= 1) || !(parts >= 1 && parts <= MAX_SIDE + 1) || !(group >= 0 && group <= 8) || !(wg >= 0 && wg <= 4))
      return set_err(MVPB_E_INVALID, "%s: malformed tuning entry", path);
    TuneParams tp;
    tp.parts = (int)parts;
    tp.group = (int)group;
    tp.wg_max = (int)wg;
    ctx->tune[(int)cls] = tp;
    ++n;
  }
  if (n_loaded) *n_loaded = n;
  return MVPB_OK;
}

extern "C" int mvpb_ctx_set_launch_shape(mvpb_ctx ctx, int n, int parts, int group, int wg_max) {
  int rc = check_ctx(ctx);
  if (rc) return rc;
  if (n < 1 || n > MAX_N || parts < 1 || parts > MAX_SIDE + 1 || !(group == 0 || group == 1 || group == 2 ||
                                                                    group == 4 || group == 8) ||
      wg_max < 0 || wg_max > 4)
    return set_err(MVPB_E_INVALID, "bad launch shape (n %d, parts %d, group %d, workgroups %d)", n, parts, group,
                   wg_max);
  TuneParams tp;
  tp.parts = parts;
  tp.group = group;
  tp.wg_max = wg_max;
  ctx->tune[size_class(n)] = tp;
  return MVPB_OK;
}

extern "C" int mvpb_ctx_get_launch_shape(mvpb_ctx ctx, int n, int *parts, int *group, int *wg_max) {
  int rc = check_ctx(ctx);
  if (rc) return rc;
  if (n < 1 || n > MAX_N) return set_err(MVPB_E_INVALID, "n out of range");
  TuneParams tp;
  auto f = ctx->tune.find(size_class(n));
  if (f != ctx->tune.end()) tp = f->second;
  if (parts) *parts = tp.parts;
  if (group) *group = tp.group;
  if (wg_max) *wg_max = tp.wg_max;
  return MVPB_OK;
}

extern "C" int mvpb_ctx_set_wait_limit(mvpb_ctx ctx, long long spins) {
  int rc = check_ctx(ctx);
  if (rc) return rc;
  if (spins < 0) return set_err(MVPB_E_INVALID, "spins must be >= 0");
  ctx->spin_limit = spins;
  return MVPB_OK;
}

extern "C" int mvpb_autotune(mvpb_plan p, int n_k, const double *Q, int n_bands, const char *cache_path,
                             double *best_ms) {
  if (!p || !Q) return set_err(MVPB_E_INVALID, "NULL argument");
  if (n_k < 1) return set_err(MVPB_E_INVALID, "n_k must be positive");
  const int bmax = (p->prec & MVPB_PREC_EIG_FP32_RR64) ? RR_MAX_BANDS : MAX_BANDS;
  if (n_bands < 1 || n_bands > p->n || n_bands > bmax)
    return set_err(MVPB_E_INVALID, "n_bands = %d outside [1, min(n_u, %d)]", n_bands, bmax);
  const int qd = p->qdim;
  if (!q_ok(Q, qd * n_k)) return set_err(MVPB_E_INVALID, "non-finite Bloch vector");
  mvpb_ctx ctx = p->ctx;
  HIP_TRY(hipSetDevice(ctx->device));
  ProfBind pb(nullptr);
  hipStream_t st = ctx->stream;
  const bool fp32 = (p->prec & MVPB_PREC_EIG_FP32_RR64) != 0;
  const size_t need = solve_bytes(n_k, item_bytes(p->n, n_bands, fp32));
  if (ctx->cap && need > ctx->cap)
    return set_err(MVPB_E_NOMEM, "the %d points need %zu bytes of workspace, cap is %zu", n_k, need, ctx->cap);
  std::vector<Job> jobs(n_k);
  for (int t = 0; t < n_k; ++t) {
    const double *q = Q + (size_t)qd * t;
    jobs[t] = Job{p, q[0], q[1], qd == 3 ? q[2] : 0.0, t};
  }
  DevBuf om(&ctx->pool);
  HIP_TRY(om.alloc(sizeof(double) * (size_t)n_k * n_bands));
  int rc0 = acc_begin(ctx);
  if (rc0) return rc0;
  hipEvent_t e0, e1;
  HIP_TRY(hipEventCreate(&e0));
  HIP_TRY(hipEventCreate(&e1));
  const int cls = size_class(p->n);
  const auto saved = ctx->tune;
  // median of three timed runs of the captured launch sequence (the first
  // run of a shape captures it)
  auto trial = [&](const TuneParams &tp, double *ms) -> int {
    ctx->tune[cls] = tp;
    int rc = run_items(ctx, jobs, n_bands, om.as<double>(), nullptr, true);
    if (rc) return rc;
    double t[3];
    for (int r = 0; r < 3; ++r) {
      HIP_TRY(hipEventRecord(e0, st));
      rc = run_items(ctx, jobs, n_bands, om.as<double>(), nullptr, true);
      if (rc) return rc;
      HIP_TRY(hipEventRecord(e1, st));
      HIP_TRY(hipEventSynchronize(e1));
      float f = 0.f;
      HIP_TRY(hipEventElapsedTime(&f, e0, e1));
      t[r] = f;
    }
    std::sort(t, t + 3);
    *ms = t[1];
    return MVPB_OK;
  };
  // coordinate search from the defaults: stage-1 parts, then the sweep
  // grouping, then the workgroups per item of the bulge chasing
  TuneParams best;
  double best_t = 0.0;
  int rc = trial(best, &best_t);
  const int parts_c[] = {2, 3, 4}, group_c[] = {1, 2, 4}, wg_c[] = {1, 2};
  const double keep = 0.98;   // a candidate must beat the best so far by 2 % (stable choices under noise)
  for (int v : parts_c) {
    if (rc) break;
    TuneParams tp = best;
    tp.parts = v;
    double t = 0.0;
    rc = trial(tp, &t);
    if (!rc && t < keep * best_t) best = tp, best_t = t;
  }
  for (int v : group_c) {
    if (rc) break;
    TuneParams tp = best;
    tp.group = v;
    double t = 0.0;
    rc = trial(tp, &t);
    if (!rc && t < keep * best_t) best = tp, best_t = t;
  }
  for (int v : wg_c) {
    if (rc) break;
    TuneParams tp = best;
    tp.wg_max = v;
    double t = 0.0;
    rc = trial(tp, &t);
    if (!rc && t < keep * best_t) best = tp, best_t = t;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc) {
    ctx->tune = saved;
    return rc;
  }
  ctx->tune[cls] = best;
  if (best_ms) *best_ms = best_t;
  if (cache_path) {
    // merge: every entry of the file except this device's entry for this class
    const std::string dev = device_key(ctx->device);
    std::vector<std::string> keep;
    for (const std::string &line : read_entries(cache_path))
      if (!(json_string(line, "device") == dev && (int)json_number(line, "n_class") == cls)) keep.push_back(line);
    char mine[512];
    snprintf(mine, sizeof mine,
             "{\"device\": \"%s\", \"n_class\": %d, \"n\": %d, \"n_bands\": %d, \"items\": %d, "
             "\"parts\": %d, \"hb2st_group\": %d, \"hb2st_wg\": %d, \"ms\": %.4f}",
             dev.c_str(), cls, p->n, n_bands, n_k, best.parts, best.group, best.wg_max, best_t);
    keep.push_back(mine);
    FILE *f = fopen(cache_path, "w");
    if (!f) return set_err(MVPB_E_INVALID, "cannot write %s", cache_path);
    fprintf(f, "{\"mvpb_tuning\": 1, \"entries\": [\n");
    for (size_t i = 0; i < keep.size(); ++i) fprintf(f, "%s%s\n", keep[i].c_str(), i + 1 < keep.size() ? "," : "");
    fprintf(f, "]}\n");
    fclose(f);
  }
  return MVPB_OK;
}

__global__ void __launch_bounds__(256) copy16(uint4 *__restrict__ dst, const uint4 *__restrict__ src, size_t n) {
  for (size_t e = blockIdx.x * (size_t)256 + threadIdx.x; e < n; e += (size_t)gridDim.x * 256) dst[e] = src[e];
}

extern "C" int mvpb_copy_device(mvpb_ctx ctx, void *dst, const void *src, size_t bytes) {
  int rc = check_ctx(ctx);
  if (rc) return rc;
  if (!dst || !src || bytes % 16 || ((uintptr_t)dst | (uintptr_t)src) % 16)
    return set_err(MVPB_E_INVALID, "copy needs 16-byte aligned buffers and a multiple of 16 bytes");
  const char *d = (const char *)dst, *s = (const char *)src;
  if (d < s + bytes && s < d + bytes) return set_err(MVPB_E_INVALID, "copy buffers overlap");
  if (bytes == 0) return MVPB_OK;
  HIP_TRY(hipSetDevice(ctx->device));
  const size_t n = bytes / 16;
  const unsigned grid = (unsigned)std::min<size_t>((n + 255) / 256, 8192);
  hipLaunchKernelGGL(copy16, dim3(grid), dim3(256), 0, ctx->stream, (uint4 *)dst, (const uint4 *)src, n);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipStreamSynchronize(ctx->stream));
  return MVPB_OK;
}

extern "C" int mvpb_kpath_square(int n_k, double *Q) {
  if (!Q || n_k < 1) return set_err(MVPB_E_INVALID, "bad arguments");
  const double cx[4] = {0.0, 0.5, 0.5, 0.0}, cy[4] = {0.0, 0.0, 0.5, 0.0};
  double seg[3], cum[4] = {0.0, 0.0, 0.0, 0.0};
  for (int s = 0; s < 3; ++s) {
    seg[s] = hypot(cx[s + 1] - cx[s], cy[s + 1] - cy[s]);
    cum[s + 1] = cum[s] + seg[s];
  }
  if (n_k == 1) {
    Q[0] = 0.0;
    Q[1] = 0.0;
    return MVPB_OK;
  }
  for (int t = 0; t < n_k; ++t) {
    const double s = cum[3] * (double)t / (double)(n_k - 1);
    int k = 0;
    while (k < 2 && s >= cum[k + 1]) ++k;
    const double u = (s - cum[k]) / seg[k];
    Q[2 * t] = cx[k] + u * (cx[k + 1] - cx[k]);
    Q[2 * t + 1] = cy[k] + u * (cy[k + 1] - cy[k]);
  }
  return MVPB_OK;
}

// Symmetry points by letter, fractional in (q1, q2).
static bool kpoint(char c, double *q) {
  switch (c) {
    case 'G': q[0] = 0.0; q[1] = 0.0; return true;
    case 'X': q[0] = 0.5; q[1] = 0.0; return true;
    case 'Y': q[0] = 0.0; q[1] = 0.5; return true;
    case 'M': q[0] = 0.5; q[1] = 0.5; return true;
    case 'J': q[0] = 2.0 / 3.0; q[1] = 1.0 / 3.0; return true;
    default: return false;
  }
}

extern "C" int mvpb_kpath(const double lattice[4], const char *path, int n_k, double *Q) {
  if (!lattice || !path || !Q || n_k < 1) return set_err(MVPB_E_INVALID, "bad arguments");
  double T[4], area;
  if (!lattice_ok(lattice, T, &area)) return set_err(MVPB_E_INVALID, "degenerate or non-finite lattice");
  const int nc = (int)strnlen(path, 64);
  if (nc < 1 || nc >= 64) return set_err(MVPB_E_INVALID, "path must have 1 to 63 letters");
  std::vector<double> fr(2 * nc), cum(nc, 0.0);
  for (int c = 0; c < nc; ++c)
    if (!kpoint(path[c], &fr[2 * c])) return set_err(MVPB_E_INVALID, "unknown symmetry point '%c'", path[c]);
  // arc length in Cartesian k = Q1 q^1 + Q2 q^2, q^i = 2 pi (column i of T)
  auto cart = [&](const double *f, double *k) {
    k[0] = 2.0 * M_PI * (T[0] * f[0] + T[1] * f[1]);
    k[1] = 2.0 * M_PI * (T[2] * f[0] + T[3] * f[1]);
  };
  for (int c = 1; c < nc; ++c) {
    double a[2], b[2];
    cart(&fr[2 * (c - 1)], a);
    cart(&fr[2 * c], b);
    cum[c] = cum[c - 1] + hypot(b[0] - a[0], b[1] - a[1]);
  }
  if (n_k == 1 || nc == 1 || !(cum[nc - 1] > 0.0)) {
    if (n_k > 1) return set_err(MVPB_E_INVALID, "path of zero length for %d points", n_k);
    Q[0] = fr[0];
    Q[1] = fr[1];
    return MVPB_OK;
  }
  for (int t = 0; t < n_k; ++t) {
    const double s = cum[nc - 1] * (double)t / (double)(n_k - 1);
    int k = 0;
    while (k < nc - 2 && s >= cum[k + 1]) ++k;
    const double len = cum[k + 1] - cum[k];
    const double u = len > 0.0 ? (s - cum[k]) / len : 0.0;
    Q[2 * t] = fr[2 * k] + u * (fr[2 * k + 2] - fr[2 * k]);
    Q[2 * t + 1] = fr[2 * k + 1] + u * (fr[2 * k + 3] - fr[2 * k + 1]);
  }
  return MVPB_OK;
}

// ---------------------------------------------------------------------------
// kernel timers
// ---------------------------------------------------------------------------
static const char *k_names[K_COUNT] = {"structure_factors", "toeplitz_scatter", "potrf_trtri", "zgemm",
                                       "combine_coefficients", "form_operator", "he2hb_panel", "he2hb_hemm",
                                       "he2hb_wform", "he2hb_her2k", "hb2st", "tridiag_eig", "backtransform",
                                       "rayleigh_ritz", "hb2st_copy"};

extern "C" int mvpb_ctx_profile(mvpb_ctx ctx, int enable) {
  int rc = check_ctx(ctx);
  if (rc) return rc;
  (void)hipSetDevice(ctx->device);
  ctx->prof.reset();
  ctx->prof.on = enable != 0;
  ctx->prof.mask = ~0ull;
  return MVPB_OK;
}

extern "C" int mvpb_ctx_profile_mask(mvpb_ctx ctx, unsigned long long mask) {
  int rc = check_ctx(ctx);
  if (rc) return rc;
  (void)hipSetDevice(ctx->device);
  ctx->prof.reset();
  ctx->prof.on = mask != 0;
  ctx->prof.mask = mask;
  return MVPB_OK;
}

extern "C" int mvpb_ctx_profile_read(mvpb_ctx ctx, int kernel, double *total_ms, long long *launches,
                                     const char **name) {
  int rc = check_ctx(ctx);
  if (rc) return rc;
  if (kernel < 0 || kernel >= K_COUNT) return set_err(MVPB_E_INVALID, "kernel id %d out of range", kernel);
  (void)hipSetDevice(ctx->device);
  ctx->prof.drain();
  if (total_ms) *total_ms = ctx->prof.total_ms[kernel];
  if (launches) *launches = ctx->prof.launches[kernel];
  if (name) *name = k_names[kernel];
  return MVPB_OK;
}
