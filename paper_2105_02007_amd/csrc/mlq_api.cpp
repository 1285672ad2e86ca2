// C ABI of the library: argument validation, level set-up, workspace layout and
// the host-steered time / Newton / GMRES loops of one batched solve.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "mlq_internal.h"

using namespace mlq;

namespace {

thread_local std::string g_err;

mlq_status fail(mlq_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  std::vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return st;
}

#define HIP_OK(expr)                                                                      \
  do {                                                                                    \
    hipError_t e_ = (expr);                                                               \
    if (e_ != hipSuccess) return fail(MLQ_EHIP, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

inline size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

// Exact integral of the 1D hat of node i (nodes x_j = lo + j h, j < n) over [a, b].
double hat_integral(int64_t i, int64_t n, double lo, double h, double a, double b) {
  const double xi = lo + h * (double)i;
  double s = 0.0;
  if (i > 0) {  // rising part on [x_{i-1}, x_i]: (x - x_{i-1}) / h
    const double x0 = xi - h;
    const double l = std::max(a, x0), r = std::min(b, xi);
    if (r > l) s += ((r - x0) * (r - x0) - (l - x0) * (l - x0)) / (2.0 * h);
  }
  if (i < n - 1) {  // falling part on [x_i, x_{i+1}]: (x_{i+1} - x) / h
    const double x1 = xi + h;
    const double l = std::max(a, xi), r = std::min(b, x1);
    if (r > l) s += ((x1 - l) * (x1 - l) - (x1 - r) * (x1 - r)) / (2.0 * h);
  }
  return s;
}

}  // namespace

struct mlq_level {
  mlq_level_desc d;
  int device = -1;              // HIP device current at creation (the blob's device)
  const double* ref = nullptr;  // reference space-time solution for the Newton guess (caller's memory)
  Geo geo;
  Ionic io;
  int64_t nn = 0, P = 0;
  int32_t M = 0;
  double h[3] = {1, 1, 1};
  double vol = 0.0;
  bool mixed = false;
  int kmax = 30;
  // device pointers inside the caller's level blob
  double* phi64 = nullptr;  // KL basis at the element centres, mode-major (M x P)
  float* phi32 = nullptr;   // its FP32 copy (mixed-precision synthesis)
  double* sqrt_lambda = nullptr;
  double* theta0 = nullptr;
  double* fbox = nullptr;
  double* wts = nullptr;
  void* tri = nullptr;  // 1 / pivots of tridiag(1, 4, 1) per axis, [3][nmax], inner precision
  bool tet = false;     // P1 tetrahedra
  TetDev td{};          // their device data (inside the blob)
  int nmax = 0;
  // pinned host flags: [0] Newton-active count as read, [1] the count entering the
  // current GMRES solve, [kFlagInner + j] GMRES-active count after iteration j (read
  // one iteration behind the launches)
  int32_t* host_flags = nullptr;
  hipEvent_t flag_ev[2] = {nullptr, nullptr};
  // kernel timing
  uint32_t tmask = 0;
  mlq_timing tim{};
  struct Pending {
    int cls;
    double units, bytes, kbytes, kbytes_fixed;
    const int32_t* count;  // host count of active samples the per-sample figures scale with
    hipEvent_t a, b;
  };
  std::vector<Pending> pending;
  std::vector<hipEvent_t> free_events;
  // GMRES iterations per captured graph (0: launched and steered one iteration at a time)
  int gmres_block = 0;
  // persistent per-sample solves (small 3D box levels, mlq_set_persistent)
  bool persistent = false;
  struct BlockGraph {
    const void* ws;
    const void* theta;
    int32_t batch, j0, jn;
    hipGraphExec_t exec;
  };
  std::vector<BlockGraph> graphs;
  hipStream_t cap_stream = nullptr;  // the level's own stream for capturing (the null stream cannot capture)
};

namespace {

constexpr int kFlagInner = 8;  // first host flag slot of the GMRES-active counts

hipEvent_t take_event(mlq_level* lv) {
  if (!lv->free_events.empty()) {
    hipEvent_t e = lv->free_events.back();
    lv->free_events.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// Brackets one launch with events when its class is timed.  units and bytes are totals,
// or, with count set, per active sample: the launch's figures are then resolved when the
// count (a pinned host slot filled by an asynchronous copy) is known, at harvest.  bytes are
// the algorithmic bytes, kbytes (+ kbytes_fixed per launch) what the kernel's own design moves.
template <typename F>
void timed(mlq_level* lv, int cls, double units, hipStream_t s, F&& launch, double bytes = 0.0,
           const int32_t* count = nullptr, double kbytes = 0.0, double kbytes_fixed = 0.0) {
  if (!(lv->tmask & (1u << cls))) {
    launch();
    return;
  }
  hipEvent_t a = take_event(lv), b = take_event(lv);
  if (a == nullptr || b == nullptr) {
    launch();
    return;
  }
  (void)hipEventRecord(a, s);
  launch();
  (void)hipEventRecord(b, s);
  lv->pending.push_back({cls, units, bytes, kbytes, kbytes_fixed, count, a, b});
}

// After a stream synchronisation: fold finished event pairs into the totals.
void harvest(mlq_level* lv) {
  for (auto& p : lv->pending) {
    float ms = 0.0f;
    if (hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
      const double n = p.count != nullptr ? (double)*p.count : 1.0;
      lv->tim.ms[p.cls] += ms;
      lv->tim.launches[p.cls] += 1;
      lv->tim.units[p.cls] += p.units * n;
      lv->tim.bytes[p.cls] += p.bytes * n;
      lv->tim.kernel_bytes[p.cls] += p.kbytes * n + p.kbytes_fixed;
    }
    lv->free_events.push_back(p.a);
    lv->free_events.push_back(p.b);
  }
  lv->pending.clear();
}

// Graph of the GMRES launches of iterations j0 .. j0 + jn - 1 for one workspace, field and
// batch: captured from the launches once, then replayed.  The launches read no host state that
// changes between replays (every per-step quantity of the iteration lives in the workspace).
template <typename F>
mlq_status block_graph(mlq_level* lv, const void* ws, const void* theta, int32_t batch, int j0, int jn, hipStream_t s,
                       hipGraphExec_t* out, F&& launches) {
  for (const auto& gr : lv->graphs)
    if (gr.ws == ws && gr.theta == theta && gr.batch == batch && gr.j0 == j0 && gr.jn == jn) {
      *out = gr.exec;
      return MLQ_OK;
    }
  // capture on the level's own stream (any stream records the same launches; the caller's may be
  // the null stream, which cannot capture); the graph is launched on the caller's stream
  (void)s;
  if (lv->cap_stream == nullptr) HIP_OK(hipStreamCreateWithFlags(&lv->cap_stream, hipStreamNonBlocking));
  hipGraph_t graph = nullptr;
  HIP_OK(hipStreamBeginCapture(lv->cap_stream, hipStreamCaptureModeRelaxed));
  launches(lv->cap_stream);
  hipError_t e = hipGetLastError();
  const hipError_t ee = hipStreamEndCapture(lv->cap_stream, &graph);
  if (e == hipSuccess) e = ee;
  hipGraphExec_t exec = nullptr;
  if (e == hipSuccess) e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  if (graph != nullptr) (void)hipGraphDestroy(graph);
  if (e != hipSuccess) return fail(MLQ_EHIP, "capturing the GMRES block failed: %s", hipGetErrorString(e));
  lv->graphs.push_back({ws, theta, batch, j0, jn, exec});
  *out = exec;
  return MLQ_OK;
}

void drop_graphs(mlq_level* lv) {
  for (auto& gr : lv->graphs) (void)hipGraphExecDestroy(gr.exec);
  lv->graphs.clear();
}

}  // namespace

namespace {

struct BlobLayout {
  size_t phi64, phi32, sl, th0, fbox, wts, tri;
  size_t ecol, ediag, em, em32, mdiag, mdiag32, ecptr, ecdat, geo, vmean;  // tetrahedral levels
  size_t total;
};

BlobLayout blob_layout(int64_t P, int64_t M, int64_t nn, int64_t nmax, const mlq::TetHost* th = nullptr) {
  BlobLayout L{};
  size_t o = 0;
  L.tri = o;   o = align256(o + sizeof(double) * 3 * nmax);
  L.phi64 = o; o = align256(o + sizeof(double) * P * M);
  L.phi32 = o; o = align256(o + sizeof(float) * P * M);
  L.sl = o;    o = align256(o + sizeof(double) * M);
  L.th0 = o;   o = align256(o + sizeof(double) * P);
  L.fbox = o;  o = align256(o + sizeof(double) * nn);
  L.wts = o;   o = align256(o + sizeof(double) * nn);
  if (th != nullptr) {
    L.ecol = o;    o = align256(o + sizeof(int32_t) * th->nell);
    L.ediag = o;   o = align256(o + sizeof(int32_t) * th->nv);
    L.em = o;      o = align256(o + sizeof(double) * th->nell);
    L.em32 = o;    o = align256(o + sizeof(float) * th->nell);
    L.mdiag = o;   o = align256(o + sizeof(double) * th->nv);
    L.mdiag32 = o; o = align256(o + sizeof(float) * th->nv);
    L.ecptr = o;   o = align256(o + sizeof(int32_t) * (th->nell + 1));
    L.ecdat = o;   o = align256(o + sizeof(int32_t) * th->nc);
    L.geo = o;     o = align256(o + sizeof(double) * mlq::kTetGeo * th->nt);
    L.vmean = o;   o = align256(o + sizeof(double) * 3 * th->nt);
  }
  L.total = o;
  return L;
}

mlq_status validate(const mlq_level_desc* d) {
  if (d == nullptr) return fail(MLQ_EINVAL, "descriptor is NULL");
  if (d->dim != 2 && d->dim != 3) return fail(MLQ_EINVAL, "dim must be 2 or 3 (got %d)", d->dim);
  if (d->mesh_kind != MLQ_MESH_Q1_BOX && d->mesh_kind != MLQ_MESH_P1_TET)
    return fail(MLQ_EINVAL, "unsupported mesh_kind %d", d->mesh_kind);
  if (d->mesh_kind == MLQ_MESH_P1_TET) {
    if (d->dim != 3) return fail(MLQ_EINVAL, "tetrahedral levels are 3D");
  } else for (int a = 0; a < d->dim; ++a) {
    if (d->n[a] < 2 || d->n[a] > (1 << 20)) return fail(MLQ_EINVAL, "n[%d] = %lld out of range", a, (long long)d->n[a]);
    if (!(d->hi[a] > d->lo[a])) return fail(MLQ_EINVAL, "box axis %d is empty", a);
  }
  if (d->mesh_kind == MLQ_MESH_Q1_BOX) {
    // per-sample offsets inside the kernels are 32-bit byte offsets
    double nn = 1.0;
    for (int a = 0; a < d->dim; ++a) nn *= (double)d->n[a];
    if (nn > (double)(1 << 27)) return fail(MLQ_EINVAL, "%.0f nodes per sample exceed the limit of 2^27", nn);
  }
  if (d->n_steps < 1) return fail(MLQ_EINVAL, "n_steps must be >= 1");
  if (!(d->t_end > 0.0)) return fail(MLQ_EINVAL, "t_end must be positive");
  if (!(d->sigma_l > 0.0) || !(d->sigma_t > 0.0)) return fail(MLQ_EINVAL, "conductivities must be positive");
  if (!(d->alpha >= 0.0)) return fail(MLQ_EINVAL, "alpha must be >= 0");
  if (d->n_modes < 0 || d->n_modes > 1024) return fail(MLQ_EINVAL, "n_modes must be in [0, 1024]");
  if (d->n_modes > 0 && (d->phi == nullptr || d->sqrt_lambda == nullptr))
    return fail(MLQ_EINVAL, "phi and sqrt_lambda are required when n_modes > 0");
  if (d->prec != MLQ_FP64 && d->prec != MLQ_MIXED) return fail(MLQ_EINVAL, "unknown precision %d", d->prec);
  if (d->qoi != MLQ_QOI_MEAN_U_FINAL && d->qoi != MLQ_QOI_MEAN_ACT_TIME) return fail(MLQ_EINVAL, "unknown qoi %d", d->qoi);
  if (!(d->newton_tol > 0.0) || !(d->inner_tol > 0.0)) return fail(MLQ_EINVAL, "tolerances must be positive");
  if (d->max_newton < 1 || d->max_newton > 1000) return fail(MLQ_EINVAL, "max_newton out of range");
  if (d->max_inner < 1 || d->max_inner > kMaxInner) return fail(MLQ_EINVAL, "max_inner must be in [1, %d]", kMaxInner);
  if (d->max_batch < 1 || d->max_batch > 65535) return fail(MLQ_EINVAL, "max_batch must be in [1, 65535]");
  if (d->newton_guess < MLQ_GUESS_PREVIOUS || d->newton_guess > MLQ_GUESS_REFERENCE_LOCAL)
    return fail(MLQ_EINVAL, "unknown newton_guess");
  if (d->diffusion != MLQ_DIFF_FIBRE && d->diffusion != MLQ_DIFF_ISO && d->diffusion != MLQ_DIFF_VECTOR)
    return fail(MLQ_EINVAL, "diffusion must be MLQ_DIFF_FIBRE, MLQ_DIFF_ISO or MLQ_DIFF_VECTOR");
  if (d->diffusion == MLQ_DIFF_VECTOR && d->mesh_kind != MLQ_MESH_P1_TET)
    return fail(MLQ_EINVAL, "the vector diffusion model is for tetrahedra");
  if (d->diffusion == MLQ_DIFF_VECTOR && d->v_mean == nullptr) return fail(MLQ_EINVAL, "v_mean is NULL");
  // uniqueness of the step equation: dt * |min I_ion'| < 1 (min over u of the cubic's derivative)
  const double dt = d->t_end / d->n_steps;
  const double r = d->u_rest, t = d->u_th, p = d->u_peak;
  const double umin = (r + t + p) / 3.0;
  const double dmin = d->alpha * ((umin - t) * (umin - p) + (umin - r) * (umin - p) + (umin - r) * (umin - t));
  if (dt * std::fabs(std::min(dmin, 0.0)) >= 1.0)
    return fail(MLQ_EINVAL, "dt * |min I_ion'| = %g >= 1: the step equation may have several roots", dt * std::fabs(dmin));
  return MLQ_OK;
}

void sizes_of(const mlq_level_desc* d, int64_t* nn, int64_t* P) {
  if (d->mesh_kind == MLQ_MESH_P1_TET) {
    *nn = d->n_vert;
    *P = d->n_tet;
    return;
  }
  int64_t a = 1, b = 1;
  for (int k = 0; k < d->dim; ++k) {
    a *= d->n[k];
    b *= d->n[k] - 1;
  }
  *nn = a;
  *P = b;
}

}  // namespace

namespace mlq {

Work carve_workspace(void* base, const Geo& geo, int32_t B, int kmax, bool mixed, int res_groups) {
  Work w{};
  const int64_t nn = geo.nn, P = geo.P;
  w.kmax = kmax;
  w.nblk = (int32_t)cdiv(nn, kBlock);
  w.nred = (int32_t)cdiv(nn, kRedChunk);
  w.nres = (geo.dim == 3 && !geo.tet) ? res_groups * stencil3_blocks(geo) : w.nblk;
  w.nwav = (geo.dim == 3 && !geo.tet) ? stencil3_blocks(geo) : 0;
  const size_t ti = mixed ? sizeof(float) : sizeof(double);
  const size_t vn = (size_t)nn * B;
  char* p = (char*)base;
  size_t o = 0;
  auto take = [&](size_t bytes) -> void* {
    void* r = p ? (void*)(p + o) : nullptr;
    o = align256(o + bytes);
    return r;
  };
  w.uk = (double*)take(vn * sizeof(double));
  w.ukm1 = (double*)take(vn * sizeof(double));
  w.u = (double*)take(vn * sizeof(double));
  w.b = (double*)take(vn * sizeof(double));
  w.act = (double*)take(vn * sizeof(double));
  w.d = take(vn * ti);
  w.z = take(vn * ti * kmax);
  w.w = take(vn * ti);
  w.V = take(vn * ti * (kmax + 1));
  // box: per element (p, q); tetrahedra: per-sample stiffness values of the CSR
  w.coef = take(geo.tet ? (size_t)geo.nnz * B * ti : (size_t)P * B * 2 * ti);
  const size_t npart = std::max((size_t)std::max(w.nblk, w.nres) * 3, (size_t)w.nred * (kmax + 1));
  w.part = (double*)take(npart * B * sizeof(double));
  w.dpart = (double*)take((size_t)std::max(w.nred, w.nwav) * (kmax + 1) * B * sizeof(double));
  w.H = (double*)take((size_t)B * (kmax + 1) * kmax * sizeof(double));
  w.cs = (double*)take((size_t)B * kmax * sizeof(double));
  w.sn = (double*)take((size_t)B * kmax * sizeof(double));
  w.g = (double*)take((size_t)B * (kmax + 1) * sizeof(double));
  w.y = (double*)take((size_t)B * kmax * sizeof(double));
  w.hc = (double*)take((size_t)B * (kmax + 1) * sizeof(double));
  w.inv_eta = (double*)take((size_t)B * (kmax + 1) * sizeof(double));
  w.beta = (double*)take((size_t)B * sizeof(double));
  w.newton_active = (int32_t*)take((size_t)B * sizeof(int32_t));
  w.inner_active = (int32_t*)take((size_t)B * sizeof(int32_t));
  w.inner_k = (int32_t*)take((size_t)B * sizeof(int32_t));
  w.status = (int32_t*)take((size_t)B * sizeof(int32_t));
  w.iters = (int64_t*)take((size_t)B * 2 * sizeof(int64_t));
  w.counter = (int32_t*)take(16);
  w.bytes = o;
  return w;
}

}  // namespace mlq

// Workspace of mlq_solve_batch_static: a file-scope device array, one copy per GPU, held
// until the process ends.  Host code never passes `scratch` itself to a kernel or a copy
// (on the host the name only stands for the symbol); it uses the device address that
// hipGetSymbolAddress returns, looked up once per device and kept in g_scratch.
static __device__ __align__(256) unsigned char scratch[MLQ_STATIC_WS_BYTES];

namespace {
constexpr int kMaxDevices = 64;
void* g_scratch[kMaxDevices] = {};
std::mutex g_scratch_mu;
}  // namespace

extern "C" {

const char* mlq_last_error(void) { return g_err.c_str(); }

mlq_status mlq_level_bytes(const mlq_level_desc* desc, size_t* level_bytes) {
  if (level_bytes == nullptr) return fail(MLQ_EINVAL, "level_bytes is NULL");
  mlq_status st = validate(desc);
  if (st != MLQ_OK) return st;
  int64_t nn, P;
  sizes_of(desc, &nn, &P);
  if (desc->mesh_kind == MLQ_MESH_P1_TET) {
    mlq::TetHost th;
    const std::string err = mlq::tet_build(desc, th, false);
    if (!err.empty()) return fail(MLQ_EINVAL, "%s", err.c_str());
    *level_bytes = blob_layout(P, desc->n_modes, nn, 1, &th).total;
    return MLQ_OK;
  }
  *level_bytes = blob_layout(P, desc->n_modes, nn, std::max({desc->n[0], desc->n[1], desc->n[2]})).total;
  return MLQ_OK;
}

mlq_status mlq_create_level(const mlq_level_desc* desc, void* level_mem_dev, size_t level_bytes, void* hip_stream,
                            mlq_level** out) {
  if (out == nullptr) return fail(MLQ_EINVAL, "out is NULL");
  *out = nullptr;
  mlq_status st = validate(desc);
  if (st != MLQ_OK) return st;
  if (level_mem_dev == nullptr) return fail(MLQ_EINVAL, "level_mem_dev is NULL");
  if (((uintptr_t)level_mem_dev & 255) != 0) return fail(MLQ_EINVAL, "level_mem_dev must be 256-byte aligned");
  int64_t nn, P;
  sizes_of(desc, &nn, &P);
  const int64_t M = desc->n_modes;
  const bool tet = desc->mesh_kind == MLQ_MESH_P1_TET;
  mlq::TetHost th;
  if (tet) {
    const std::string err = mlq::tet_build(desc, th, true);
    if (!err.empty()) return fail(MLQ_EINVAL, "%s", err.c_str());
  }
  const int64_t nmax = tet ? 1 : std::max({desc->n[0], desc->n[1], desc->n[2]});
  const BlobLayout L = blob_layout(P, M, nn, nmax, tet ? &th : nullptr);
  if (level_bytes < L.total) return fail(MLQ_ESIZE, "level blob too small: %zu < %zu", level_bytes, L.total);
  hipStream_t s = (hipStream_t)hip_stream;

  mlq_level* lv = new (std::nothrow) mlq_level();
  if (lv == nullptr) return fail(MLQ_EINVAL, "out of host memory");
  lv->d = *desc;
  lv->d.phi = lv->d.sqrt_lambda = lv->d.theta0 = nullptr;
  lv->nn = nn;
  lv->P = P;
  lv->M = (int32_t)M;
  lv->mixed = desc->prec == MLQ_MIXED;
  lv->kmax = desc->max_inner;
  const int dim = desc->dim;
  lv->tet = tet;
  if (!tet)
    for (int a = 0; a < 3; ++a) lv->h[a] = a < dim ? (desc->hi[a] - desc->lo[a]) / (double)(desc->n[a] - 1) : 1.0;
  const double hx = lv->h[0], hy = lv->h[1], hz = lv->h[2];

  Geo& g = lv->geo;
  g.dim = dim;
  g.nx = (int32_t)desc->n[0];
  g.ny = (int32_t)desc->n[1];
  g.nz = dim == 3 ? (int32_t)desc->n[2] : 1;
  g.nn = nn;
  g.P = P;
  if (dim == 3) {
    g.Hm = hx * hy * hz;
    g.Hxx = hy * hz / hx;
    g.Hyy = hx * hz / hy;
    g.Hzz = hx * hy / hz;
    g.Hxy = hz;
  } else {
    g.Hm = hx * hy;
    g.Hxx = hy / hx;
    g.Hyy = hx / hy;
    g.Hzz = 0.0;
    g.Hxy = 1.0;
  }
  g.Hx = hx;
  g.Hy = hy;
  g.Hz = hz;
  g.iso = desc->diffusion == MLQ_DIFF_ISO ? 1 : 0;
  g.cfa = g.iso ? desc->sigma_t : 0.5 * (desc->sigma_l - desc->sigma_t);
  if (desc->diffusion == MLQ_DIFF_ISO) {
    g.cx0 = g.cy0 = g.cz0 = 0.0;
    g.cx1 = g.cy1 = g.cz1 = 1.0;
  } else {
    g.cx0 = g.cy0 = 0.5 * (desc->sigma_l + desc->sigma_t);
    g.cx1 = 1.0;
    g.cy1 = -1.0;
    g.cz0 = desc->sigma_t;
    g.cz1 = 0.0;
  }
  g.tet = tet ? 1 : 0;
  g.nnz = tet ? th.nell : 0;
  g.lx = 0;
  g.group = 0;
  if (tet) g.nx = g.ny = g.nz = 0;
  lv->io = Ionic{desc->alpha, desc->u_rest, desc->u_th, desc->u_peak, desc->t_end / desc->n_steps};

  // host-side level data: stimulus load vector (exact integral of the box
  // indicator against each tensor-product hat) and node weights w = M 1
  std::vector<double> f1[3], w1[3];
  double vol = 1.0;
  for (int a = 0; a < 3 && !tet; ++a) {
    const int64_t n = a < dim ? desc->n[a] : 1;
    f1[a].assign(n, 1.0);
    w1[a].assign(n, 1.0);
    if (a >= dim) continue;
    for (int64_t i = 0; i < n; ++i) {
      f1[a][i] = hat_integral(i, n, desc->lo[a], lv->h[a], desc->stim_lo[a], desc->stim_hi[a]);
      w1[a][i] = (i == 0 || i == n - 1) ? 0.5 * lv->h[a] : lv->h[a];
    }
    vol *= desc->hi[a] - desc->lo[a];
  }
  lv->vol = tet ? th.vol : vol;
  std::vector<double> fbox, wts;
  if (tet) {
    fbox.swap(th.fload);
    wts.swap(th.wts);
  } else {
    fbox.resize(nn);
    wts.resize(nn);
  }
  for (int64_t k = 0; k < (tet ? 0 : (dim == 3 ? desc->n[2] : 1)); ++k)
    for (int64_t j = 0; j < desc->n[1]; ++j)
      for (int64_t i = 0; i < desc->n[0]; ++i) {
        const int64_t id = i + desc->n[0] * (j + desc->n[1] * k);
        fbox[id] = f1[0][i] * f1[1][j] * f1[2][k];
        wts[id] = w1[0][i] * w1[1][j] * w1[2][k];
      }

  char* base = (char*)level_mem_dev;
  lv->phi64 = (double*)(base + L.phi64);
  lv->phi32 = (float*)(base + L.phi32);
  lv->sqrt_lambda = (double*)(base + L.sl);
  lv->theta0 = (double*)(base + L.th0);
  lv->fbox = (double*)(base + L.fbox);
  lv->wts = (double*)(base + L.wts);
  lv->tri = (void*)(base + L.tri);
  lv->nmax = (int)nmax;
  // preconditioner tables: pivots of tridiag(1, 4, 1) with 2 at both ends, per axis
  std::vector<double> tri64(3 * nmax, 0.0);
  std::vector<float> tri32(3 * nmax, 0.0f);
  for (int a = 0; a < 3 && !tet; ++a) {
    const int64_t n = a < dim ? desc->n[a] : 1;
    double prev = 0.0;
    for (int64_t i = 0; i < n; ++i) {
      const double diag = (i == 0 || i == n - 1) ? 2.0 : 4.0;
      const double piv = diag - (i > 0 ? prev : 0.0);
      prev = 1.0 / piv;
      tri64[a * nmax + i] = prev;
      tri32[a * nmax + i] = (float)prev;
    }
  }
  // LDS staging of the preconditioner's line solves
  if (!tet) {
    const size_t ti = lv->mixed ? sizeof(float) : sizeof(double);
    // one x-y plane per workgroup (2D: the whole sample)
    const size_t plane = ti * (size_t)desc->n[0] * (size_t)desc->n[1];
    int dev = 0;
    hipDeviceProp_t prop{};
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) {
      delete lv;
      return fail(MLQ_EHIP, "cannot query the device");
    }
    const size_t lim = std::max(prop.sharedMemPerBlock, prop.sharedMemPerBlockOptin);
    if (plane > lim) {
      delete lv;
      return fail(MLQ_EINVAL, "a grid plane (%zu bytes) exceeds the LDS of one workgroup (%zu bytes)", plane, lim);
    }
    if (prepare_minv_kernels(plane) != hipSuccess) {
      delete lv;
      return fail(MLQ_EHIP, "cannot raise the LDS limit of the preconditioner kernels to %zu bytes", plane);
    }
  }

  auto cleanup = [&](mlq_status e) {
    if (lv->host_flags) (void)hipHostFree(lv->host_flags);
    delete lv;
    return e;
  };
  hipError_t e = hipSuccess;
  std::vector<float> phi32;
  std::vector<double> phiT;
  std::vector<double> th0;
  if (desc->arrays_on_device) {
    const hipMemcpyKind k = hipMemcpyDeviceToDevice;
    if (M > 0) {
      // the blob keeps the basis mode-major (M x P): contiguous per mode for the MFMA synthesis
      launch_transpose_f64(desc->phi, lv->phi64, P, M, s);
      e = hipGetLastError();
      if (e == hipSuccess) launch_cast_f32(lv->phi64, lv->phi32, P * M, s);
      if (e == hipSuccess) e = hipMemcpyAsync(lv->sqrt_lambda, desc->sqrt_lambda, sizeof(double) * M, k, s);
    }
    if (e == hipSuccess) {
      if (desc->theta0 != nullptr)
        e = hipMemcpyAsync(lv->theta0, desc->theta0, sizeof(double) * P, k, s);
      else
        e = hipMemsetAsync(lv->theta0, 0, sizeof(double) * P, s);
    }
  } else {
    // mode-major copies (M x P) of the P x M row-major input
    phiT.resize((size_t)P * M);
    phi32.resize((size_t)P * M);
    for (int64_t p = 0; p < P; ++p)
      for (int32_t k = 0; k < M; ++k) {
        phiT[(size_t)k * P + p] = desc->phi[(size_t)p * M + k];
        phi32[(size_t)k * P + p] = (float)desc->phi[(size_t)p * M + k];
      }
    th0.assign(P, 0.0);
    if (desc->theta0 != nullptr) std::memcpy(th0.data(), desc->theta0, sizeof(double) * P);
    if (M > 0) {
      e = hipMemcpyAsync(lv->phi64, phiT.data(), sizeof(double) * P * M, hipMemcpyHostToDevice, s);
      if (e == hipSuccess) e = hipMemcpyAsync(lv->phi32, phi32.data(), sizeof(float) * P * M, hipMemcpyHostToDevice, s);
      if (e == hipSuccess) e = hipMemcpyAsync(lv->sqrt_lambda, desc->sqrt_lambda, sizeof(double) * M, hipMemcpyHostToDevice, s);
    }
    if (e == hipSuccess) e = hipMemcpyAsync(lv->theta0, th0.data(), sizeof(double) * P, hipMemcpyHostToDevice, s);
  }
  if (e == hipSuccess) {
    if (lv->mixed)
      e = hipMemcpyAsync(lv->tri, tri32.data(), sizeof(float) * 3 * nmax, hipMemcpyHostToDevice, s);
    else
      e = hipMemcpyAsync(lv->tri, tri64.data(), sizeof(double) * 3 * nmax, hipMemcpyHostToDevice, s);
  }
  if (e == hipSuccess && tet) {
    TetDev& t = lv->td;
    t.nv = th.nv;
    t.nt = th.nt;
    t.nell = th.nell;
    t.width = th.width;
    t.nc = th.nc;
    t.ecol = (const int32_t*)(base + L.ecol);
    t.ediag = (const int32_t*)(base + L.ediag);
    t.em = (const double*)(base + L.em);
    t.em32 = (const float*)(base + L.em32);
    t.mdiag = (const double*)(base + L.mdiag);
    t.mdiag32 = (const float*)(base + L.mdiag32);
    t.ecptr = (const int32_t*)(base + L.ecptr);
    t.ecdat = (const int32_t*)(base + L.ecdat);
    t.geo = (const double*)(base + L.geo);
    t.model = desc->diffusion;
    t.vmean = (const double*)(base + L.vmean);
    std::vector<float> m32(th.em.begin(), th.em.end()), d32(th.mdiag.begin(), th.mdiag.end());
    auto up = [&](const void* dst, const void* src, size_t bytes) {
      if (e == hipSuccess) e = hipMemcpyAsync((void*)dst, src, bytes, hipMemcpyHostToDevice, s);
    };
    up(t.ecol, th.ecol.data(), sizeof(int32_t) * th.ecol.size());
    up(t.ediag, th.ediag.data(), sizeof(int32_t) * th.ediag.size());
    up(t.em, th.em.data(), sizeof(double) * th.em.size());
    up(t.em32, m32.data(), sizeof(float) * m32.size());
    up(t.mdiag, th.mdiag.data(), sizeof(double) * th.mdiag.size());
    up(t.mdiag32, d32.data(), sizeof(float) * d32.size());
    up(t.ecptr, th.ecptr.data(), sizeof(int32_t) * th.ecptr.size());
    up(t.ecdat, th.ecdat.data(), sizeof(int32_t) * th.ecdat.size());
    up(t.geo, th.geo.data(), sizeof(double) * th.geo.size());
    if (t.model == MLQ_DIFF_VECTOR) up(t.vmean, desc->v_mean, sizeof(double) * 3 * th.nt);
    // the host vectors must outlive the asynchronous copies
    if (e == hipSuccess) e = hipStreamSynchronize(s);
  }
  if (e == hipSuccess) e = hipMemcpyAsync(lv->fbox, fbox.data(), sizeof(double) * nn, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipMemcpyAsync(lv->wts, wts.data(), sizeof(double) * nn, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e == hipSuccess)
    e = hipHostMalloc((void**)&lv->host_flags, sizeof(int32_t) * (kFlagInner + kMaxInner + 1), hipHostMallocDefault);
  for (int q = 0; q < 2 && e == hipSuccess; ++q) e = hipEventCreateWithFlags(&lv->flag_ev[q], hipEventDisableTiming);
  if (e == hipSuccess) e = hipGetDevice(&lv->device);
  if (e != hipSuccess) return cleanup(fail(MLQ_EHIP, "level upload failed: %s", hipGetErrorString(e)));
  *out = lv;
  return MLQ_OK;
}

void mlq_destroy_level(mlq_level* level) {
  if (level == nullptr) return;
  for (auto& p : level->pending) {
    (void)hipEventDestroy(p.a);
    (void)hipEventDestroy(p.b);
  }
  for (hipEvent_t e : level->free_events) (void)hipEventDestroy(e);
  for (hipEvent_t e : level->flag_ev)
    if (e) (void)hipEventDestroy(e);
  if (level->host_flags) (void)hipHostFree(level->host_flags);
  drop_graphs(level);
  if (level->cap_stream) (void)hipStreamDestroy(level->cap_stream);
  delete level;
}

mlq_status mlq_timing_enable(mlq_level* level, uint32_t kernel_mask) {
  if (level == nullptr) return fail(MLQ_EINVAL, "level is NULL");
  level->tmask = kernel_mask;
  return MLQ_OK;
}

mlq_status mlq_timing_read(mlq_level* level, mlq_timing* out, int32_t reset) {
  if (level == nullptr || out == nullptr) return fail(MLQ_EINVAL, "NULL argument");
  *out = level->tim;
  if (reset) level->tim = mlq_timing{};
  return MLQ_OK;
}

mlq_status mlq_level_sizes(const mlq_level* level, int64_t* n_nodes, int64_t* n_elems) {
  if (level == nullptr || n_nodes == nullptr || n_elems == nullptr) return fail(MLQ_EINVAL, "NULL argument");
  *n_nodes = level->nn;
  *n_elems = level->P;
  return MLQ_OK;
}

mlq_status mlq_workspace_bytes(const mlq_level* level, int32_t batch, size_t* ws_bytes) {
  if (level == nullptr || ws_bytes == nullptr) return fail(MLQ_EINVAL, "NULL argument");
  if (batch < 1 || batch > level->d.max_batch) return fail(MLQ_EINVAL, "batch %d outside [1, max_batch]", batch);
  *ws_bytes = carve_workspace(nullptr, level->geo, batch, level->kmax, level->mixed).bytes;
  return MLQ_OK;
}

mlq_status mlq_sample_fields(mlq_level* level, const double* Y_dev, int32_t batch, void* theta_dev, void* hip_stream) {
  if (level == nullptr || Y_dev == nullptr || theta_dev == nullptr) return fail(MLQ_EINVAL, "NULL argument");
  if (batch < 1 || batch > level->d.max_batch) return fail(MLQ_EINVAL, "batch %d outside [1, max_batch]", batch);
  if (level->M < 1) return fail(MLQ_ESTATE, "level has no KL modes");
  launch_kl(level->phi64, level->phi32, level->sqrt_lambda, level->theta0, Y_dev, level->P, level->M, batch, theta_dev,
            level->mixed, (hipStream_t)hip_stream);
  HIP_OK(hipGetLastError());
  return MLQ_OK;
}

mlq_status mlq_apply(mlq_level* level, const void* theta_dev, int32_t batch, const void* x_dev, const void* d_dev,
                     void* y_dev, void* ws_dev, size_t ws_bytes, void* hip_stream) {
  if (level == nullptr || theta_dev == nullptr || x_dev == nullptr || d_dev == nullptr || y_dev == nullptr ||
      ws_dev == nullptr)
    return fail(MLQ_EINVAL, "NULL argument");
  if (batch < 1 || batch > level->d.max_batch) return fail(MLQ_EINVAL, "batch %d outside [1, max_batch]", batch);
  Work w = carve_workspace(ws_dev, level->geo, batch, level->kmax, level->mixed);
  if (ws_bytes < w.bytes) return fail(MLQ_ESIZE, "workspace too small: %zu < %zu", ws_bytes, w.bytes);
  hipStream_t s = (hipStream_t)hip_stream;
  if (level->tet) {
    launch_tet_assemble(level->td, theta_dev, w.coef, batch, level->d.sigma_t, level->d.sigma_l - level->d.sigma_t,
                        level->mixed, s);
    launch_tet_apply(level->td, w.coef, x_dev, d_dev, y_dev, 0.5 * level->io.dt, batch, nullptr, level->mixed, s);
    HIP_OK(hipGetLastError());
    return MLQ_OK;
  }
  const bool iso = level->d.diffusion == MLQ_DIFF_ISO;
  if (level->geo.dim == 3 && level->mixed) {  // the kernel forms the coefficients from theta
    launch_apply_full3(level->geo, theta_dev, x_dev, d_dev, y_dev, 0.5 * level->io.dt, batch, true, s);
    HIP_OK(hipGetLastError());
    return MLQ_OK;
  }
  launch_coefs(theta_dev, w.coef, level->P, batch, iso ? level->d.sigma_t : 0.5 * (level->d.sigma_l - level->d.sigma_t),
               iso, level->mixed, s);
  if (level->geo.dim == 3)
    launch_apply_full3(level->geo, w.coef, x_dev, d_dev, y_dev, 0.5 * level->io.dt, batch, level->mixed, s);
  else
    launch_apply_public(level->geo, w.coef, x_dev, d_dev, y_dev, 0.5 * level->io.dt, batch, level->mixed, s);
  HIP_OK(hipGetLastError());
  return MLQ_OK;
}

static mlq_status read_counter(mlq_level* lv, const Work& w, hipStream_t s, int32_t* value) {
  HIP_OK(hipMemcpyAsync(lv->host_flags, w.counter, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  HIP_OK(hipStreamSynchronize(s));
  *value = lv->host_flags[0];
  harvest(lv);
  return MLQ_OK;
}

// Probe table of a field request: validated against the level's node count.
static mlq_status probe_table(const mlq_level* level, const mlq_field_out* f, ProbeTab* tab) {
  tab->n = 0;
  if (f == nullptr || (f->probe == nullptr && f->probe_sum == nullptr)) return MLQ_OK;
  if (f->n_probe < 1 || f->n_probe > kMaxProbes) return fail(MLQ_EINVAL, "n_probe outside [1, %d]", kMaxProbes);
  if (f->probe_node == nullptr || f->probe_w == nullptr) return fail(MLQ_EINVAL, "probe nodes or weights are NULL");
  for (int i = 0; i < f->n_probe * kProbeNodes; ++i) {
    if (f->probe_node[i] < 0 || f->probe_node[i] >= level->nn) return fail(MLQ_EINVAL, "probe node out of range");
    if (!std::isfinite(f->probe_w[i])) return fail(MLQ_EINVAL, "probe weight not finite");
    tab->node[i] = f->probe_node[i];
    tab->w[i] = f->probe_w[i];
  }
  tab->n = f->n_probe;
  return MLQ_OK;
}

static mlq_status solve_impl(mlq_level* level, const void* theta_dev, int32_t batch, int32_t n_steps, void* ws_dev,
                             size_t ws_bytes, double* qoi_dev, int32_t* status_dev, int64_t* iters_dev,
                             double* u_out_dev, double* act_out_dev, const mlq_field_out* fields, void* hip_stream) {
  if (level == nullptr || theta_dev == nullptr || ws_dev == nullptr || qoi_dev == nullptr || status_dev == nullptr ||
      iters_dev == nullptr)
    return fail(MLQ_EINVAL, "NULL argument");
  ProbeTab tab;
  {
    const mlq_status pst = probe_table(level, fields, &tab);
    if (pst != MLQ_OK) return pst;
  }
  double* const u_sum = fields != nullptr ? fields->u_sum : nullptr;
  double* const act_sum = fields != nullptr ? fields->act_sum : nullptr;
  double* const probe = tab.n > 0 ? fields->probe : nullptr;
  double* const probe_sum = tab.n > 0 ? fields->probe_sum : nullptr;
  if (batch < 1 || batch > level->d.max_batch) return fail(MLQ_EINVAL, "batch %d outside [1, max_batch]", batch);
  if (n_steps < 0 || n_steps > level->d.n_steps) return fail(MLQ_EINVAL, "n_steps %d outside [0, %d]", n_steps, level->d.n_steps);
  if (((uintptr_t)ws_dev & 255) != 0) return fail(MLQ_EINVAL, "workspace must be 256-byte aligned");
  Work w = carve_workspace(ws_dev, level->geo, batch, level->kmax, level->mixed);
  if (ws_bytes < w.bytes) return fail(MLQ_ESIZE, "workspace too small: %zu < %zu", ws_bytes, w.bytes);
  hipStream_t s = (hipStream_t)hip_stream;
  const mlq_level_desc& d = level->d;
  const Geo& g = level->geo;
  const bool mixed = level->mixed;
  const double dt = level->io.dt;
  const int kmax = level->kmax;

  const bool tet = level->tet;
  const TetDev& td = level->td;
  w.theta = theta_dev;
  if (tet)
    launch_tet_assemble(td, theta_dev, w.coef, batch, d.sigma_t, d.sigma_l - d.sigma_t, mixed, s);
  else  // (mixed 3D boxes: for the residual and right-hand side; the Krylov apply reads theta)
    launch_coefs(theta_dev, w.coef, level->P, batch,
                 d.diffusion == MLQ_DIFF_ISO ? d.sigma_t : 0.5 * (d.sigma_l - d.sigma_t), d.diffusion == MLQ_DIFF_ISO,
                 mixed, s);
  const bool ref_guess0 = (d.newton_guess == MLQ_GUESS_REFERENCE || d.newton_guess == MLQ_GUESS_REFERENCE_LOCAL) &&
                          level->ref != nullptr;
  if (level->persistent && small_solver_fits(g, mixed) && u_sum == nullptr && act_sum == nullptr && tab.n == 0 &&
      !ref_guess0) {
    // one launch: every sample's time loop in a workgroup of its own; enqueue only
    SmallArgs sa{};
    sa.g = g;
    sa.io = level->io;
    sa.B = batch;
    sa.n_steps = n_steps;
    sa.kmax = kmax;
    sa.max_newton = d.max_newton;
    sa.extrap = d.newton_guess == MLQ_GUESS_EXTRAPOLATE ? 1 : 0;
    sa.qoi = d.qoi;
    sa.newton_tol = d.newton_tol;
    sa.inner_tol = d.inner_tol;
    sa.t_on = d.stim_t_on;
    sa.t_off = d.stim_t_off;
    sa.amp = d.stim_amp;
    sa.fbox = level->fbox;
    sa.wts = level->wts;
    sa.vol = level->vol;
    sa.tri = level->tri;
    sa.nmax = level->nmax;
    sa.w = w;
    sa.qoi_out = qoi_dev;
    sa.status_out = status_dev;
    sa.iters_out = iters_dev;
    sa.u_out = u_out_dev;
    sa.act_out = act_out_dev;
    hipError_t e = hipSuccess;
    timed(level, MLQ_K_PERSISTENT, (double)level->nn * batch * n_steps, s, [&] { e = launch_solve_small(sa, mixed, s); });
    if (e != hipSuccess) return fail(MLQ_EHIP, "persistent solve launch failed: %s", hipGetErrorString(e));
    return MLQ_OK;
  }
  launch_init(w, level->nn, batch, d.u_th, s);
  HIP_OK(hipGetLastError());
  // field outputs of time level k (the state u_k sits in w.uk)
  auto stream_fields = [&](int32_t k) {
    if (u_sum != nullptr) launch_field_sum(w.uk, batch, level->nn, u_sum + (size_t)k * level->nn, s);
    if (probe != nullptr) launch_probe(w.uk, batch, level->nn, tab, k, n_steps + 1, probe, s);
    if (probe_sum != nullptr) launch_probe_sum(w.uk, batch, level->nn, tab, k, n_steps + 1, probe_sum, s);
  };
  stream_fields(0);

  auto rate = [&](double t) { return (d.stim_t_on <= t && t < d.stim_t_off) ? d.stim_amp : 0.0; };
  const double nn = (double)level->nn;
  for (int32_t k = 0; k < n_steps; ++k) {
    const double t0 = (double)k * dt, t1 = (double)(k + 1) * dt;
    const double load = 0.5 * dt * (rate(t1) + rate(t0));
    // 3D boxes need no right-hand side: the first residual of the step forms the Newton start and
    // the previous step's activation times (launch_residual3f)
    const bool box3 = g.dim == 3 && !tet;
    if (!box3)
      timed(level, MLQ_K_RHS, nn * batch, s, [&] {
        if (tet)  // also the extrapolated start and the previous step's activation
          launch_tet_rhs(td, w, level->fbox, load, dt, batch, mixed, s, k > 0 ? w.ukm1 : nullptr,
                         d.newton_guess == MLQ_GUESS_EXTRAPOLATE, d.u_th, (double)(k - 1) * dt);
        else
          launch_rhs(g, w, level->fbox, load, dt, batch, mixed, s);
      });
    // the rhs kernels start Newton from u = u_k; the extrapolated guess replaces it
    const bool fused3 = g.dim == 3 || tet;  // the 3D and tetrahedral rhs kernels did the two steps below
    if (d.newton_guess == MLQ_GUESS_EXTRAPOLATE && k > 0 && !fused3) launch_extrapolate(w, level->nn, batch, s);
    const bool ref_guess = (d.newton_guess == MLQ_GUESS_REFERENCE || d.newton_guess == MLQ_GUESS_REFERENCE_LOCAL) &&
                           level->ref != nullptr;
    if (ref_guess)
      launch_guess_reference(w, level->ref + (size_t)k * level->nn, level->ref + (size_t)(k + 1) * level->nn,
                             level->nn, batch, d.newton_guess == MLQ_GUESS_REFERENCE_LOCAL, s);
    launch_newton_reset(w, batch, s);
    int32_t active = batch;
    for (int it = 0;; ++it) {
      timed(level, MLQ_K_RESIDUAL, nn * active, s, [&] {
        if (tet) {
          launch_tet_residual(td, level->io, w, batch, mixed, s);
        } else if (box3) {
          // first iteration of the step: the iterate starts at u_k, its extrapolation, or the
          // reference guess already written to w.u
          const int start = it > 0 || ref_guess ? 0 : (d.newton_guess == MLQ_GUESS_EXTRAPOLATE && k > 0 ? 2 : 1);
          launch_residual3f(g, level->io, w, batch, mixed, s, start, it == 0 && k > 0 ? w.ukm1 : nullptr,
                            level->fbox, load, d.u_th, (double)(k - 1) * dt);
        } else {
          launch_residual(g, level->io, w, batch, mixed, s);
        }
      });
      timed(level, MLQ_K_SMALL, 0.0, s, [&] {
        launch_newton_check(g, w, batch, d.newton_tol, s);
        // the Newton count; also clears the counter that GMRES iteration 0 accumulates into
        launch_count(w.newton_active, batch, w.counter, w.counter + 1, s);
      });
      mlq_status st = read_counter(level, w, s, &active);
      if (st != MLQ_OK) return st;
      if (active == 0) break;
      if (it >= d.max_newton) {
        launch_mark_failed(w, batch, s);
        break;
      }
      // active samples entering iteration j: the Newton count for j = 0, else the host
      // slot of iteration j - 1 (filled by then whenever the launch figures are harvested)
      int32_t* const cnt = level->host_flags + kFlagInner;
      level->host_flags[1] = active;  // slot 0 is refilled by the next Newton check before harvest
      auto entering = [&](int j) -> const int32_t* { return j == 0 ? &level->host_flags[1] : &cnt[j - 1]; };
      // The launches of GMRES iteration j (preconditioner, apply with the fused projections,
      // projections, orthogonalisation, Givens rotation + active count); untimed while captured.
      auto gmres_iteration = [&](int j, bool capturing, hipStream_t s) {
        const int32_t* nin = entering(j);
        auto tm = [&](int cls, double units, auto&& launch, double bytes = 0.0, const int32_t* count = nullptr,
                      double kbytes = 0.0, double kfixed = 0.0) {
          if (capturing)
            launch();
          else
            timed(level, cls, units, s, launch, bytes, count, kbytes, kfixed);
        };
        tm(MLQ_K_PRECOND, nn, [&] {
          if (tet)
            launch_tet_jacobi_basis(td, w, j, 0.5 * dt, batch, mixed, s);
          else
            launch_minv_basis(g, w, level->tri, level->nmax, j, batch, mixed, s);
        }, 0.0, nin);
        // 3D boxes, j < 8: the apply kernel also forms the projections w . v_i (i <= j)
        const bool fuse = g.dim == 3 && !tet && j < 8;
        const double ti = mixed ? 4.0 : 8.0;
        // Algorithmic bytes per active sample, each operand once: boxes z, v_j and the
        // element's field value theta read, w written (one element per node), v_0..v_{j-1}
        // read for the fused projections; tetrahedra z, d read, w written per vertex and theta
        // once per tetrahedron.  The kernel's own bytes: FP64 and 2D boxes read the element
        // coefficient pair (p, q) instead of theta; tetrahedra read the assembled stiffness values of
        // every slot of a row instead of theta, and the shared pattern (columns, mass) once
        // per launch.
        const double slots = tet ? (double)td.nell / (double)td.nv : 0.0;
        const double apply_bytes =
            tet ? ti * (3.0 * nn + (td.model == MLQ_DIFF_VECTOR ? 3.0 : 1.0) * (double)level->P)
                : nn * ti * (4.0 + (fuse ? j : 0));
        const double box_vals = (mixed && g.dim == 3 ? 4.0 : 5.0) + (fuse ? j : 0);  // mixed 3D: theta
        const double apply_kbytes = nn * ti * (tet ? slots + 3.0 : box_vals);
        const double apply_fixed = tet ? (double)td.nell * (4.0 + ti) : 0.0;
        tm(
            MLQ_K_APPLY, nn,
            [&] {
              if (tet)  // the full Jacobian applied to z_j
                launch_tet_apply(td, w.coef, (const char*)w.z + (size_t)j * level->nn * batch * (size_t)ti, w.d,
                                 w.w, 0.5 * dt, batch, w.inner_active, mixed, s);
              else if (g.dim == 3)
                launch_apply_pk3(g, w, j, 0.5 * dt, batch, mixed, s, fuse ? (j == 0 ? 1 : j < 4 ? 4 : 8) : 0);
              else
                launch_apply_pk(g, w, j, 0.5 * dt, batch, mixed, s);
            },
            apply_bytes, nin, apply_kbytes, apply_fixed);
        if (!fuse) tm(MLQ_K_DOTS, nn, [&] { launch_dots(g, w, j, batch, mixed, s); }, 0.0, nin);
        tm(MLQ_K_ORTH, nn, [&] { launch_orth(g, w, j, batch, mixed, s, fuse ? w.nwav : w.nred); }, 0.0, nin);
        tm(MLQ_K_SMALL, 0.0, [&] {
          launch_givens(g, w, j, batch, d.inner_tol, s, w.nred);  // counts into counter[1 + (j & 1)]
        });
      };
      const int J = level->gmres_block;
      if (J <= 0) {
        for (int j = 0; j < kmax; ++j) {
          gmres_iteration(j, false, s);
          // The count of iteration j is read while iteration j + 1 is already queued, so
          // the GPU does not idle during the host round trip; an iteration queued after
          // every sample has stopped finds no active sample and does nothing.
          HIP_OK(hipMemcpyAsync(&cnt[j], w.counter + 1 + (j & 1), sizeof(int32_t), hipMemcpyDeviceToHost, s));
          HIP_OK(hipEventRecord(level->flag_ev[j & 1], s));
          if (j > 0) {
            HIP_OK(hipEventSynchronize(level->flag_ev[(j - 1) & 1]));
            if (cnt[j - 1] == 0) break;
          }
        }
      } else {
        // Blocks of J iterations, each replayed from a graph captured once per (workspace,
        // field, batch, block); one count read per block, one block behind the launches.
        int prev = -1;
        for (int j0 = 0, nb = 0; j0 < kmax; j0 += J, ++nb) {
          const int jn = std::min(J, kmax - j0);
          hipGraphExec_t ge = nullptr;
          const mlq_status gs = block_graph(level, ws_dev, theta_dev, batch, j0, jn, s, &ge, [&](hipStream_t cs) {
            for (int j = j0; j < j0 + jn; ++j) gmres_iteration(j, true, cs);
          });
          if (gs != MLQ_OK) return gs;
          HIP_OK(hipGraphLaunch(ge, s));
          const int jl = j0 + jn - 1;
          HIP_OK(hipMemcpyAsync(&cnt[jl], w.counter + 1 + (jl & 1), sizeof(int32_t), hipMemcpyDeviceToHost, s));
          HIP_OK(hipEventRecord(level->flag_ev[nb & 1], s));
          if (prev >= 0) {
            HIP_OK(hipEventSynchronize(level->flag_ev[(nb - 1) & 1]));
            if (cnt[prev] == 0) break;
          }
          prev = jl;
        }
      }
      timed(level, MLQ_K_UPDATE, nn * active, s, [&] {
        launch_solve_y(w, batch, false, s);
        launch_update_zbasis(g, w, batch, mixed, s);
      });
    }
    if (!fused3)
      timed(level, MLQ_K_QOI, nn * batch, s, [&] { launch_activation(w, level->nn, batch, d.u_th, t0, dt, s); });
    // u_{k-1} <- u_k <- u (the old u_{k-1} becomes the next Newton iterate's storage)
    double* old = w.ukm1;
    w.ukm1 = w.uk;
    w.uk = w.u;
    w.u = old;
    stream_fields(k + 1);
  }
  // 3D boxes and tetrahedra: the last step's activation (the rhs kernel of each step recorded
  // the one before)
  if ((g.dim == 3 || tet) && n_steps > 0)
    timed(level, MLQ_K_QOI, nn * batch, s, [&] {
      launch_activation_between(w.ukm1, w.uk, w.act, level->nn, batch, d.u_th, (double)(n_steps - 1) * dt, dt, s);
    });
  if (act_sum != nullptr) launch_act_sum(w.act, batch, level->nn, (double)n_steps * dt, act_sum, s);
  launch_qoi(w, level->wts, level->nn, batch, d.qoi, (double)n_steps * dt, level->vol, qoi_dev, s);
  HIP_OK(hipMemcpyAsync(status_dev, w.status, sizeof(int32_t) * batch, hipMemcpyDeviceToDevice, s));
  HIP_OK(hipMemcpyAsync(iters_dev, w.iters, sizeof(int64_t) * 2 * batch, hipMemcpyDeviceToDevice, s));
  if (u_out_dev)
    HIP_OK(hipMemcpyAsync(u_out_dev, w.uk, sizeof(double) * level->nn * batch, hipMemcpyDeviceToDevice, s));
  if (act_out_dev)
    HIP_OK(hipMemcpyAsync(act_out_dev, w.act, sizeof(double) * level->nn * batch, hipMemcpyDeviceToDevice, s));
  // samples that failed: counted on the device, one integer read back
  launch_count(w.status, batch, w.counter + 3, nullptr, s);
  HIP_OK(hipGetLastError());
  HIP_OK(hipMemcpyAsync(level->host_flags + 2, w.counter + 3, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  HIP_OK(hipStreamSynchronize(s));
  harvest(level);
  const int32_t bad = level->host_flags[2];
  if (bad) return fail(MLQ_ENOCONV, "%d of %d samples did not converge", bad, batch);
  return MLQ_OK;
}

// Geometry of the all-at-once block solve: the stencil view (every time level of a block a
// virtual sample) and the vector view (a sample's block of m' + 1 time levels one vector).
static mlq_status block_geos(const mlq_level* level, int32_t batch, int32_t mb, Geo* gs, Geo* gv) {
  if (level->tet || level->geo.dim != 3) return fail(MLQ_EINVAL, "time blocks are solved on 3D box levels");
  if (mb < 1 || level->d.n_steps % mb != 0)
    return fail(MLQ_EINVAL, "steps per block %d must divide the %d steps", mb, level->d.n_steps);
  if (batch < 1 || batch > level->d.max_batch) return fail(MLQ_EINVAL, "batch %d outside [1, max_batch]", batch);
  if ((int64_t)batch * (mb + 1) > 65535) return fail(MLQ_EINVAL, "batch x (steps per block + 1) exceeds 65535");
  if ((int64_t)(mb + 1) * level->nn > (int64_t(1) << 29)) return fail(MLQ_EINVAL, "time block too large");
  *gs = level->geo;
  gs->group = mb + 1;
  *gv = level->geo;
  gv->nn = (int64_t)(mb + 1) * level->nn;
  gv->group = 0;
  return MLQ_OK;
}

// All-at-once solve of the space-time system in time blocks of mb steps (Section 3.3, multiple
// time blocks; eq. (system_C) with the reaction term of eq. (mono_disc)): per block, Newton's method
// on all its time levels at once, each linear system by GMRES on the block with the block-Jacobi
// preconditioner (per time level M (I + D_q), the preconditioner of the time-stepping solve).
static mlq_status solve_blocks_impl(mlq_level* level, const void* theta_dev, int32_t batch, int32_t mb, int32_t guess,
                                    void* ws_dev, size_t ws_bytes, double* qoi_dev, int32_t* status_dev,
                                    int64_t* iters_dev, double* u_out_dev, void* hip_stream) {
  if (level == nullptr || theta_dev == nullptr || ws_dev == nullptr || qoi_dev == nullptr || status_dev == nullptr ||
      iters_dev == nullptr)
    return fail(MLQ_EINVAL, "NULL argument");
  if (guess != MLQ_GUESS_PREVIOUS && guess != MLQ_GUESS_REFERENCE && guess != MLQ_GUESS_REFERENCE_LOCAL)
    return fail(MLQ_EINVAL, "block guess %d: previous block, reference or local reference", guess);
  if (guess != MLQ_GUESS_PREVIOUS && level->ref == nullptr)
    return fail(MLQ_ESTATE, "the reference guesses need mlq_set_reference");
  if (((uintptr_t)ws_dev & 255) != 0) return fail(MLQ_EINVAL, "workspace must be 256-byte aligned");
  Geo gs, gv;
  {
    const mlq_status st = block_geos(level, batch, mb, &gs, &gv);
    if (st != MLQ_OK) return st;
  }
  const int kmax = level->kmax;
  const bool mixed = level->mixed;
  const int G = mb + 1;
  // residual partials of a sample: the workgroups of its G time levels
  Work w = carve_workspace(ws_dev, gv, batch, kmax, mixed, G);
  if (ws_bytes < w.bytes) return fail(MLQ_ESIZE, "workspace too small: %zu < %zu", ws_bytes, w.bytes);
  const int32_t Bv = batch * G;
  w.theta = theta_dev;
  hipStream_t s = (hipStream_t)hip_stream;
  const mlq_level_desc& d = level->d;
  const double dt = level->io.dt;
  const int64_t n = level->nn;
  const size_t ti = mixed ? sizeof(float) : sizeof(double);
  const size_t vn = (size_t)gv.nn * batch;
  launch_coefs(theta_dev, w.coef, level->P, batch,
               d.diffusion == MLQ_DIFF_ISO ? d.sigma_t : 0.5 * (d.sigma_l - d.sigma_t), d.diffusion == MLQ_DIFF_ISO,
               mixed, s);
  // the unused slot 0 of every Krylov vector stays zero, so the block vectors' dot products,
  // norms and updates see only the unknown time levels
  HIP_OK(hipMemsetAsync(w.u, 0, sizeof(double) * vn, s));
  HIP_OK(hipMemsetAsync(w.V, 0, ti * vn * (kmax + 1), s));
  HIP_OK(hipMemsetAsync(w.z, 0, ti * vn * kmax, s));
  HIP_OK(hipMemsetAsync(w.w, 0, ti * vn, s));
  HIP_OK(hipMemsetAsync(w.d, 0, ti * vn, s));
  launch_init(w, n, batch, d.u_th, s);  // activation flags of the [B][n] map, status, counters
  HIP_OK(hipGetLastError());
  const int gmode = guess == MLQ_GUESS_PREVIOUS ? 0 : guess == MLQ_GUESS_REFERENCE ? 1 : 2;
  int32_t* const cnt = level->host_flags + kFlagInner;
  for (int k0 = 0; k0 < d.n_steps; k0 += mb) {
    launch_block_guess(w.u, G, n, batch, level->ref, k0, gmode, s);
    launch_newton_reset(w, batch, s);
    for (int it = 0;; ++it) {
      launch_rhs3_block(gs, w.u, w.b, w.coef, level->fbox, k0, dt, d.stim_t_on, d.stim_t_off, d.stim_amp, Bv, mixed,
                        s);
      launch_residual3(gs, level->io, w, Bv, mixed, s);
      launch_newton_check(gv, w, batch, d.newton_tol, s);
      launch_count(w.newton_active, batch, w.counter, w.counter + 1, s);
      int32_t active = 0;
      const mlq_status st = read_counter(level, w, s, &active);
      if (st != MLQ_OK) return st;
      if (active == 0) break;
      if (it >= d.max_newton) {
        launch_mark_failed(w, batch, s);
        break;
      }
      for (int j = 0; j < kmax; ++j) {
        launch_minv_basis(gs, w, level->tri, level->nmax, j, Bv, mixed, s);
        launch_apply_pk3(gs, w, j, 0.5 * dt, Bv, mixed, s, 0);
        launch_coupling3(gs, (const char*)w.z + (size_t)j * vn * ti, w.w, mixed ? theta_dev : w.coef, 0.5 * dt, Bv,
                         w.inner_active, mixed, s);
        launch_dots(gv, w, j, batch, mixed, s);
        launch_orth(gv, w, j, batch, mixed, s, w.nred);
        launch_givens(gv, w, j, batch, d.inner_tol, s, w.nred);
        HIP_OK(hipMemcpyAsync(&cnt[j], w.counter + 1 + (j & 1), sizeof(int32_t), hipMemcpyDeviceToHost, s));
        HIP_OK(hipEventRecord(level->flag_ev[j & 1], s));
        if (j > 0) {
          HIP_OK(hipEventSynchronize(level->flag_ev[(j - 1) & 1]));
          if (cnt[j - 1] == 0) break;
        }
      }
      launch_solve_y(w, batch, false, s);
      launch_update_zbasis(gv, w, batch, mixed, s);
    }
    launch_block_close(w.u, G, n, batch, w.act, d.u_th, k0, dt, s);
  }
  // the final state (slot 0 after the last block) for the quantities of interest
  HIP_OK(hipMemcpy2DAsync(w.uk, sizeof(double) * n, w.u, sizeof(double) * n * G, sizeof(double) * n, batch,
                          hipMemcpyDeviceToDevice, s));
  launch_qoi(w, level->wts, n, batch, d.qoi, (double)d.n_steps * dt, level->vol, qoi_dev, s);
  HIP_OK(hipMemcpyAsync(status_dev, w.status, sizeof(int32_t) * batch, hipMemcpyDeviceToDevice, s));
  HIP_OK(hipMemcpyAsync(iters_dev, w.iters, sizeof(int64_t) * 2 * batch, hipMemcpyDeviceToDevice, s));
  if (u_out_dev)
    HIP_OK(hipMemcpyAsync(u_out_dev, w.uk, sizeof(double) * n * batch, hipMemcpyDeviceToDevice, s));
  launch_count(w.status, batch, w.counter + 3, nullptr, s);
  HIP_OK(hipGetLastError());
  HIP_OK(hipMemcpyAsync(level->host_flags + 2, w.counter + 3, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  HIP_OK(hipStreamSynchronize(s));
  harvest(level);
  const int32_t bad = level->host_flags[2];
  if (bad) return fail(MLQ_ENOCONV, "%d of %d samples did not converge", bad, batch);
  return MLQ_OK;
}

mlq_status mlq_workspace_bytes_blocks(const mlq_level* level, int32_t batch, int32_t steps_per_block,
                                      size_t* ws_bytes) {
  if (level == nullptr || ws_bytes == nullptr) return fail(MLQ_EINVAL, "NULL argument");
  Geo gs, gv;
  const mlq_status st = block_geos(level, batch, steps_per_block, &gs, &gv);
  if (st != MLQ_OK) return st;
  *ws_bytes = carve_workspace(nullptr, gv, batch, level->kmax, level->mixed, steps_per_block + 1).bytes;
  return MLQ_OK;
}

mlq_status mlq_solve_batch_blocks(mlq_level* level, const void* theta_dev, int32_t batch, int32_t steps_per_block,
                                  int32_t guess, void* ws_dev, size_t ws_bytes, double* qoi_dev, int32_t* status_dev,
                                  int64_t* iters_dev, double* u_out_dev, void* hip_stream) {
  return solve_blocks_impl(level, theta_dev, batch, steps_per_block, guess, ws_dev, ws_bytes, qoi_dev, status_dev,
                           iters_dev, u_out_dev, hip_stream);
}

mlq_status mlq_solve_batch_ex(mlq_level* level, const void* theta_dev, int32_t batch, int32_t n_steps, void* ws_dev,
                              size_t ws_bytes, double* qoi_dev, int32_t* status_dev, int64_t* iters_dev,
                              double* u_out_dev, double* act_out_dev, void* hip_stream) {
  return solve_impl(level, theta_dev, batch, n_steps, ws_dev, ws_bytes, qoi_dev, status_dev, iters_dev, u_out_dev,
                    act_out_dev, nullptr, hip_stream);
}

mlq_status mlq_solve_batch(mlq_level* level, const void* theta_dev, int32_t batch, void* ws_dev, size_t ws_bytes,
                           double* qoi_dev, int32_t* status_dev, int64_t* iters_dev, void* hip_stream) {
  if (level == nullptr) return fail(MLQ_EINVAL, "level is NULL");
  return solve_impl(level, theta_dev, batch, level->d.n_steps, ws_dev, ws_bytes, qoi_dev, status_dev, iters_dev,
                    nullptr, nullptr, nullptr, hip_stream);
}

mlq_status mlq_solve_batch_static(mlq_level* level, const void* theta_dev, int32_t batch, double* qoi_dev,
                                  int32_t* status_dev, int64_t* iters_dev, void* hip_stream) {
  if (level == nullptr) return fail(MLQ_EINVAL, "level is NULL");
  if (batch < 1 || batch > level->d.max_batch) return fail(MLQ_EINVAL, "batch %d outside [1, max_batch]", batch);
  const size_t need = carve_workspace(nullptr, level->geo, batch, level->kmax, level->mixed).bytes;
  if (need > (size_t)MLQ_STATIC_WS_BYTES)
    return fail(MLQ_ESIZE, "the solve needs %zu workspace bytes, more than the static %zu", need,
                (size_t)MLQ_STATIC_WS_BYTES);
  int dev = -1;
  HIP_OK(hipGetDevice(&dev));
  if (dev != level->device)
    return fail(MLQ_EINVAL, "device %d is current, the level lives on device %d", dev, level->device);
  if (dev < 0 || dev >= kMaxDevices) return fail(MLQ_EINVAL, "device index %d not supported", dev);
  void* ws = nullptr;
  {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch[dev] == nullptr) {
      void* p = nullptr;
      HIP_OK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
      if (p == nullptr) return fail(MLQ_EHIP, "hipGetSymbolAddress returned NULL for the static workspace");
      g_scratch[dev] = p;
    }
    ws = g_scratch[dev];
  }
  return solve_impl(level, theta_dev, batch, level->d.n_steps, ws, (size_t)MLQ_STATIC_WS_BYTES, qoi_dev, status_dev,
                    iters_dev, nullptr, nullptr, nullptr, hip_stream);
}

mlq_status mlq_set_lane_layout(mlq_level* level, int32_t lanes_x) {
  if (level == nullptr) return fail(MLQ_EINVAL, "level is NULL");
  if (lanes_x != 0 && lanes_x != 8 && lanes_x != 16) return fail(MLQ_EINVAL, "lanes_x must be 0, 8 or 16");
  if (level->tet || level->geo.dim != 3) return fail(MLQ_EINVAL, "the lane layout applies to 3D box levels");
  level->geo.lx = lanes_x;
  drop_graphs(level);
  return MLQ_OK;
}

mlq_status mlq_set_gmres_block(mlq_level* level, int32_t iterations) {
  if (level == nullptr) return fail(MLQ_EINVAL, "level is NULL");
  if (iterations < 0 || iterations > kMaxInner) return fail(MLQ_EINVAL, "block of %d iterations", iterations);
  if (iterations != level->gmres_block) drop_graphs(level);
  level->gmres_block = iterations;
  return MLQ_OK;
}

mlq_status mlq_set_persistent(mlq_level* level, int32_t on) {
  if (level == nullptr) return fail(MLQ_EINVAL, "level is NULL");
  if (on != 0 && on != 1) return fail(MLQ_EINVAL, "on must be 0 or 1");
  if (on && !small_solver_fits(level->geo, level->mixed))
    return fail(MLQ_EINVAL, "persistent solves need a 3D box level of at most %zu bytes per vector",
                (size_t)kSmallMaxLds);
  level->persistent = on != 0;
  return MLQ_OK;
}

mlq_status mlq_set_reference(mlq_level* level, const double* ref_dev) {
  if (level == nullptr) return fail(MLQ_EINVAL, "level is NULL");
  level->ref = ref_dev;
  return MLQ_OK;
}

mlq_status mlq_solve_batch_fields(mlq_level* level, const void* theta_dev, int32_t batch, void* ws_dev,
                                  size_t ws_bytes, double* qoi_dev, int32_t* status_dev, int64_t* iters_dev,
                                  const mlq_field_out* fields, void* hip_stream) {
  if (level == nullptr || fields == nullptr) return fail(MLQ_EINVAL, "NULL argument");
  return solve_impl(level, theta_dev, batch, level->d.n_steps, ws_dev, ws_bytes, qoi_dev, status_dev, iters_dev,
                    nullptr, nullptr, fields, hip_stream);
}

mlq_status mlq_probe_weights(const mlq_level* level, const double* xyz, int32_t n_points, int64_t* node_out,
                             double* w_out) {
  if (level == nullptr || (n_points > 0 && (xyz == nullptr || node_out == nullptr || w_out == nullptr)))
    return fail(MLQ_EINVAL, "NULL argument");
  if (n_points < 0) return fail(MLQ_EINVAL, "negative point count");
  if (level->tet) return fail(MLQ_EINVAL, "probe weights are computed for box levels; use vertex probes on tetrahedra");
  const mlq_level_desc& d = level->d;
  for (int32_t p = 0; p < n_points; ++p) {
    int64_t q[3] = {0, 0, 0};
    double x[3] = {0.0, 0.0, 0.0};
    for (int a = 0; a < d.dim; ++a) {
      const double h = (d.hi[a] - d.lo[a]) / (double)(d.n[a] - 1);
      const double r = (xyz[3 * p + a] - d.lo[a]) / h;
      if (!(r >= -1e-12 * (double)(d.n[a] - 1) && r <= (double)(d.n[a] - 1) * (1.0 + 1e-12)))
        return fail(MLQ_EINVAL, "probe point %d lies outside the box", p);
      int64_t c = (int64_t)std::floor(r);
      c = std::min<int64_t>(std::max<int64_t>(c, 0), d.n[a] - 2);
      q[a] = c;
      x[a] = std::min(std::max(r - (double)c, 0.0), 1.0);
    }
    for (int c = 0; c < kProbeNodes; ++c) {
      double w = 1.0;
      int64_t idx = 0, stride = 1;
      bool used = true;
      for (int a = 0; a < 3; ++a) {
        const int o = (c >> a) & 1;
        if (a >= d.dim) {
          if (o) used = false;
          continue;
        }
        w *= o ? x[a] : 1.0 - x[a];
        idx += (q[a] + o) * stride;
        stride *= d.n[a];
      }
      node_out[kProbeNodes * p + c] = used ? idx : 0;
      w_out[kProbeNodes * p + c] = used ? w : 0.0;
    }
  }
  return MLQ_OK;
}

mlq_status mlq_tet_locate(const double* xyz, int64_t n_vert, const int32_t* tets, int64_t n_tet, const double* pts,
                          int64_t n_pts, int64_t* node_out, double* w_out) {
  if (xyz == nullptr || tets == nullptr || (n_pts > 0 && (pts == nullptr || node_out == nullptr || w_out == nullptr)))
    return fail(MLQ_EINVAL, "NULL argument");
  if (n_vert < 4 || n_tet < 1 || n_pts < 0) return fail(MLQ_EINVAL, "invalid mesh or point count");
  for (int64_t i = 0; i < 4 * n_tet; ++i)
    if (tets[i] < 0 || tets[i] >= n_vert) return fail(MLQ_EINVAL, "tetrahedron vertex out of range");
  if (n_pts == 0) return MLQ_OK;
  mlq_kl_desc kd{};
  kd.dim = 3;
  kd.mesh_kind = MLQ_MESH_P1_TET;
  kd.n_vert = n_vert;
  kd.n_tet = n_tet;
  kd.xyz = xyz;
  kd.tets = tets;
  std::vector<int32_t> vid;
  std::vector<double> wts;
  std::string err;
  const mlq_status st = locate_points_tet(&kd, pts, n_pts, vid, wts, err);
  if (st != MLQ_OK) return fail(st, "%s", err.c_str());
  for (int64_t i = 0; i < 4 * n_pts; ++i) {
    node_out[i] = vid[i];
    w_out[i] = wts[i];
  }
  return MLQ_OK;
}

mlq_status mlq_transfer_add_weighted(const mlq_level* from, const mlq_level* to, int32_t time, int64_t rows,
                                     int32_t K, const int64_t* node_dev, const double* w_dev, double alpha,
                                     const double* src_dev, double* dst_dev, void* hip_stream) {
  if (from == nullptr || to == nullptr || node_dev == nullptr || w_dev == nullptr || src_dev == nullptr ||
      dst_dev == nullptr)
    return fail(MLQ_EINVAL, "NULL argument");
  if (rows < 1) return fail(MLQ_EINVAL, "rows must be >= 1");
  if (K < 1 || K > kProbeNodes) return fail(MLQ_EINVAL, "nodes per point outside [1, %d]", kProbeNodes);
  XferGeo g;
  for (int a = 0; a < 3; ++a) g.sn_f[a] = g.sn_t[a] = 1;
  g.tn_f = g.tn_t = 1;
  g.m_f = g.m_t = 1;
  if (time) {
    const mlq_level_desc& df = from->d;
    const mlq_level_desc& dt = to->d;
    if (std::fabs(df.t_end - dt.t_end) > 1e-12 * df.t_end) return fail(MLQ_EINVAL, "levels end at different times");
    if (dt.n_steps % df.n_steps != 0) return fail(MLQ_EINVAL, "time grids are not nested");
    g.tn_f = df.n_steps + 1;
    g.tn_t = dt.n_steps + 1;
    g.m_f = df.n_steps;
    g.m_t = dt.n_steps;
  }
  launch_transfer_weighted(g, rows, from->nn, to->nn, K, node_dev, w_dev, alpha, src_dev, dst_dev,
                           (hipStream_t)hip_stream);
  HIP_OK(hipGetLastError());
  return MLQ_OK;
}

mlq_status mlq_field_norm2(const mlq_level* level, int32_t space, int32_t q, int64_t rows, const double* f_dev,
                           double* part_dev, double* out_dev, void* hip_stream) {
  if (level == nullptr || f_dev == nullptr || out_dev == nullptr) return fail(MLQ_EINVAL, "NULL argument");
  if (q != 0 && q != 1) return fail(MLQ_EINVAL, "q must be 0 (L2) or 1 (H1)");
  if (rows < 1 || rows > 65535) return fail(MLQ_EINVAL, "rows outside [1, 65535]");
  const mlq_level_desc& d = level->d;
  const double dt = d.t_end / (double)d.n_steps;
  hipStream_t s = (hipStream_t)hip_stream;
  if (space) {
    if (level->tet) return fail(MLQ_EINVAL, "space-time norms are computed on box levels");
    if (part_dev == nullptr) return fail(MLQ_EINVAL, "space-time norms need the partial-sum scratch");
    NormGeo g;
    g.dim = d.dim;
    for (int a = 0; a < 3; ++a) {
      g.n[a] = a < d.dim ? d.n[a] : 1;
      g.h[a] = a < d.dim ? (d.hi[a] - d.lo[a]) / (double)(d.n[a] - 1) : 1.0;
    }
    g.m = d.n_steps;
    g.dt = dt;
    g.q = q;
    launch_st_norm(g, rows, f_dev, part_dev, out_dev, s);
  } else {
    launch_time_norm(f_dev, rows, d.n_steps, dt, q, out_dev, s);
  }
  HIP_OK(hipGetLastError());
  return MLQ_OK;
}

mlq_status mlq_transfer_add(const mlq_level* from, const mlq_level* to, int32_t space, int32_t time, int64_t rows,
                            double alpha, const double* src_dev, double* dst_dev, void* hip_stream) {
  if (from == nullptr || to == nullptr || src_dev == nullptr || dst_dev == nullptr)
    return fail(MLQ_EINVAL, "NULL argument");
  if (rows < 1) return fail(MLQ_EINVAL, "rows must be >= 1");
  XferGeo g;
  for (int a = 0; a < 3; ++a) g.sn_f[a] = g.sn_t[a] = 1;
  g.tn_f = g.tn_t = 1;
  g.m_f = g.m_t = 1;
  const mlq_level_desc& df = from->d;
  const mlq_level_desc& dt = to->d;
  if (space) {
    if (from->tet || to->tet) return fail(MLQ_EINVAL, "space transfer needs nested box levels");
    if (df.dim != dt.dim) return fail(MLQ_EINVAL, "levels of different dimension");
    for (int a = 0; a < df.dim; ++a) {
      const double tol = 1e-12 * std::max(1.0, std::fabs(df.hi[a] - df.lo[a]));
      if (std::fabs(df.lo[a] - dt.lo[a]) > tol || std::fabs(df.hi[a] - dt.hi[a]) > tol)
        return fail(MLQ_EINVAL, "levels cover different boxes");
      if ((dt.n[a] - 1) % (df.n[a] - 1) != 0) return fail(MLQ_EINVAL, "levels are not nested along axis %d", a);
      g.sn_f[a] = df.n[a];
      g.sn_t[a] = dt.n[a];
    }
  }
  if (time) {
    if (std::fabs(df.t_end - dt.t_end) > 1e-12 * df.t_end) return fail(MLQ_EINVAL, "levels end at different times");
    if (dt.n_steps % df.n_steps != 0) return fail(MLQ_EINVAL, "time grids are not nested");
    g.tn_f = df.n_steps + 1;
    g.tn_t = dt.n_steps + 1;
    g.m_f = df.n_steps;
    g.m_t = dt.n_steps;
  }
  launch_transfer(g, rows, alpha, src_dev, dst_dev, (hipStream_t)hip_stream);
  HIP_OK(hipGetLastError());
  return MLQ_OK;
}

mlq_status mlq_check(const int32_t* status_host, int32_t batch) {
  if (status_host == nullptr || batch < 0) return fail(MLQ_EINVAL, "invalid status array");
  int32_t bad = 0;
  for (int32_t i = 0; i < batch; ++i) bad += status_host[i] != MLQ_SAMPLE_OK;
  if (bad) return fail(MLQ_ENOCONV, "%d of %d samples did not converge", bad, batch);
  return MLQ_OK;
}

mlq_status mlq_lattice_normals(const int64_t* z_dev, const double* shift_dev, int32_t s, int64_t N, int64_t first,
                               int32_t count, double* Y_dev, void* hip_stream) {
  if (z_dev == nullptr || shift_dev == nullptr || Y_dev == nullptr) return fail(MLQ_EINVAL, "NULL argument");
  if (s < 1 || N < 1 || first < 0 || count < 0 || N > (int64_t(1) << 31))
    return fail(MLQ_EINVAL, "invalid lattice size");
  if (count == 0) return MLQ_OK;
  launch_lattice(z_dev, shift_dev, s, N, first, count, false, Y_dev, (hipStream_t)hip_stream);
  HIP_OK(hipGetLastError());
  return MLQ_OK;
}

mlq_status mlq_lattice_points(const int64_t* z_dev, const double* shift_dev, int32_t s, int64_t N, int64_t first,
                              int32_t count, int32_t map, double* Y_dev, void* hip_stream) {
  if (z_dev == nullptr || shift_dev == nullptr || Y_dev == nullptr) return fail(MLQ_EINVAL, "NULL argument");
  if (map != MLQ_MAP_NORMAL && map != MLQ_MAP_UNIFORM) return fail(MLQ_EINVAL, "unknown coordinate map");
  if (s < 1 || N < 1 || first < 0 || count < 0 || N > (int64_t(1) << 31))
    return fail(MLQ_EINVAL, "invalid lattice size");
  if (count == 0) return MLQ_OK;
  launch_lattice(z_dev, shift_dev, s, N, first, count, map == MLQ_MAP_UNIFORM, Y_dev, (hipStream_t)hip_stream);
  HIP_OK(hipGetLastError());
  return MLQ_OK;
}

mlq_status mlq_halton(int32_t s, int64_t first, int32_t count, const double* shift_dev, int32_t map, double* Y_dev,
                      void* hip_stream) {
  if (map != MLQ_MAP_NORMAL && map != MLQ_MAP_UNIFORM) return fail(MLQ_EINVAL, "unknown coordinate map");
  if (s < 1 || s > kHaltonMaxDims) return fail(MLQ_EINVAL, "Halton dimension outside [1, 1024]");
  if (first < 0 || count < 0 || first + count > (int64_t(1) << 32)) return fail(MLQ_EINVAL, "Halton index range");
  if (count == 0) return MLQ_OK;
  if (Y_dev == nullptr) return fail(MLQ_EINVAL, "NULL argument");
  launch_halton(s, first, count, shift_dev, map == MLQ_MAP_UNIFORM, Y_dev, (hipStream_t)hip_stream);
  HIP_OK(hipGetLastError());
  return MLQ_OK;
}

mlq_status mlq_accumulate(const double* f_fine_dev, const double* f_coarse_dev, int32_t count, double* acc_dev,
                          void* hip_stream) {
  if (f_fine_dev == nullptr || acc_dev == nullptr || count < 0) return fail(MLQ_EINVAL, "invalid argument");
  launch_accumulate(f_fine_dev, f_coarse_dev, count, acc_dev, (hipStream_t)hip_stream);
  HIP_OK(hipGetLastError());
  return MLQ_OK;
}

mlq_status mlq_kl_weights(const double* lambda, int32_t M, int32_t map, double* out) {
  if (M < 0 || (M > 0 && (lambda == nullptr || out == nullptr))) return fail(MLQ_EINVAL, "invalid arguments");
  if (map != MLQ_MAP_NORMAL && map != MLQ_MAP_UNIFORM) return fail(MLQ_EINVAL, "unknown coordinate map %d", map);
  // E[y^2] = 1 for a standard normal coordinate, 1/3 for a uniform one on [-1, 1]
  const double inv_second_moment = map == MLQ_MAP_UNIFORM ? 3.0 : 1.0;
  for (int32_t k = 0; k < M; ++k) {
    if (!(lambda[k] >= 0.0) || !std::isfinite(lambda[k])) return fail(MLQ_EINVAL, "eigenvalue %d is %g", k, lambda[k]);
    out[k] = std::sqrt(inv_second_moment * lambda[k]);
  }
  return MLQ_OK;
}

mlq_status mlq_lattice_weights(const double* lambda, int32_t M, int32_t components, double* gamma_out) {
  if (M < 1 || components < 1 || lambda == nullptr || gamma_out == nullptr) return fail(MLQ_EINVAL, "invalid arguments");
  if (!(lambda[0] > 0.0) || !std::isfinite(lambda[0])) return fail(MLQ_EINVAL, "the largest eigenvalue must be positive");
  for (int32_t c = 0; c < components; ++c)
    for (int32_t k = 0; k < M; ++k) {
      if (!(lambda[k] >= 0.0) || lambda[k] > lambda[0]) return fail(MLQ_EINVAL, "eigenvalues must be in [0, lambda_0]");
      gamma_out[(int64_t)c * M + k] = lambda[k] / lambda[0];
    }
  return MLQ_OK;
}

mlq_status mlq_fibre_field(int64_t n, const double* theta0, const double* e_circ, const double* e_long, double scale,
                           double* v_out) {
  if (n < 0 || (n > 0 && (theta0 == nullptr || e_circ == nullptr || e_long == nullptr || v_out == nullptr)))
    return fail(MLQ_EINVAL, "invalid arguments");
  for (int64_t e = 0; e < n; ++e) {
    const double c = std::cos(theta0[e]), sn = std::sin(theta0[e]);
    for (int a = 0; a < 3; ++a) v_out[3 * e + a] = scale * (c * e_circ[3 * e + a] + sn * e_long[3 * e + a]);
  }
  return MLQ_OK;
}

// Component-by-component construction; operations in the order k = 0..N-1 with
// one accumulator and no contraction, so the argmin is reproducible exactly.
mlq_status mlq_cbc(int64_t N, int32_t s, const double* gamma, int64_t* z_out) {
#pragma clang fp contract(off)
  if (gamma == nullptr || z_out == nullptr || N < 1 || s < 1 || N > (int64_t(1) << 20))
    return fail(MLQ_EINVAL, "invalid CBC arguments");
  if (N == 1) {
    for (int j = 0; j < s; ++j) z_out[j] = 1;
    return MLQ_OK;
  }
  std::vector<int64_t> cands;
  for (int64_t z = 1; z < N; ++z) {
    int64_t a = z, b = N;
    while (b) {
      const int64_t t = a % b;
      a = b;
      b = t;
    }
    if (a == 1) cands.push_back(z);
  }
  std::vector<double> Pk(N, 1.0);
  const double Nd = (double)N;
  std::vector<double> err(cands.size());
  for (int j = 0; j < s; ++j) {
    double emin = 0.0;
    for (size_t c = 0; c < cands.size(); ++c) {
      const int64_t z = cands[c];
      double acc = 0.0;
      for (int64_t k = 0; k < N; ++k) {
        const double x = (double)((k * z) % N) / Nd;
        const double b2 = x * x - x + 1.0 / 6.0;
        acc = acc + Pk[k] * (1.0 + gamma[j] * b2);
      }
      err[c] = -1.0 + acc / Nd;
      if (c == 0 || err[c] < emin) emin = err[c];
    }
    // criteria equal up to rounding count as ties and go to the smallest candidate
    const double cut = emin + 1e-12 * std::fabs(emin);
    int64_t bestz = cands[0];
    for (size_t c = 0; c < cands.size(); ++c)
      if (err[c] <= cut) {
        bestz = cands[c];
        break;
      }
    z_out[j] = bestz;
    for (int64_t k = 0; k < N; ++k) {
      const double x = (double)((k * bestz) % N) / Nd;
      const double b2 = x * x - x + 1.0 / 6.0;
      Pk[k] = Pk[k] * (1.0 + gamma[j] * b2);
    }
  }
  return MLQ_OK;
}

// ---------------------------------------------------------------------------
// Estimators, host FP64 (eqs. (SL), (StandardML), (PimpedML)).
static double mean_of(const double* v, int64_t n) {
  double s = 0.0;
  for (int64_t i = 0; i < n; ++i) s += v[i];
  return s / (double)n;
}

static double var_of(const double* v, int64_t n) {
  if (n < 2) return 0.0;
  const double m = mean_of(v, n);
  double s = 0.0;
  for (int64_t i = 0; i < n; ++i) s += (v[i] - m) * (v[i] - m);
  return s / (double)(n - 1);
}

mlq_status mlq_estimate(int32_t kind, int32_t n_levels, int32_t n_shifts, const int64_t* n_per_level,
                        const double* const* f_fine, const double* const* f_coarse, mlq_estimate_out* out) {
  if (out == nullptr || n_per_level == nullptr || f_fine == nullptr) return fail(MLQ_EINVAL, "NULL argument");
  if (n_levels < 1 || n_levels > 16) return fail(MLQ_EINVAL, "n_levels must be in [1, 16]");
  std::memset(out, 0, sizeof(*out));
  out->n_levels = n_levels;
  for (int l = 0; l < n_levels; ++l)
    if (n_per_level[l] < 1 || f_fine[l] == nullptr) return fail(MLQ_EINVAL, "level %d has no samples", l);
  if (kind == MLQ_EST_MC) {
    if (n_levels != 1) return fail(MLQ_EINVAL, "MC estimator takes one level");
    const int64_t n = n_per_level[0];
    out->estimate = mean_of(f_fine[0], n);
    out->level_mean[0] = out->estimate;
    out->level_var[0] = var_of(f_fine[0], n);
    out->rmse = std::sqrt(out->level_var[0] / (double)n);
    return MLQ_OK;
  }
  if (kind == MLQ_EST_MLMC || kind == MLQ_EST_MLQMC) {
    const int S = kind == MLQ_EST_MLQMC ? n_shifts : 1;
    if (S < 1) return fail(MLQ_EINVAL, "n_shifts must be >= 1");
    double est = 0.0, mse = 0.0;
    for (int l = 0; l < n_levels; ++l) {
      if (l > 0 && (f_coarse == nullptr || f_coarse[l] == nullptr)) return fail(MLQ_EINVAL, "level %d needs f_coarse", l);
      const int64_t n = n_per_level[l];
      std::vector<double> y((size_t)S * n);
      for (int64_t i = 0; i < (int64_t)S * n; ++i) y[i] = f_fine[l][i] - (l > 0 ? f_coarse[l][i] : 0.0);
      if (kind == MLQ_EST_MLMC) {
        const double m = mean_of(y.data(), n), v = var_of(y.data(), n);
        out->level_mean[l] = m;
        out->level_var[l] = v;
        est += m;
        mse += v / (double)n;
      } else {
        std::vector<double> q(S);
        for (int sh = 0; sh < S; ++sh) q[sh] = mean_of(y.data() + (size_t)sh * n, n);
        const double m = mean_of(q.data(), S);
        double ss = 0.0;
        for (int sh = 0; sh < S; ++sh) ss += (q[sh] - m) * (q[sh] - m);
        out->level_mean[l] = m;
        out->level_var[l] = var_of(y.data(), (int64_t)S * n);
        est += m;
        if (S > 1) mse += ss / ((double)S * (double)(S - 1));
      }
    }
    out->estimate = est;
    out->rmse = std::sqrt(mse);
    return MLQ_OK;
  }
  if (kind == MLQ_EST_COMBINATION) {
    const int L = n_levels - 1;
    double est = 0.0;
    for (int l = 0; l <= L; ++l) {
      if (l > 0 && n_per_level[l] < n_per_level[l - 1]) return fail(MLQ_EINVAL, "point sets must be nested");
      const double* F = f_fine[L - l];
      const double ql = mean_of(F, n_per_level[l]);
      const double qm = l > 0 ? mean_of(F, n_per_level[l - 1]) : 0.0;
      out->level_mean[l] = ql - qm;
      est += ql - qm;
    }
    out->estimate = est;
    out->rmse = 0.0;
    return MLQ_OK;
  }
  return fail(MLQ_EINVAL, "unknown estimator kind %d", kind);
}

// ---------------------------------------------------------------------------
// KL set-up
mlq_status mlq_kl_workspace_bytes(const mlq_kl_desc* kd, size_t* ws_bytes) {
  if (ws_bytes == nullptr || kl_validate(kd) != MLQ_OK) return fail(MLQ_EINVAL, "invalid KL descriptor");
  *ws_bytes = kl_workspace_bytes(kd);
  if (*ws_bytes == 0) return fail(MLQ_EHIP, "FFT plans of the exact KL route could not be created");
  return MLQ_OK;
}

mlq_status mlq_kl_modes(const mlq_kl_desc* kd, void* ws_dev, size_t ws_bytes, double* lambda_host, double* psi_dev,
                        int32_t* rank_out, double* resid_out, void* hip_stream) {
  if (kl_validate(kd) != MLQ_OK) return fail(MLQ_EINVAL, "invalid KL descriptor");
  if (ws_dev == nullptr || (kd->n_modes > 0 && (lambda_host == nullptr || psi_dev == nullptr)))
    return fail(MLQ_EINVAL, "NULL argument");
  if (ws_bytes < kl_workspace_bytes(kd)) return fail(MLQ_ESIZE, "KL workspace too small");
  if (((uintptr_t)ws_dev & 255) != 0) return fail(MLQ_EINVAL, "workspace must be 256-byte aligned");
  std::string err;
  mlq_status st = kl_modes(kd, ws_dev, lambda_host, psi_dev, rank_out, resid_out, (hipStream_t)hip_stream, err);
  if (st != MLQ_OK) return fail(st, "%s", err.c_str());
  return MLQ_OK;
}

mlq_status mlq_kl_transfer(const mlq_kl_desc* kd, const double* psi_dev, const int64_t* level_n,
                           const double* level_lo, const double* level_hi, double* phi_dev, void* hip_stream) {
  if (kl_validate(kd) != MLQ_OK) return fail(MLQ_EINVAL, "invalid KL descriptor");
  if (psi_dev == nullptr || level_n == nullptr || level_lo == nullptr || level_hi == nullptr || phi_dev == nullptr)
    return fail(MLQ_EINVAL, "NULL argument");
  for (int a = 0; a < kd->dim; ++a)
    if (level_n[a] < 2 || !(level_hi[a] > level_lo[a])) return fail(MLQ_EINVAL, "invalid level box");
  mlq_status st = kl_transfer(kd, psi_dev, level_n, level_lo, level_hi, phi_dev, (hipStream_t)hip_stream);
  if (st != MLQ_OK) return fail(st, "transfer launch failed");
  return MLQ_OK;
}

mlq_status mlq_kl_transfer_tet_bytes(int64_t n_tet, size_t* ws_bytes) {
  if (ws_bytes == nullptr || n_tet < 1) return fail(MLQ_EINVAL, "invalid argument");
  *ws_bytes = kl_transfer_tet_bytes(n_tet);
  return MLQ_OK;
}

mlq_status mlq_kl_transfer_tet(const mlq_kl_desc* kd, const double* psi_dev, int64_t n_vert, const double* xyz,
                               int64_t n_tet, const int32_t* tets, void* ws_dev, size_t ws_bytes, double* phi_dev,
                               void* hip_stream) {
  if (kl_validate(kd) != MLQ_OK || kd->mesh_kind != MLQ_MESH_P1_TET)
    return fail(MLQ_EINVAL, "invalid tetrahedral KL descriptor");
  if (psi_dev == nullptr || xyz == nullptr || tets == nullptr || ws_dev == nullptr || phi_dev == nullptr)
    return fail(MLQ_EINVAL, "NULL argument");
  if (n_vert < 4 || n_tet < 1) return fail(MLQ_EINVAL, "invalid level mesh");
  for (int64_t i = 0; i < 4 * n_tet; ++i)
    if (tets[i] < 0 || tets[i] >= n_vert) return fail(MLQ_EINVAL, "level vertex index out of range");
  if (ws_bytes < kl_transfer_tet_bytes(n_tet)) return fail(MLQ_ESIZE, "transfer workspace too small");
  if (((uintptr_t)ws_dev & 255) != 0) return fail(MLQ_EINVAL, "workspace must be 256-byte aligned");
  std::string err;
  mlq_status st = kl_transfer_tet(kd, psi_dev, n_vert, xyz, n_tet, tets, ws_dev, phi_dev, (hipStream_t)hip_stream, err);
  if (st != MLQ_OK) return fail(st, "%s", err.c_str());
  return MLQ_OK;
}

}  // extern "C"
