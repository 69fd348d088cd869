// C ABI of the library (declared in include/wfd.h): argument validation,
// model preparation, workspace carving, and the stream-ordered time loops of
// forward modeling (Alg. 1) and the one-shot gradient (Alg. 3).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "wfd.h"
#include "wfd_internal.h"
#include "wfd_plan.h"

namespace {

thread_local std::string g_last_error;

wfd_status fail(wfd_status s, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return s;
}

#define HIP_TRY(expr)                                                                   \
  do {                                                                                  \
    hipError_t e_ = (expr);                                                             \
    if (e_ != hipSuccess)                                                               \
      return fail(WFD_E_HIP, "%s failed: %s (%s:%d)", #expr, hipGetErrorString(e_),    \
                  __FILE__, __LINE__);                                                  \
  } while (0)

constexpr size_t kAlign = 256;
inline size_t align_up(size_t v, size_t a = kAlign) { return (v + a - 1) / a * a; }

// Bump allocator over a caller buffer (or a null base for sizing).
struct Carve {
  char *base;
  size_t off = 0;
  explicit Carve(void *b) : base((char *)b) {}
  template <class T>
  T *take(size_t count) {
    off = align_up(off);
    T *p = base ? (T *)(base + off) : nullptr;
    off += count * sizeof(T);
    return p;
  }
};

constexpr int kReducePartials = 1024;
constexpr int kMaxBatch = 64;  // shots per wfd_batch

}  // namespace

// Device staging volumes of the host-stored forward wavefield (WFD_CKPT_HOST).
constexpr int kHostRing = 4;

struct wfd_ctx {
  int device = 0;
  hipStream_t stream = nullptr;

  // model
  bool has_model = false;
  uint64_t model_gen = 0;  // incremented by every wfd_set_model (batches check it)
  wfd_grid grid{};
  int Nx = 0, Ny = 0, Nz = 0, pitch = 0;
  int64_t plane = 0, vol = 0;  // floats
  bool vd = false;
  float *k = nullptr, *m2 = nullptr, *sqrt_rho = nullptr;
  float *gx = nullptr, *gy = nullptr, *gz = nullptr;
  bool cpml = false;         // CPML layer instead of the sponge
  wfd::CpmlTables cpml_tab{};
  wfd::Shell shell{};        // the points the layer's terms reach
  int64_t cpml_len[3] = {1, 1, 1};  // floats of a compact memory variable per axis

  // host staging of the receiver tables (kept alive until the upload ends)
  std::vector<char> stage;
  hipEvent_t upload_done = nullptr;
  bool upload_pending = false;

  wfd::Tuning tuning;  // forward tile shape / z chunking (wfd_set_tuning, wfd_autotune)

  // host-stored forward wavefield (WFD_CKPT_HOST): a copy stream and the
  // events that order it against the step kernels, created on first use
  hipStream_t copy_stream = nullptr;
  hipEvent_t host_ev_step[kHostRing] = {};  // recorded on the compute stream
  hipEvent_t host_ev_copy[kHostRing] = {};  // recorded on the copy stream
  hipEvent_t host_ev_end = nullptr;

  // profiling
  bool prof = false;
  std::vector<hipEvent_t> pool;
  size_t pool_used = 0;
  std::vector<int> rec_class;  // class of event pair i (pool[2i], pool[2i+1])
  int64_t launches[WFD_K_COUNT] = {0, 0, 0};
  double ms[WFD_K_COUNT] = {0, 0, 0};
};

// A set of shots advanced together: one launch per time step covers every
// shot's window (its own context, model and workspace); the time loop can be
// captured once into a HIP graph and replayed.
struct wfd_batch {
  std::vector<wfd_ctx *> ctxs;
  std::vector<uint64_t> model_gen;  // each context's model generation at creation
  std::vector<float *> W1, W2, seis_tm, seis_out;
  std::vector<int> nrec;
  wfd::WindowStep *d_wins[2] = {nullptr, nullptr};  // device descriptors per step parity
  std::vector<wfd::WindowStep> h_wins[2];
  int nblocks = 0, variant = 0, nt = 0;
  bool vd = false;
  bool fs = false;  // some shot has a free surface
  hipStream_t stream = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

namespace {

struct ScopedDevice {
  int prev = -1;
  explicit ScopedDevice(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    if (prev != dev) (void)hipSetDevice(dev);
  }
  ~ScopedDevice() {
    int cur = -1;
    if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
  }
};

// Per-launch HIP-event timing (only when profiling is on).
struct Timed {
  wfd_ctx *c;
  int cls;
  size_t idx = 0;
  bool on;
  Timed(wfd_ctx *ctx, int klass) : c(ctx), cls(klass), on(ctx->prof) {
    if (!on) return;
    if (c->pool_used + 2 > c->pool.size()) {
      for (int i = 0; i < 256; ++i) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) {
          on = false;
          return;
        }
        c->pool.push_back(e);
      }
    }
    idx = c->pool_used;
    c->pool_used += 2;
    c->rec_class.push_back(cls);
    (void)hipEventRecord(c->pool[idx], c->stream);
  }
  ~Timed() {
    if (on) (void)hipEventRecord(c->pool[idx + 1], c->stream);
  }
};

wfd_status drain_profile(wfd_ctx *c) {
  if (c->pool_used == 0) return WFD_OK;
  HIP_TRY(hipStreamSynchronize(c->stream));
  for (size_t i = 0; i + 1 < c->pool_used; i += 2) {
    float t = 0.0f;
    HIP_TRY(hipEventElapsedTime(&t, c->pool[i], c->pool[i + 1]));
    const int cls = c->rec_class[i / 2];
    c->launches[cls] += 1;
    c->ms[cls] += t;
  }
  c->pool_used = 0;
  c->rec_class.clear();
  return WFD_OK;
}

wfd_status check_grid(const wfd_grid *g) {
  if (!g) return fail(WFD_E_ARG, "grid is NULL");
  if (g->nx < 1 || g->ny < 1 || g->nz < 1)
    return fail(WFD_E_ARG, "model size must be >= 1 per axis (got %d %d %d)", g->nx, g->ny, g->nz);
  if (!(g->dx > 0) || !(g->dy > 0) || !(g->dz > 0) || !std::isfinite(g->dx) ||
      !std::isfinite(g->dy) || !std::isfinite(g->dz))
    return fail(WFD_E_ARG, "grid spacing must be finite and > 0");
  if (!std::isfinite(g->ox) || !std::isfinite(g->oy) || !std::isfinite(g->oz))
    return fail(WFD_E_ARG, "origin must be finite");
  if (g->border < 0) return fail(WFD_E_ARG, "border must be >= 0 (got %d)", g->border);
  if (!(g->dt > 0) || !std::isfinite(g->dt)) return fail(WFD_E_ARG, "dt must be finite and > 0");
  if (g->nt < 1) return fail(WFD_E_ARG, "nt must be >= 1 (got %d)", g->nt);
  if (g->free_surface != 0 && g->free_surface != 1)
    return fail(WFD_E_ARG, "free_surface must be 0 or 1 (got %d)", g->free_surface);
  if (g->cpml != 0 && g->cpml != 1)
    return fail(WFD_E_ARG, "cpml must be 0 or 1 (got %d)", g->cpml);
  if (g->cpml && (!(g->fpeak >= 0) || !std::isfinite(g->fpeak)))
    return fail(WFD_E_ARG, "fpeak must be finite and >= 0");
  if (g->cpml && (!(g->cpml_vmax >= 0) || !std::isfinite(g->cpml_vmax)))
    return fail(WFD_E_ARG, "cpml_vmax must be finite and >= 0");
  const int64_t Nx = (int64_t)g->nx + 2 * g->border, Ny = (int64_t)g->ny + 2 * g->border,
                Nz = (int64_t)g->nz + 2 * g->border;
  // the step kernels address a pitched x-y plane with 32-bit byte offsets
  if (Nx > (1 << 24) || Ny > (1 << 24) || Nz > (1 << 24) ||
      (Nx + 63) / 64 * 64 * Ny >= (int64_t(1) << 30))
    return fail(WFD_E_ARG, "padded grid too large");
  return WFD_OK;
}

int pitch_of(int Nx) { return (Nx + 63) / 64 * 64; }

// Model buffer layout (shared by wfd_model_bytes and wfd_set_model).
struct ModelLayout {
  float *k, *m2, *sqrt_rho, *gx, *gy, *gz, *part_v, *part_m;
  float *cpml[6];  // a_x, b_x, a_y, b_y, a_z, b_z (CPML only)
  size_t bytes;
};
ModelLayout model_layout(const wfd_grid &g, bool vd, void *base) {
  const int Nx = g.nx + 2 * g.border, Ny = g.ny + 2 * g.border, Nz = g.nz + 2 * g.border;
  const size_t vol = (size_t)pitch_of(Nx) * Ny * Nz;
  Carve cv(base);
  ModelLayout L{};
  L.k = cv.take<float>(vol);
  L.m2 = vd ? cv.take<float>(vol) : nullptr;
  L.sqrt_rho = vd ? cv.take<float>((size_t)g.nx * g.ny * g.nz) : nullptr;
  L.gx = cv.take<float>(Nx);
  L.gy = cv.take<float>(Ny);
  L.gz = cv.take<float>(Nz);
  L.part_v = cv.take<float>(kReducePartials);
  L.part_m = cv.take<float>(kReducePartials);
  if (g.cpml) {
    const int len[6] = {Nx, Nx, Ny, Ny, Nz, Nz};
    for (int i = 0; i < 6; ++i) L.cpml[i] = cv.take<float>(len[i]);
  }
  L.bytes = align_up(cv.off);
  return L;
}

// CPML recursive-convolution coefficients along one padded axis: depth delta
// into the layer, d = d0 (delta/N)^2 with d0 = -3 vmax ln(1e-3) / (2 N h),
// alpha = pi fpeak (1 - delta/N), b = exp(-(d + alpha) dt),
// a = d (b - 1) / (d + alpha) (0 outside the layer).  FP64, stored as FP32.
void cpml_table(int n, int border, double h, double dt, double vmax, double fpeak,
                bool free_top, std::vector<float> &a, std::vector<float> &b) {
  const int total = n + 2 * border;
  a.assign(total, 0.0f);
  b.assign(total, 1.0f);
  if (border == 0) return;
  const double d0 = -3.0 * vmax * std::log(1.0e-3) / (2.0 * border * h);
  for (int i = 0; i < total; ++i) {
    const int before = free_top ? 0 : border - i;
    const int delta = std::max(std::max(before, 0), i - (border + n - 1));
    if (delta == 0) continue;
    const double r = (double)delta / border;
    const double d = d0 * r * r;
    const double alpha = M_PI * fpeak * (1.0 - r);
    const double bb = std::exp(-(d + alpha) * dt);
    b[i] = (float)bb;
    a[i] = (float)(d * (bb - 1.0) / (d + alpha));
  }
}

// The shell: padded points within 4 cells (along an axis) of that axis'
// layer, i.e. the grid minus the inner box, as up to 6 boxes.
wfd::Shell make_shell(const wfd_grid &g, int Nx, int Ny, int Nz) {
  const int N = g.border;
  auto inner = [&](int n, int total, bool low_layer, int &lo, int &hi) {
    lo = (N > 0 && low_layer) ? N + wfd::kStencilRadius : 0;
    hi = N > 0 ? N + n - 1 - wfd::kStencilRadius : total - 1;  // inclusive
  };
  int zlo, zhi, ylo, yhi, xlo, xhi;
  inner(g.nz, Nz, g.free_surface == 0, zlo, zhi);
  inner(g.ny, Ny, true, ylo, yhi);
  inner(g.nx, Nx, true, xlo, xhi);
  wfd::Shell sh{};
  const bool empty_inner = N == 0 || zlo > zhi || ylo > yhi || xlo > xhi;
  sh.lo[0] = empty_inner ? Nx : xlo, sh.hi[0] = empty_inner ? -1 : xhi;
  sh.lo[1] = empty_inner ? Ny : ylo, sh.hi[1] = empty_inner ? -1 : yhi;
  sh.lo[2] = empty_inner ? Nz : zlo, sh.hi[2] = empty_inner ? -1 : zhi;
  auto add = [&](int z0, int z1, int y0, int y1, int x0, int x1) {
    if (z1 <= z0 || y1 <= y0 || x1 <= x0) return;
    const int b = sh.nbox++;
    sh.z0[b] = z0, sh.z1[b] = z1, sh.y0[b] = y0, sh.y1[b] = y1, sh.x0[b] = x0, sh.x1[b] = x1;
    sh.zfirst[b] = (z1 - z0) < (y1 - y0);
  };
  if (N == 0) {
    // no layer: empty shell
  } else if (zlo > zhi || ylo > yhi || xlo > xhi) {
    add(0, Nz, 0, Ny, 0, Nx);  // the inner box is empty: every point
  } else {
    add(0, zlo, 0, Ny, 0, Nx);
    add(zhi + 1, Nz, 0, Ny, 0, Nx);
    add(zlo, zhi + 1, 0, ylo, 0, Nx);
    add(zlo, zhi + 1, yhi + 1, Ny, 0, Nx);
    add(zlo, zhi + 1, ylo, yhi + 1, 0, xlo);
    add(zlo, zhi + 1, ylo, yhi + 1, xhi + 1, Nx);
  }
  sh.start[0] = 0;
  sh.bstart[0] = 0;
  for (int b = 0; b < sh.nbox; ++b) {
    const int nxb = sh.x1[b] - sh.x0[b], nyb = sh.y1[b] - sh.y0[b], nzb = sh.z1[b] - sh.z0[b];
    sh.start[b + 1] = sh.start[b] + (int64_t)nzb * nyb * nxb;
    // a plane of the box within reach of a z layer
    sh.zq[b] = sh.z0[b] < sh.lo[2] || sh.z1[b] - 1 > sh.hi[2];
    sh.cz[b] = sh.zq[b] ? wfd::kShellChunkZ : wfd::kShellChunk;
    sh.tx[b] = (nxb + wfd::kShellTileX - 1) / wfd::kShellTileX;
    sh.ty[b] = (nyb + wfd::kShellTileY - 1) / wfd::kShellTileY;
    sh.nch[b] = (nzb + sh.cz[b] - 1) / sh.cz[b];
    sh.bstart[b + 1] = sh.bstart[b] + (int64_t)sh.tx[b] * sh.ty[b] * sh.nch[b];
  }
  return sh;
}

// Sponge profile of one padded axis; free_top: no damping before the model
// (the side of a free surface).
std::vector<float> sponge_table(int n, int border, bool free_top = false) {
  std::vector<float> t(n + 2 * border, 1.0f);
  if (border == 0) return t;
  for (int i = 0; i < n + 2 * border; ++i) {
    const int before = free_top ? 0 : border - i;
    int d = std::max(std::max(before, 0), i - (border + n - 1));
    const double r = 0.4 * (double)d / (double)border;
    t[i] = (float)std::exp(-r * r);
  }
  return t;
}

// Workspace layout for one shot.
struct Work {
  // receiver tables (uploaded)
  int *col_start, *ent_z, *ent_rp, *perm, *rec_model_idx;
  int64_t *rec_idx;
  // device-computed scalars / scales
  wfd::ShotScale *scale;  // sigma 2^e and the field exponent e
  float *rec_scale, *rec_adj;
  float *seis_tm;
  float *W1, *W2;
  wfd::WindowStep *wins;  // batch step descriptors (two parities x kMaxBatch)
  wfd::GradWindow *gwins;  // batched-gradient window descriptors (kMaxBatch)
  // gradient only
  float *res_tm, *P1, *P2, *g, *store;
  double *partial;
  int64_t n_store_vols;
  float *mem[6];   // CPML memory variables psi_x..z, zeta_x..z (adjoint: mu, nu)
  float *cstore;   // CPML, full storage: correction C^n of every step on the shell
  // CPML with checkpointing: the adjoint's own mu, nu; one memory-variable set
  // per checkpoint slot; the correction of the latest forward step and one
  // recomputed for a visit (both on the shell)
  float *amem[6];
  float *smem;
  float *lastc, *visitc;
  size_t bytes;
};

// Floats of CPML memory variable i (psi or zeta, mu or nu, of axis i % 3) and
// of a set of all six.
int64_t mem_len(const wfd_ctx *c, int i) { return c->cpml_len[i % 3]; }
int64_t mem_set_len(const wfd_ctx *c) {
  return 2 * (c->cpml_len[0] + c->cpml_len[1] + c->cpml_len[2]);
}

int64_t snapshots_for(const wfd_ctx *c, const wfd_ckpt *ck) {
  if (ck->mode == WFD_CKPT_FULL) return c->grid.nt;
  if (ck->mode == WFD_CKPT_HOST) return 0;
  if (ck->n_snapshots > 0) return ck->n_snapshots;
  size_t free_b = 0, total_b = 0;
  if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) return 0;
  const double frac = (ck->mem_fraction > 0 && ck->mem_fraction <= 1.0) ? ck->mem_fraction : 0.8;
  // a checkpoint holds a leapfrog pair, and with CPML a set of six memory
  // variables on the layer
  const double pair =
      (2.0 * (double)c->vol + (c->cpml ? (double)mem_set_len(c) : 0.0)) * sizeof(float);
  int64_t s = (int64_t)(frac * (double)free_b / pair);
  return std::max<int64_t>(1, std::min<int64_t>(s, c->grid.nt));
}

wfd_status check_ckpt_mode(const wfd_ckpt *ck) {
  if (ck->mode != WFD_CKPT_FULL && ck->mode != WFD_CKPT_REVOLVE && ck->mode != WFD_CKPT_HOST)
    return fail(WFD_E_ARG, "unknown checkpoint mode %d", ck->mode);
  if (ck->mode == WFD_CKPT_REVOLVE && ck->n_snapshots < 0)
    return fail(WFD_E_ARG, "n_snapshots must be >= 0");
  return WFD_OK;
}

size_t host_store_bytes(const wfd_ctx *c) {
  return (size_t)c->grid.nt * (size_t)c->vol * sizeof(float);
}

// The host store of WFD_CKPT_HOST: present, large enough and page-locked
// (pageable memory would make every copy synchronous).
wfd_status check_host_store(const wfd_ctx *c, const wfd_ckpt *ck) {
  if (!ck->host_store) return fail(WFD_E_ARG, "host store is NULL");
  if (ck->host_bytes < host_store_bytes(c))
    return fail(WFD_E_NOMEM, "host store has %llu bytes, %zu needed",
                (unsigned long long)ck->host_bytes, host_store_bytes(c));
  hipPointerAttribute_t attr{};
  if (hipPointerGetAttributes(&attr, ck->host_store) != hipSuccess ||
      attr.type != hipMemoryTypeHost) {
    (void)hipGetLastError();
    return fail(WFD_E_ARG, "host store must be page-locked host memory (hipHostMalloc)");
  }
  return WFD_OK;
}

// The copy stream and events of WFD_CKPT_HOST (default priority, non-blocking
// with respect to the legacy stream).
wfd_status ensure_copy_stream(wfd_ctx *c) {
  if (c->host_ev_end) return WFD_OK;
  if (!c->copy_stream) HIP_TRY(hipStreamCreateWithFlags(&c->copy_stream, hipStreamNonBlocking));
  for (int i = 0; i < kHostRing; ++i) {
    if (!c->host_ev_step[i])
      HIP_TRY(hipEventCreateWithFlags(&c->host_ev_step[i], hipEventDisableTiming));
    if (!c->host_ev_copy[i])
      HIP_TRY(hipEventCreateWithFlags(&c->host_ev_copy[i], hipEventDisableTiming));
  }
  HIP_TRY(hipEventCreateWithFlags(&c->host_ev_end, hipEventDisableTiming));  // last: marks done
  return WFD_OK;
}

enum class WorkKind { Forward, Misfit, Gradient };

// Workspace layout of one shot.  Forward: tables, traces, two fields; Misfit
// adds the residual; Gradient adds the adjoint pair, g and the stored states.
Work work_layout(const wfd_ctx *c, int nrec, WorkKind kind, const wfd_ckpt *ck, int64_t nsnap,
                 void *base) {
  Carve cv(base);
  Work w{};
  const int ncol = c->Nx * c->Ny;
  w.col_start = cv.take<int>((size_t)ncol + 1);
  w.ent_z = cv.take<int>((size_t)std::max(nrec, 1));
  w.ent_rp = cv.take<int>((size_t)nrec + 1);
  w.perm = cv.take<int>((size_t)std::max(nrec, 1));
  w.rec_model_idx = cv.take<int>((size_t)std::max(nrec, 1));
  w.rec_idx = cv.take<int64_t>((size_t)std::max(nrec, 1));
  w.scale = cv.take<wfd::ShotScale>(1);
  w.rec_scale = cv.take<float>((size_t)std::max(nrec, 1));
  w.rec_adj = cv.take<float>((size_t)std::max(nrec, 1));
  w.seis_tm = cv.take<float>((size_t)c->grid.nt * std::max(nrec, 1));
  w.W1 = cv.take<float>((size_t)c->vol);
  w.W2 = cv.take<float>((size_t)c->vol);
  w.wins = kind == WorkKind::Forward ? cv.take<wfd::WindowStep>(2 * kMaxBatch) : nullptr;
  w.gwins = kind == WorkKind::Gradient ? cv.take<wfd::GradWindow>(kMaxBatch) : nullptr;
  if (kind != WorkKind::Forward) {
    w.res_tm = cv.take<float>((size_t)c->grid.nt * std::max(nrec, 1));
    w.partial = cv.take<double>((size_t)std::max(1, wfd::residual_partial_count(nrec, c->grid.nt)));
  }
  if (c->cpml) {
    const size_t S = (size_t)c->shell.start[c->shell.nbox];
    for (int i = 0; i < 6; ++i) w.mem[i] = cv.take<float>((size_t)mem_len(c, i));
    if (kind == WorkKind::Gradient && ck && ck->mode == WFD_CKPT_FULL)
      w.cstore = cv.take<float>((size_t)c->grid.nt * S);
    if (kind == WorkKind::Gradient && ck && ck->mode == WFD_CKPT_REVOLVE) {
      for (int i = 0; i < 6; ++i) w.amem[i] = cv.take<float>((size_t)mem_len(c, i));
      w.smem = cv.take<float>((size_t)nsnap * (size_t)mem_set_len(c));
      w.lastc = cv.take<float>(std::max<size_t>(S, 1));
      w.visitc = cv.take<float>(std::max<size_t>(S, 1));
    }
  }
  if (kind == WorkKind::Gradient) {
    w.P1 = cv.take<float>((size_t)c->vol);
    w.P2 = cv.take<float>((size_t)c->vol);
    w.g = cv.take<float>((size_t)c->vol);
    w.n_store_vols = ck->mode == WFD_CKPT_FULL   ? (int64_t)c->grid.nt
                     : ck->mode == WFD_CKPT_HOST ? (int64_t)kHostRing
                                                 : 2 * nsnap;
    w.store = cv.take<float>((size_t)w.n_store_vols * (size_t)c->vol);
  }
  w.bytes = align_up(cv.off);
  return w;
}

wfd::StepGrid step_grid(const wfd_ctx *c) {
  wfd::StepGrid g;
  g.nx = c->Nx;
  g.ny = c->Ny;
  g.nz = c->Nz;
  g.pitch = c->pitch;
  g.plane = c->plane;
  g.cx = (float)(1.0 / (c->grid.dx * c->grid.dx));
  g.cy = (float)(1.0 / (c->grid.dy * c->grid.dy));
  g.cz = (float)(1.0 / (c->grid.dz * c->grid.dz));
  g.gx = c->gx;
  g.gy = c->gy;
  g.gz = c->gz;
  g.k = c->k;
  g.m2 = c->vd ? c->m2 : nullptr;
  g.zs = c->grid.free_surface ? c->grid.border : wfd::kNoSurface;
  return g;
}

int64_t lin(const wfd_ctx *c, const int32_t ijk[3]) {
  return (int64_t)ijk[2] * c->plane + (int64_t)ijk[1] * c->pitch + ijk[0];
}

// Map positions, group receivers by column, upload tables, launch shot setup.
wfd_status prepare_shot(wfd_ctx *c, const float *wavelet, const double src_xyz[3], int nrec,
                        const double *rec_xyz, const Work &w, int64_t &src_idx) {
  const wfd_grid &g = c->grid;
  int32_t s[3];
  if (!wfd::map_position(g, src_xyz, s))
    return fail(WFD_E_RANGE, "source (%g, %g, %g) is outside the model", src_xyz[0], src_xyz[1],
                src_xyz[2]);
  src_idx = lin(c, s);
  const int src_model =
      ((s[2] - g.border) * g.ny + (s[1] - g.border)) * g.nx + (s[0] - g.border);

  struct R {
    int col, z, id;
    int64_t idx;
    int model;
  };
  std::vector<R> recs((size_t)nrec);
  for (int r = 0; r < nrec; ++r) {
    int32_t ijk[3];
    if (!wfd::map_position(g, rec_xyz + 3 * (size_t)r, ijk))
      return fail(WFD_E_RANGE, "receiver %d (%g, %g, %g) is outside the model", r,
                  rec_xyz[3 * r], rec_xyz[3 * r + 1], rec_xyz[3 * r + 2]);
    recs[r] = R{ijk[1] * c->Nx + ijk[0], ijk[2], r, lin(c, ijk),
                ((ijk[2] - g.border) * g.ny + (ijk[1] - g.border)) * g.nx + (ijk[0] - g.border)};
  }
  std::vector<R> sorted = recs;
  std::stable_sort(sorted.begin(), sorted.end(), [](const R &a, const R &b) {
    return a.col != b.col ? a.col < b.col : a.z < b.z;
  });
  const int ncol = c->Nx * c->Ny;
  std::vector<int> col_start((size_t)ncol + 1, 0), ent_z, ent_rp, perm;
  ent_rp.push_back(0);
  std::vector<int> ent_col;
  for (size_t i = 0; i < sorted.size(); ++i) {
    if (i == 0 || sorted[i].col != sorted[i - 1].col || sorted[i].z != sorted[i - 1].z) {
      if (i > 0) ent_rp.push_back((int)i);
      ent_z.push_back(sorted[i].z);
      ent_col.push_back(sorted[i].col);
    }
    perm.push_back(sorted[i].id);
  }
  if (!sorted.empty()) ent_rp.push_back((int)sorted.size());
  // col_start: first entry of each column
  {
    size_t e = 0;
    for (int col = 0; col <= ncol; ++col) {
      while (e < ent_col.size() && ent_col[e] < col) ++e;
      col_start[col] = (int)e;
    }
  }
  // staging blob: ints then int64
  if (c->upload_pending) {
    HIP_TRY(hipEventSynchronize(c->upload_done));
    c->upload_pending = false;
  }
  const size_t n_ent = ent_z.size();
  const size_t sz_col = (size_t)(ncol + 1) * sizeof(int);
  const size_t total = sz_col + (n_ent + (n_ent + 1) + 2 * (size_t)nrec) * sizeof(int) +
                       (size_t)nrec * sizeof(int64_t) + 64;
  c->stage.resize(total);
  char *p = c->stage.data();
  std::memcpy(p, col_start.data(), sz_col);
  HIP_TRY(hipMemcpyAsync(w.col_start, p, sz_col, hipMemcpyHostToDevice, c->stream));
  p += sz_col;
  auto up = [&](void *dst, const void *src, size_t bytes) -> hipError_t {
    if (bytes == 0) return hipSuccess;
    std::memcpy(p, src, bytes);
    hipError_t e = hipMemcpyAsync(dst, p, bytes, hipMemcpyHostToDevice, c->stream);
    p += bytes;
    return e;
  };
  std::vector<int> rmodel((size_t)nrec);
  std::vector<int64_t> ridx((size_t)nrec);
  for (int r = 0; r < nrec; ++r) {
    rmodel[r] = recs[r].model;
    ridx[r] = recs[r].idx;
  }
  HIP_TRY(up(w.ent_z, ent_z.data(), n_ent * sizeof(int)));
  HIP_TRY(up(w.ent_rp, ent_rp.data(), ent_rp.size() * sizeof(int)));
  HIP_TRY(up(w.perm, perm.data(), perm.size() * sizeof(int)));
  HIP_TRY(up(w.rec_model_idx, rmodel.data(), rmodel.size() * sizeof(int)));
  HIP_TRY(up(w.rec_idx, ridx.data(), ridx.size() * sizeof(int64_t)));
  HIP_TRY(hipEventRecord(c->upload_done, c->stream));
  c->upload_pending = true;

  const double dt2_over_h3 = g.dt * g.dt / (g.dx * g.dy * g.dz);
  {
    Timed t(c, WFD_K_OTHER);
    HIP_TRY(wfd::launch_shot_setup(c->k, c->vd ? c->sqrt_rho : nullptr, src_idx, src_model,
                                   dt2_over_h3, wavelet, g.nt, w.rec_idx, w.rec_model_idx, nrec,
                                   w.scale, w.rec_scale, w.rec_adj, c->stream));
  }
  return WFD_OK;
}

wfd::RecTable rec_table(const Work &w, int nrec) {
  wfd::RecTable t;
  t.col_start = w.col_start;
  t.ent_z = w.ent_z;
  t.ent_rp = w.ent_rp;
  t.perm = w.perm;
  t.nrec = nrec;
  return t;
}

wfd_status zero(wfd_ctx *c, float *p, int64_t n) {
  Timed t(c, WFD_K_OTHER);
  HIP_TRY(wfd::launch_fill_zero(p, n, c->stream));
  return WFD_OK;
}

wfd_status common_checks(wfd_ctx *c, const float *wavelet, const double *src, int nrec,
                         const double *rec) {
  if (!c) return fail(WFD_E_ARG, "ctx is NULL");
  if (!c->has_model) return fail(WFD_E_STATE, "no model: call wfd_set_model first");
  if (!wavelet) return fail(WFD_E_ARG, "wavelet is NULL");
  if (!src) return fail(WFD_E_ARG, "source position is NULL");
  if (nrec < 0) return fail(WFD_E_ARG, "nrec must be >= 0");
  if (nrec > 0 && !rec) return fail(WFD_E_ARG, "receiver positions are NULL");
  return WFD_OK;
}

}  // namespace

namespace {

// Average time (ms) of `steps` launches of `launch` on the context's stream,
// after one untimed launch.
template <class F>
hipError_t time_steps(wfd_ctx *c, int steps, hipEvent_t e0, hipEvent_t e1, F launch, float *ms) {
  hipError_t err = launch();
  if (err == hipSuccess) err = hipEventRecord(e0, c->stream);
  for (int n = 0; n < steps && err == hipSuccess; ++n) err = launch();
  if (err == hipSuccess) err = hipEventRecord(e1, c->stream);
  if (err == hipSuccess) err = hipEventSynchronize(e1);
  if (err == hipSuccess) err = hipEventElapsedTime(ms, e0, e1);
  if (err == hipSuccess) *ms /= (float)steps;
  return err;
}

}  // namespace

namespace wfd {
int ctx_device(const wfd_ctx *c) { return c->device; }
wfd_status set_error(wfd_status status, const char *message) {
  g_last_error = message;
  return status;
}
}  // namespace wfd

extern "C" {

const char *wfd_last_error(void) { return g_last_error.c_str(); }

wfd_status wfd_create(wfd_ctx **out, int32_t device, void *hip_stream) {
  if (!out) return fail(WFD_E_ARG, "ctx pointer is NULL");
  *out = nullptr;
  int n = 0;
  HIP_TRY(hipGetDeviceCount(&n));
  if (device < 0 || device >= n) return fail(WFD_E_ARG, "device %d out of range (%d)", device, n);
  wfd_ctx *c = new (std::nothrow) wfd_ctx();
  if (!c) return fail(WFD_E_NOMEM, "out of host memory");
  c->device = device;
  c->stream = (hipStream_t)hip_stream;
  ScopedDevice sd(device);
  if (hipEventCreateWithFlags(&c->upload_done, hipEventDisableTiming) != hipSuccess) {
    delete c;
    return fail(WFD_E_HIP, "hipEventCreate failed");
  }
  *out = c;
  return WFD_OK;
}

wfd_status wfd_set_stream(wfd_ctx *c, void *hip_stream) {
  if (!c) return fail(WFD_E_ARG, "ctx is NULL");
  c->stream = (hipStream_t)hip_stream;
  return WFD_OK;
}

wfd_status wfd_destroy(wfd_ctx *c) {
  if (!c) return WFD_OK;
  ScopedDevice sd(c->device);
  if (c->upload_pending) (void)hipEventSynchronize(c->upload_done);
  if (c->upload_done) (void)hipEventDestroy(c->upload_done);
  for (hipEvent_t e : c->pool) (void)hipEventDestroy(e);
  if (c->copy_stream) (void)hipStreamSynchronize(c->copy_stream);
  for (int i = 0; i < kHostRing; ++i) {
    if (c->host_ev_step[i]) (void)hipEventDestroy(c->host_ev_step[i]);
    if (c->host_ev_copy[i]) (void)hipEventDestroy(c->host_ev_copy[i]);
  }
  if (c->host_ev_end) (void)hipEventDestroy(c->host_ev_end);
  if (c->copy_stream) (void)hipStreamDestroy(c->copy_stream);
  delete c;
  return WFD_OK;
}

wfd_status wfd_model_bytes(const wfd_grid *grid, int32_t variable_density, size_t *bytes) {
  if (!bytes) return fail(WFD_E_ARG, "bytes is NULL");
  wfd_status s = check_grid(grid);
  if (s != WFD_OK) return s;
  *bytes = model_layout(*grid, variable_density != 0, nullptr).bytes;
  return WFD_OK;
}

wfd_status wfd_set_model(wfd_ctx *c, const wfd_grid *grid, const float *vel,
                         const float *rho, void *model, size_t model_bytes) {
  if (!c) return fail(WFD_E_ARG, "ctx is NULL");
  wfd_status s = check_grid(grid);
  if (s != WFD_OK) return s;
  if (!vel) return fail(WFD_E_ARG, "velocity is NULL");
  if (!model) return fail(WFD_E_ARG, "model buffer is NULL");
  const bool vd = rho != nullptr;
  ModelLayout L = model_layout(*grid, vd, model);
  if (model_bytes < L.bytes)
    return fail(WFD_E_NOMEM, "model buffer has %zu bytes, %zu needed", model_bytes, L.bytes);
  if ((uintptr_t)model % kAlign) return fail(WFD_E_ARG, "model buffer must be 256-byte aligned");
  ScopedDevice sd(c->device);
  c->has_model = false;
  c->grid = *grid;
  c->Nx = grid->nx + 2 * grid->border;
  c->Ny = grid->ny + 2 * grid->border;
  c->Nz = grid->nz + 2 * grid->border;
  c->pitch = pitch_of(c->Nx);
  c->plane = (int64_t)c->pitch * c->Ny;
  c->vol = c->plane * c->Nz;
  c->vd = vd;
  c->k = L.k;
  c->m2 = L.m2;
  c->sqrt_rho = L.sqrt_rho;
  c->gx = L.gx;
  c->gy = L.gy;
  c->gz = L.gz;
  c->cpml = grid->cpml != 0;

  // pitch padding of the coefficient volumes is never read by the kernels
  // but is cleared so the buffer holds no stale values
  {
    Timed t(c, WFD_K_OTHER);
    HIP_TRY(wfd::launch_fill_zero(c->k, c->vol, c->stream));
  }
  if (vd) {
    Timed t(c, WFD_K_OTHER);
    HIP_TRY(wfd::launch_fill_zero(c->m2, c->vol, c->stream));
  }
  // with the CPML layer the sponge tables are all ones (no damping)
  const int sb = c->cpml ? 0 : grid->border;
  std::vector<float> tx = sponge_table(grid->nx + 2 * grid->border - 2 * sb, sb);
  std::vector<float> ty = sponge_table(grid->ny + 2 * grid->border - 2 * sb, sb);
  std::vector<float> tz =
      sponge_table(grid->nz + 2 * grid->border - 2 * sb, sb, grid->free_surface != 0);
  HIP_TRY(hipMemcpyAsync(c->gx, tx.data(), tx.size() * 4, hipMemcpyHostToDevice, c->stream));
  HIP_TRY(hipMemcpyAsync(c->gy, ty.data(), ty.size() * 4, hipMemcpyHostToDevice, c->stream));
  HIP_TRY(hipMemcpyAsync(c->gz, tz.data(), tz.size() * 4, hipMemcpyHostToDevice, c->stream));
  {
    Timed t(c, WFD_K_OTHER);
    HIP_TRY(wfd::launch_precompute_k(vel, grid->nx, grid->ny, grid->nz, grid->border, grid->dt,
                                     c->k, c->pitch, c->Ny, c->Nz, L.part_v, kReducePartials,
                                     c->stream));
  }
  if (vd) {
    Timed t(c, WFD_K_OTHER);
    HIP_TRY(wfd::launch_precompute_m2(rho, grid->nx, grid->ny, grid->nz, grid->border,
                                      grid->free_surface, 1.0 / (grid->dx * grid->dx), 1.0 / (grid->dy * grid->dy),
                                      1.0 / (grid->dz * grid->dz), c->m2, c->pitch, c->Ny, c->Nz,
                                      c->sqrt_rho, L.part_m, kReducePartials, c->stream));
  }
  std::vector<float> pv(kReducePartials), pm(kReducePartials, 0.0f);
  HIP_TRY(hipMemcpyAsync(pv.data(), L.part_v, kReducePartials * 4, hipMemcpyDeviceToHost,
                         c->stream));
  if (vd)
    HIP_TRY(hipMemcpyAsync(pm.data(), L.part_m, kReducePartials * 4, hipMemcpyDeviceToHost,
                           c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  const double vmax = *std::max_element(pv.begin(), pv.end());
  const double m2max = vd ? *std::max_element(pm.begin(), pm.end()) : 0.0;
  if (!(vmax > 0) || !std::isfinite(vmax))
    return fail(WFD_E_ARG, "velocity must be finite and > 0 (max %g)", vmax);
  const double ratio = wfd::cfl_ratio(*grid, vmax, m2max);
  if (!(ratio < 1.0))
    return fail(WFD_E_CFL,
                "unstable: dt^2 vmax^2 (Lambda + m2max) / 4 = %g >= 1 (vmax %g, dt %g); "
                "reduce dt below %g",
                ratio, vmax, grid->dt, grid->dt / std::sqrt(ratio));
  if (c->cpml) {
    const double v = grid->cpml_vmax > 0 ? grid->cpml_vmax : vmax;
    std::vector<float> ab[6];
    cpml_table(grid->nx, grid->border, grid->dx, grid->dt, v, grid->fpeak, false, ab[0], ab[1]);
    cpml_table(grid->ny, grid->border, grid->dy, grid->dt, v, grid->fpeak, false, ab[2], ab[3]);
    cpml_table(grid->nz, grid->border, grid->dz, grid->dt, v, grid->fpeak,
               grid->free_surface != 0, ab[4], ab[5]);
    for (int i = 0; i < 6; ++i)
      HIP_TRY(hipMemcpyAsync(L.cpml[i], ab[i].data(), ab[i].size() * sizeof(float),
                             hipMemcpyHostToDevice, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    c->cpml_tab = wfd::CpmlTables{L.cpml[0], L.cpml[1], L.cpml[2], L.cpml[3], L.cpml[4],
                                  L.cpml[5], (float)(1.0 / grid->dx), (float)(1.0 / grid->dy),
                                  (float)(1.0 / grid->dz),
                                  {wfd::cpml_slab_half(c->Nx, grid->border),
                                   wfd::cpml_slab_half(c->Ny, grid->border),
                                   wfd::cpml_slab_half(c->Nz, grid->border)},
                                  {wfd::cpml_slab_len(c->Nx, grid->border),
                                   wfd::cpml_slab_len(c->Ny, grid->border),
                                   wfd::cpml_slab_len(c->Nz, grid->border)}};
    for (int d = 0; d < 3; ++d)
      c->cpml_len[d] = std::max<int64_t>(
          1, wfd::cpml_mem_len(d, c->Nx, c->Ny, c->Nz, grid->border));
    c->shell = make_shell(*grid, c->Nx, c->Ny, c->Nz);
    for (int b = 0; b < c->shell.nbox; ++b)
      if (c->shell.start[b + 1] - c->shell.start[b] >= (int64_t(1) << 31))
        return fail(WFD_E_ARG, "padded grid too large for the CPML layer's point boxes");
  }
  c->has_model = true;
  ++c->model_gen;
  return WFD_OK;
}

wfd_status wfd_misfit_workspace_bytes(const wfd_ctx *c, int32_t nrec, size_t *bytes) {
  if (!c || !bytes) return fail(WFD_E_ARG, "NULL argument");
  if (!c->has_model) return fail(WFD_E_STATE, "no model: call wfd_set_model first");
  if (nrec < 0) return fail(WFD_E_ARG, "nrec must be >= 0");
  *bytes = work_layout(c, nrec, WorkKind::Misfit, nullptr, 0, nullptr).bytes;
  return WFD_OK;
}

wfd_status wfd_workspace_bytes(const wfd_ctx *c, int32_t nrec, const wfd_ckpt *ck, size_t *bytes) {
  if (!c || !bytes) return fail(WFD_E_ARG, "NULL argument");
  if (!c->has_model) return fail(WFD_E_STATE, "no model: call wfd_set_model first");
  if (nrec < 0) return fail(WFD_E_ARG, "nrec must be >= 0");
  int64_t nsnap = 0;
  if (ck) {
    wfd_status s = check_ckpt_mode(ck);
    if (s != WFD_OK) return s;
    ScopedDevice sd(c->device);
    nsnap = snapshots_for(c, ck);
  }
  *bytes = work_layout(c, nrec, ck ? WorkKind::Gradient : WorkKind::Forward, ck, nsnap, nullptr)
               .bytes;
  return WFD_OK;
}

wfd_status wfd_host_store_bytes(const wfd_ctx *c, size_t *bytes) {
  if (!c || !bytes) return fail(WFD_E_ARG, "NULL argument");
  if (!c->has_model) return fail(WFD_E_STATE, "no model: call wfd_set_model first");
  *bytes = host_store_bytes(c);
  return WFD_OK;
}

namespace {

// The CPML layer's share of forward step n (after the step kernel wrote out
// from cur): memory variables, the correction k C added to out, C kept in
// cstore when given, and the receivers read from out afterwards.
wfd_status cpml_forward_terms(wfd_ctx *c, const wfd::StepGrid &g, const Work &w,
                              const float *cur, float *out, float *cstore, int nrec, int n,
                              float *const *mem = nullptr) {
  Timed t(c, WFD_K_OTHER);
  float *const *m = mem ? mem : w.mem;  // out == nullptr: only the memory variables and C
  HIP_TRY(wfd::launch_cpml_psi(g, c->cpml_tab, c->shell, cur, m[0], m[1], m[2], c->stream));
  HIP_TRY(wfd::launch_cpml_zeta(g, c->cpml_tab, c->shell, cur, m[0], m[1], m[2], m[3], m[4],
                                m[5], out, cstore, c->stream));
  if (nrec > 0 && out)
    HIP_TRY(wfd::launch_record(out, w.rec_idx, w.rec_scale, nrec, n, w.seis_tm, c->stream));
  return WFD_OK;
}

// The CPML layer's share of adjoint step m: nu and mu from phi^{m+1} (phi1)
// before the step kernel, then (pre = false) the correction of phi^m and the
// imaging term phi^{m+1} C^m.
wfd_status cpml_adjoint_terms(wfd_ctx *c, const wfd::StepGrid &g, const Work &w,
                              const float *phi1, float *phi, int m, bool pre,
                              const float *corr_m = nullptr) {
  Timed t(c, WFD_K_OTHER);
  float *const *v = w.smem ? w.amem : w.mem;  // mu = v[0..2], nu = v[3..5]
  if (pre) {
    HIP_TRY(wfd::launch_cpml_nu(g, c->cpml_tab, c->shell, phi1, v[3], v[4], v[5], c->stream));
    HIP_TRY(wfd::launch_cpml_mu(g, c->cpml_tab, c->shell, phi1, v[3], v[4], v[5], v[0], v[1],
                                v[2], c->stream));
    return WFD_OK;
  }
  const float *cst = m >= c->grid.nt ? nullptr
                     : corr_m      ? corr_m
                     : w.cstore    ? w.cstore + (size_t)m * (size_t)c->shell.start[c->shell.nbox]
                                   : nullptr;
  HIP_TRY(wfd::launch_cpml_adjoint(g, c->cpml_tab, c->shell, v[3], v[4], v[5], v[0], v[1], v[2],
                                   phi, phi1, cst, w.g, c->stream));
  return WFD_OK;
}

// Forward sweep of one shot; optionally the trace output, the final states and
// the misfit against observed data (then the workspace also holds the residual).
wfd_status forward_core(wfd_ctx *c, const float *wavelet, const double src_xyz[3], int32_t nrec,
                        const double *rec_xyz, float *seis, float *final_dev, const float *dobs,
                        double *misfit, void *work, size_t work_bytes, bool with_misfit) {
  wfd_status s = common_checks(c, wavelet, src_xyz, nrec, rec_xyz);
  if (s != WFD_OK) return s;
  if (!work) return fail(WFD_E_ARG, "workspace is NULL");
  if ((uintptr_t)work % kAlign) return fail(WFD_E_ARG, "workspace must be 256-byte aligned");
  Work w = work_layout(c, nrec, with_misfit ? WorkKind::Misfit : WorkKind::Forward, nullptr, 0,
                       work);
  if (work_bytes < w.bytes)
    return fail(WFD_E_NOMEM, "workspace has %zu bytes, %zu needed", work_bytes, w.bytes);
  ScopedDevice sd(c->device);
  int64_t src_idx = 0;
  s = prepare_shot(c, wavelet, src_xyz, nrec, rec_xyz, w, src_idx);
  if (s != WFD_OK) return s;
  if ((s = zero(c, w.W1, c->vol)) != WFD_OK) return s;
  if ((s = zero(c, w.W2, c->vol)) != WFD_OK) return s;
  const wfd::StepGrid g = step_grid(c);
  const wfd::RecTable rt = rec_table(w, nrec);
  const wfd::Source src{src_idx, &w.scale->sigma, wavelet};
  if (c->cpml)
    for (int i = 0; i < 6; ++i)
      if ((s = zero(c, w.mem[i], mem_len(c, i))) != WFD_OK) return s;
  float *cur = w.W1, *prev = w.W2;
  for (int n = 0; n < c->grid.nt; ++n) {
    {
      Timed t(c, WFD_K_FORWARD);
      HIP_TRY(wfd::launch_forward_step(g, cur, prev, prev, src, n,
                                       (nrec > 0 && !c->cpml) ? &rt : nullptr, w.rec_scale,
                                       w.seis_tm, c->tuning, c->stream));
    }
    if (c->cpml && (s = cpml_forward_terms(c, g, w, cur, prev, nullptr, nrec, n)) != WFD_OK)
      return s;
    std::swap(cur, prev);
  }
  if (nrec > 0 && seis) {
    Timed t(c, WFD_K_OTHER);
    HIP_TRY(wfd::launch_transpose(w.seis_tm, seis, nrec, c->grid.nt, c->stream));
  }
  if (with_misfit && nrec > 0) {
    int np = 0;
    {
      Timed t(c, WFD_K_OTHER);
      HIP_TRY(wfd::launch_residual(w.seis_tm, dobs, w.rec_adj, w.scale, nrec, c->grid.nt,
                                   w.res_tm, w.partial, &np, c->stream));
    }
    Timed t(c, WFD_K_OTHER);
    HIP_TRY(wfd::launch_sum_partials(w.partial, np, misfit, c->stream));
  }
  if (final_dev) {  // the last two states, back from 2^e w to w
    const size_t dense = (size_t)c->Nx * c->Ny * c->Nz;
    Timed t(c, WFD_K_OTHER);
    HIP_TRY(wfd::launch_unscale_copy(cur, final_dev, c->Nx, c->Ny, c->Nz, c->pitch, w.scale,
                                     c->stream));
    HIP_TRY(wfd::launch_unscale_copy(prev, final_dev + dense, c->Nx, c->Ny, c->Nz, c->pitch,
                                     w.scale, c->stream));
  }
  return WFD_OK;
}

}  // namespace

wfd_status wfd_forward(wfd_ctx *c, const float *wavelet, const double src_xyz[3], int32_t nrec,
                       const double *rec_xyz, float *seis, float *final_dev, void *work,
                       size_t work_bytes) {
  if (c && nrec > 0 && !seis) return fail(WFD_E_ARG, "seismogram output is NULL");
  return forward_core(c, wavelet, src_xyz, nrec, rec_xyz, seis, final_dev, nullptr, nullptr,
                      work, work_bytes, false);
}

wfd_status wfd_forward_misfit(wfd_ctx *c, const float *wavelet, const double src_xyz[3],
                              int32_t nrec, const double *rec_xyz, const float *dobs,
                              float *seis_or_null, double *misfit, void *work,
                              size_t work_bytes) {
  if (c && nrec > 0 && !dobs) return fail(WFD_E_ARG, "observed data is NULL");
  if (c && !misfit) return fail(WFD_E_ARG, "misfit output is NULL");
  return forward_core(c, wavelet, src_xyz, nrec, rec_xyz, seis_or_null, nullptr, dobs, misfit,
                      work, work_bytes, true);
}

wfd_status wfd_gradient(wfd_ctx *c, const float *wavelet, const double src_xyz[3], int32_t nrec,
                        const double *rec_xyz, const float *dobs, const wfd_ckpt *ck,
                        float *seis, double *misfit, float *grad, float *illum, void *work,
                        size_t work_bytes) {
  return wfd_gradient_ex(c, wavelet, src_xyz, nrec, rec_xyz, dobs, ck, seis, misfit, grad, illum,
                         nullptr, work, work_bytes);
}

wfd_status wfd_gradient_ex(wfd_ctx *c, const float *wavelet, const double src_xyz[3],
                           int32_t nrec, const double *rec_xyz, const float *dobs,
                           const wfd_ckpt *ck, float *seis, double *misfit, float *grad,
                           float *illum, const wfd_gradient_opts *opts, void *work,
                           size_t work_bytes) {
  float *const wavelet_grad = opts ? opts->wavelet_grad_dev : nullptr;
  const int out_exp2 = opts ? opts->out_exp2 : 0;
  int32_t *const field_exp2 = opts ? opts->field_exp2_dev : nullptr;
  if (out_exp2 < -2 * wfd::kMaxFieldExp || out_exp2 > 2 * wfd::kMaxFieldExp)
    return fail(WFD_E_ARG, "out_exp2 must be in [-%d, %d]", 2 * wfd::kMaxFieldExp,
                2 * wfd::kMaxFieldExp);
  wfd_status s = common_checks(c, wavelet, src_xyz, nrec, rec_xyz);
  if (s != WFD_OK) return s;
  if (!ck) return fail(WFD_E_ARG, "checkpoint policy is NULL");
  if ((s = check_ckpt_mode(ck)) != WFD_OK) return s;
  if (nrec > 0 && !dobs) return fail(WFD_E_ARG, "observed data is NULL");
  if (!misfit || !grad) return fail(WFD_E_ARG, "misfit / gradient output is NULL");
  if (!work) return fail(WFD_E_ARG, "workspace is NULL");
  if ((uintptr_t)work % kAlign) return fail(WFD_E_ARG, "workspace must be 256-byte aligned");
  ScopedDevice sd(c->device);
  if (c->cpml && ck->mode == WFD_CKPT_HOST)
    return fail(WFD_E_ARG, "the CPML gradient needs device storage (full or checkpointed)");
  if (ck->mode == WFD_CKPT_HOST) {
    if ((s = check_host_store(c, ck)) != WFD_OK) return s;
    if ((s = ensure_copy_stream(c)) != WFD_OK) return s;
  }
  int64_t nsnap = 0;
  if (ck->mode == WFD_CKPT_FULL) {
    nsnap = c->grid.nt;
  } else if (ck->mode == WFD_CKPT_HOST) {
    nsnap = 0;
  } else if (ck->n_snapshots > 0) {
    nsnap = ck->n_snapshots;
  } else {
    // derived count: as many pairs as the given workspace holds
    const size_t base = work_layout(c, nrec, WorkKind::Gradient, ck, 0, nullptr).bytes;
    const size_t pair = align_up((size_t)c->vol * sizeof(float)) * 2 +
                        (c->cpml ? (size_t)mem_set_len(c) * sizeof(float) : 0);
    nsnap = work_bytes > base ? (int64_t)((work_bytes - base) / pair) : 0;
    nsnap = std::min<int64_t>(nsnap, c->grid.nt);
    if (nsnap < 1) return fail(WFD_E_NOMEM, "workspace holds no checkpoint pair");
    while (nsnap > 1 && work_layout(c, nrec, WorkKind::Gradient, ck, nsnap, nullptr).bytes > work_bytes)
      --nsnap;
  }
  Work w = work_layout(c, nrec, WorkKind::Gradient, ck, nsnap, work);
  if (work_bytes < w.bytes)
    return fail(WFD_E_NOMEM, "workspace has %zu bytes, %zu needed", work_bytes, w.bytes);
  int64_t src_idx = 0;
  s = prepare_shot(c, wavelet, src_xyz, nrec, rec_xyz, w, src_idx);
  if (s != WFD_OK) return s;
  const int nt = c->grid.nt;
  const wfd::StepGrid g = step_grid(c);
  const wfd::RecTable rt = rec_table(w, nrec);
  const wfd::Source src{src_idx, &w.scale->sigma, wavelet};
  const wfd::IllumOut il{illum, c->grid.border, c->grid.nx, c->grid.ny, c->grid.nz, w.scale,
                         out_exp2};
  if (field_exp2) {
    Timed t(c, WFD_K_OTHER);
    HIP_TRY(hipMemcpyAsync(field_exp2, &w.scale->e, sizeof(int32_t), hipMemcpyDeviceToDevice,
                           c->stream));
  }
  for (float *p : {w.W1, w.W2, w.P1, w.P2, w.g})
    if ((s = zero(c, p, c->vol)) != WFD_OK) return s;

  // adjoint state: psi^{m+1} = A1, psi^{m+2} = A2 (psi^m overwrites A2)
  float *A1 = w.P1, *A2 = w.P2;
  bool residual_done = false;
  auto residual = [&]() -> wfd_status {
    if (residual_done) return WFD_OK;
    residual_done = true;
    if (nrec == 0) return WFD_OK;
    int np = 0;
    {
      Timed t(c, WFD_K_OTHER);
      HIP_TRY(wfd::launch_residual(w.seis_tm, dobs, w.rec_adj, w.scale, nrec, nt, w.res_tm,
                                   w.partial, &np, c->stream));
    }
    {
      Timed t(c, WFD_K_OTHER);
      HIP_TRY(wfd::launch_sum_partials(w.partial, np, misfit, c->stream));
    }
    if (seis) {
      Timed t(c, WFD_K_OTHER);
      HIP_TRY(wfd::launch_transpose(w.seis_tm, seis, nrec, nt, c->stream));
    }
    return WFD_OK;
  };
  auto adjoint = [&](int m, const float *wm, const float *corr_m = nullptr) -> wfd_status {
    if (c->cpml && (s = cpml_adjoint_terms(c, g, w, A1, A2, m, true)) != WFD_OK) return s;
    {
      Timed t(c, WFD_K_ADJOINT);
      HIP_TRY(wfd::launch_adjoint_step(c->tuning, g, A1, A2, A2, rt, w.res_tm, m, wm, w.g, il,
                                       c->stream));
    }
    if (c->cpml && (s = cpml_adjoint_terms(c, g, w, A1, A2, m, false, corr_m)) != WFD_OK)
      return s;
    if (wavelet_grad) {  // psi^m (in A2) at the source
      Timed t(c, WFD_K_OTHER);
      HIP_TRY(wfd::launch_source_gradient(A2, c->k, src_idx, w.scale, out_exp2, m, wavelet_grad,
                                          c->stream));
    }
    std::swap(A1, A2);
    return WFD_OK;
  };
  int last_c_step = -1;  // CPML with checkpointing: the step whose C w.lastc holds
  auto fwd = [&](const float *cur, const float *prev, float *out, int n, bool rec) -> wfd_status {
    {
      Timed t(c, WFD_K_FORWARD);
      HIP_TRY(wfd::launch_forward_step(g, cur, prev, out, src, n,
                                       (rec && nrec > 0 && !c->cpml) ? &rt : nullptr, w.rec_scale,
                                       w.seis_tm, c->tuning, c->stream));
    }
    if (c->cpml) {  // full storage keeps every step's C; checkpointing the latest
      float *cst = w.cstore ? w.cstore + (size_t)n * (size_t)c->shell.start[c->shell.nbox]
                            : w.lastc;
      if ((s = cpml_forward_terms(c, g, w, cur, out, cst, rec ? nrec : 0, n)) != WFD_OK)
        return s;
      last_c_step = n;
    }
    return WFD_OK;
  };

  if (ck->mode == WFD_CKPT_FULL) {
    // slot m holds w^m (m = 1..nt); w^0 = W1 and w^-1 = W2 are zero
    auto S = [&](int m) -> float * {
      if (m == 0) return w.W1;
      if (m < 0) return w.W2;
      return w.store + (size_t)(m - 1) * (size_t)c->vol;
    };
    if (c->cpml)
      for (int i = 0; i < 6; ++i)
        if ((s = zero(c, w.mem[i], mem_len(c, i))) != WFD_OK) return s;
    for (int n = 0; n < nt; ++n)
      if ((s = fwd(S(n), S(n - 1), S(n + 1), n, true)) != WFD_OK) return s;
    if ((s = residual()) != WFD_OK) return s;
    if (c->cpml)  // the adjoint's mu and nu start at zero
      for (int i = 0; i < 6; ++i)
        if ((s = zero(c, w.mem[i], mem_len(c, i))) != WFD_OK) return s;
    for (int m = nt; m >= 1; --m)
      if ((s = adjoint(m, S(m))) != WFD_OK) return s;
  } else if (ck->mode == WFD_CKPT_HOST) {
    // w^m (m >= 1) is staged in D[(m - 1) % R] and kept in host slot m - 1.
    // Forward: once the step that writes D[i] is done, the copy stream moves
    // it to the host; the step that next writes D[i] waits for that copy.
    // Adjoint (m = nt .. 1): the last R states are still staged; w^(m-R) is
    // fetched into D[i] as soon as the adjoint step that read w^m from D[i]
    // is done, so each fetch overlaps R - 1 adjoint steps.
    const int R = kHostRing;
    float *D[kHostRing];
    for (int i = 0; i < R; ++i) D[i] = w.store + (size_t)i * (size_t)c->vol;
    float *host = static_cast<float *>(ck->host_store);
    const size_t vbytes = (size_t)c->vol * sizeof(float);
    hipStream_t cs = c->copy_stream;
    auto S = [&](int m) -> float * {
      if (m == 0) return w.W1;
      if (m < 0) return w.W2;
      return D[(m - 1) % R];
    };
    for (int n = 0; n < nt; ++n) {
      const int i = n % R;  // receives w^(n+1)
      if (n >= R) HIP_TRY(hipStreamWaitEvent(c->stream, c->host_ev_copy[i], 0));
      if ((s = fwd(S(n), S(n - 1), D[i], n, true)) != WFD_OK) return s;
      HIP_TRY(hipEventRecord(c->host_ev_step[i], c->stream));
      HIP_TRY(hipStreamWaitEvent(cs, c->host_ev_step[i], 0));
      HIP_TRY(hipMemcpyAsync(host + (size_t)n * (size_t)c->vol, D[i], vbytes,
                             hipMemcpyDeviceToHost, cs));
      HIP_TRY(hipEventRecord(c->host_ev_copy[i], cs));
    }
    if ((s = residual()) != WFD_OK) return s;
    for (int m = nt; m >= 1; --m) {
      const int i = (m - 1) % R;
      if (m <= nt - R) HIP_TRY(hipStreamWaitEvent(c->stream, c->host_ev_copy[i], 0));
      if ((s = adjoint(m, D[i])) != WFD_OK) return s;
      if (m - R >= 1) {
        HIP_TRY(hipEventRecord(c->host_ev_step[i], c->stream));
        HIP_TRY(hipStreamWaitEvent(cs, c->host_ev_step[i], 0));
        HIP_TRY(hipMemcpyAsync(D[i], host + (size_t)(m - R - 1) * (size_t)c->vol, vbytes,
                               hipMemcpyHostToDevice, cs));
        HIP_TRY(hipEventRecord(c->host_ev_copy[i], cs));
      }
    }
    // the caller's stream passes the end of the call only after every copy
    HIP_TRY(hipEventRecord(c->host_ev_end, cs));
    HIP_TRY(hipStreamWaitEvent(c->stream, c->host_ev_end, 0));
  } else {
    std::vector<int32_t> plan;
    int64_t nsteps = 0;
    wfd::build_checkpoint_plan(nt, (int32_t)nsnap, plan, nsteps);
    // Zero-copy checkpointing: W1, W2 and the 2*nsnap store volumes form one
    // pool.  Storing a state pins the two buffers the current state already
    // holds; advancing from a pinned state writes into free buffers, and a
    // step updates in place only over a buffer nobody has pinned.
    std::vector<float *> buf;
    buf.push_back(w.W1);
    buf.push_back(w.W2);
    for (int64_t i = 0; i < 2 * nsnap; ++i) buf.push_back(w.store + (size_t)i * (size_t)c->vol);
    std::vector<int> pins(buf.size(), 0);
    struct Slot {
      int state = -1, a = -1, b = -1;  // state index, buffers of w^state and w^(state-1)
    };
    std::vector<Slot> slots((size_t)nsnap);
    int cur_state = -1, cur = -1, prev = -1;  // working state and its buffers
    int reached = 0;                         // steps whose data has been recorded
    auto slot_of = [&](int state) -> Slot * {
      for (auto &sl : slots)
        if (sl.state == state) return &sl;
      return nullptr;
    };
    auto free_buffer = [&](int not1, int not2) -> int {
      for (size_t i = 0; i < buf.size(); ++i)
        if (pins[i] == 0 && (int)i != not1 && (int)i != not2) return (int)i;
      return -1;
    };
    // CPML: a state m also carries the memory variables of step m - 1, kept in
    // w.mem while m is the working state and copied to and from slot sets.
    auto slot_mem = [&](size_t slot) {
      std::array<float *, 6> m;
      float *p = w.smem + slot * (size_t)mem_set_len(c);
      for (int i = 0; i < 6; ++i) {
        m[i] = p;
        p += mem_len(c, i);
      }
      return m;
    };
    auto copy_mem = [&](float *const *dst, float *const *src) -> wfd_status {
      for (int i = 0; i < 6; ++i)
        HIP_TRY(hipMemcpyAsync(dst[i], src[i], (size_t)mem_len(c, i) * sizeof(float),
                               hipMemcpyDeviceToDevice, c->stream));
      return WFD_OK;
    };
    if (c->cpml)
      for (int i = 0; i < 6; ++i)
        if ((s = zero(c, w.amem[i], mem_len(c, i))) != WFD_OK) return s;
    for (size_t i = 0; i + 3 <= plan.size(); i += 3) {
      const int op = plan[i], a = plan[i + 1], b = plan[i + 2];
      if (op == wfd::kAdvance) {
        if (cur_state != a) {
          if (a == 0) {  // the zero initial state, in two scratch buffers
            cur = free_buffer(-1, -1);
            prev = free_buffer(cur, -1);
            if (cur < 0 || prev < 0) return fail(WFD_E_STATE, "checkpoint pool exhausted");
            if ((s = zero(c, buf[cur], c->vol)) != WFD_OK) return s;
            if ((s = zero(c, buf[prev], c->vol)) != WFD_OK) return s;
            if (c->cpml)
              for (int i = 0; i < 6; ++i)
                if ((s = zero(c, w.mem[i], mem_len(c, i))) != WFD_OK) return s;
          } else {
            Slot *sl = slot_of(a);
            if (!sl) return fail(WFD_E_STATE, "checkpoint plan: state %d not stored", a);
            cur = sl->a;
            prev = sl->b;
            if (c->cpml && (s = copy_mem(w.mem, slot_mem((size_t)(sl - slots.data())).data())) !=
                               WFD_OK)
              return s;
          }
        }
        for (int n = a; n < b; ++n) {
          int out = pins[prev] == 0 ? prev : free_buffer(cur, prev);
          if (out < 0) return fail(WFD_E_STATE, "checkpoint pool exhausted");
          if ((s = fwd(buf[cur], buf[prev], buf[out], n, n >= reached)) != WFD_OK) return s;
          if (n >= reached) reached = n + 1;
          prev = cur;
          cur = out;
        }
        cur_state = b;
      } else if (op == wfd::kStore) {
        if (cur_state != a) return fail(WFD_E_STATE, "checkpoint plan: store of non-current state");
        Slot &sl = slots[(size_t)b];
        sl.state = a;
        sl.a = cur;
        sl.b = prev;
        ++pins[cur];
        ++pins[prev];
        if (c->cpml && (s = copy_mem(slot_mem((size_t)b).data(), w.mem)) != WFD_OK) return s;
      } else if (op == wfd::kVisit) {
        if ((s = residual()) != WFD_OK) return s;
        const float *wm = nullptr;
        if (cur_state == a)
          wm = buf[cur];
        else if (Slot *sl = slot_of(a))
          wm = buf[sl->a];
        else if (cur_state == a + 1)
          wm = buf[prev];
        if (!wm) return fail(WFD_E_STATE, "checkpoint plan: state %d unavailable", a);
        const float *corr = nullptr;
        if (c->cpml && a < nt) {
          // C^a comes from the step that leaves state a: the latest forward
          // step, or recomputed from state a and its memory variables (the
          // visit is the state's last use, so they may be overwritten)
          if (last_c_step == a) {
            corr = w.lastc;
          } else if (cur_state == a) {
            if ((s = cpml_forward_terms(c, g, w, buf[cur], nullptr, w.visitc, 0, a)) != WFD_OK)
              return s;
            corr = w.visitc;
          } else if (Slot *sl = slot_of(a)) {
            const auto m = slot_mem((size_t)(sl - slots.data()));
            if ((s = cpml_forward_terms(c, g, w, buf[sl->a], nullptr, w.visitc, 0, a,
                                        m.data())) != WFD_OK)
              return s;
            corr = w.visitc;
          } else {
            return fail(WFD_E_STATE, "checkpoint plan: the layer's correction of step %d is lost",
                        a);
          }
        }
        if ((s = adjoint(a, wm, corr)) != WFD_OK) return s;
      } else if (op == wfd::kFree) {
        Slot &sl = slots[(size_t)b];
        --pins[sl.a];
        --pins[sl.b];
        sl = Slot{};
      }
    }
  }
  {
    Timed t(c, WFD_K_OTHER);
    HIP_TRY(wfd::launch_grad_fold(w.g, c->k, c->pitch, c->Ny, c->grid.border, c->grid.nx,
                                  c->grid.ny, c->grid.nz, c->grid.dt, w.scale, out_exp2, grad,
                                  c->stream));
  }
  return WFD_OK;
}

wfd_status wfd_gradient_finish(wfd_ctx *c, float *grad, int32_t zero_top_planes) {
  if (!c) return fail(WFD_E_ARG, "ctx is NULL");
  if (!c->has_model) return fail(WFD_E_STATE, "no model: call wfd_set_model first");
  if (!grad) return fail(WFD_E_ARG, "gradient is NULL");
  if (zero_top_planes < 0 || zero_top_planes > c->grid.nz)
    return fail(WFD_E_ARG, "zero_top_planes must be in [0, nz]");
  if (zero_top_planes == 0) return WFD_OK;
  ScopedDevice sd(c->device);
  return zero(c, grad, (int64_t)zero_top_planes * c->grid.ny * c->grid.nx);
}

wfd_status wfd_set_tuning(wfd_ctx *c, const wfd_tuning *t) {
  if (!c || !t) return fail(WFD_E_ARG, "NULL argument");
  if (t->fwd_variant < 0 || t->fwd_variant >= wfd::kFwdVariants)
    return fail(WFD_E_ARG, "forward tile variant must be in [0, %d)", wfd::kFwdVariants);
  if (t->adj_variant < 0 || t->adj_variant >= wfd::kAdjVariants)
    return fail(WFD_E_ARG, "adjoint tile variant must be in [0, %d)", wfd::kAdjVariants);
  if (t->fwd_rounds < 0 || t->fwd_rounds > 64 || t->adj_rounds < 0 || t->adj_rounds > 64)
    return fail(WFD_E_ARG, "rounds must be in [0, 64]");
  c->tuning = wfd::Tuning{t->fwd_variant, t->fwd_rounds, t->adj_variant, t->adj_rounds};
  return WFD_OK;
}

wfd_status wfd_get_tuning(const wfd_ctx *c, wfd_tuning *t) {
  if (!c || !t) return fail(WFD_E_ARG, "NULL argument");
  *t = wfd_tuning{c->tuning.variant, c->tuning.rounds, c->tuning.adj_variant,
                  c->tuning.adj_rounds};
  return WFD_OK;
}


wfd_status wfd_autotune(wfd_ctx *c, int32_t steps, void *work, size_t work_bytes,
                        wfd_tuning *best, double *us_per_step) {
  if (!c) return fail(WFD_E_ARG, "ctx is NULL");
  if (!c->has_model) return fail(WFD_E_STATE, "no model: call wfd_set_model first");
  if (steps < 1) return fail(WFD_E_ARG, "steps must be >= 1");
  if (!work) return fail(WFD_E_ARG, "workspace is NULL");
  if ((uintptr_t)work % kAlign) return fail(WFD_E_ARG, "workspace must be 256-byte aligned");
  wfd_ckpt one{};  // one stored pair, no host store
  one.mode = WFD_CKPT_REVOLVE;
  one.n_snapshots = 1;
  Work w = work_layout(c, 0, WorkKind::Gradient, &one, 1, work);
  if (work_bytes < w.bytes)
    return fail(WFD_E_NOMEM, "workspace has %zu bytes, %zu needed", work_bytes, w.bytes);
  ScopedDevice sd(c->device);
  wfd_status s;
  for (float *v : {w.W1, w.W2, w.P1, w.P2, w.g})
    if ((s = zero(c, v, c->vol)) != WFD_OK) return s;
  // an empty receiver table: every column starts (and ends) at entry 0
  if ((s = zero(c, reinterpret_cast<float *>(w.col_start), (int64_t)c->Nx * c->Ny + 1)) !=
      WFD_OK)
    return s;
  const wfd::StepGrid g = step_grid(c);
  const wfd::RecTable rt = rec_table(w, 0);
  // index -1 matches no point: nothing is injected (the pointers stay valid)
  const wfd::Source none_src{-1, &w.scale->sigma, &w.scale->sigma};
  hipEvent_t e0, e1;
  HIP_TRY(hipEventCreate(&e0));
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return fail(WFD_E_HIP, "hipEventCreate failed");
  }
  const int rounds_opts[] = {0, 2, 3, 4, 6, 8};
  wfd::Tuning bt = c->tuning;
  float best_f = 3.0e38f, best_a = 3.0e38f;
  hipError_t err = hipSuccess;
  for (int v = 0; v < wfd::kFwdVariants && err == hipSuccess; ++v)
    for (int r : rounds_opts) {
      wfd::Tuning tu = bt;
      tu.variant = v;
      tu.rounds = r;
      float *cur = w.W1, *prev = w.W2;
      float ms = 0.0f;
      err = time_steps(c, steps, e0, e1, [&] {
        hipError_t e = wfd::launch_forward_step(g, cur, prev, prev, none_src, 0, nullptr, nullptr,
                                                nullptr, tu, c->stream);
        std::swap(cur, prev);
        return e;
      }, &ms);
      if (err != hipSuccess) break;
      if (ms < best_f) {
        best_f = ms;
        bt.variant = v;
        bt.rounds = r;
      }
    }
  for (int v = 0; v < wfd::kAdjVariants && err == hipSuccess; ++v)
    for (int r : rounds_opts) {
      wfd::Tuning tu = bt;
      tu.adj_variant = v;
      tu.adj_rounds = r;
      float *a1 = w.P1, *a2 = w.P2;
      float ms = 0.0f;
      err = time_steps(c, steps, e0, e1, [&] {
        hipError_t e = wfd::launch_adjoint_step(tu, g, a1, a2, a2, rt, w.seis_tm, 1, w.W1, w.g,
                                                wfd::IllumOut{}, c->stream);
        std::swap(a1, a2);
        return e;
      }, &ms);
      if (err != hipSuccess) break;
      if (ms < best_a) {
        best_a = ms;
        bt.adj_variant = v;
        bt.adj_rounds = r;
      }
    }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (err != hipSuccess) return fail(WFD_E_HIP, "autotune: %s", hipGetErrorString(err));
  c->tuning = bt;
  if (best) *best = wfd_tuning{bt.variant, bt.rounds, bt.adj_variant, bt.adj_rounds};
  if (us_per_step) {
    us_per_step[0] = 1e3 * (double)best_f;
    us_per_step[1] = 1e3 * (double)best_a;
  }
  return WFD_OK;
}

wfd_status wfd_batch_create(wfd_batch **out, int32_t nshot, wfd_ctx *const *ctxs,
                            const float *wavelet, const double *src_xyz, const int32_t *nrec,
                            const double *const *rec_xyz, float *const *seis,
                            void *const *work, const size_t *work_bytes) {
  if (!out) return fail(WFD_E_ARG, "batch pointer is NULL");
  *out = nullptr;
  if (nshot < 1 || nshot > kMaxBatch)
    return fail(WFD_E_ARG, "batch size must be in [1, %d] (got %d)", kMaxBatch, nshot);
  if (!ctxs || !src_xyz || !nrec || !work || !work_bytes || !wavelet)
    return fail(WFD_E_ARG, "NULL argument");
  wfd_ctx *c0 = ctxs[0];
  for (int i = 0; i < nshot; ++i) {
    wfd_ctx *c = ctxs[i];
    if (!c || !c->has_model) return fail(WFD_E_STATE, "shot %d: context without a model", i);
    if (c->device != c0->device) return fail(WFD_E_ARG, "shot %d: other device", i);
    if (c->stream != c0->stream) return fail(WFD_E_ARG, "shot %d: contexts must share one stream", i);
    if (c->grid.nt != c0->grid.nt) return fail(WFD_E_ARG, "shot %d: nt differs", i);
    if (c->vd != c0->vd) return fail(WFD_E_ARG, "shot %d: density mode differs", i);
    if (c->cpml) return fail(WFD_E_ARG, "shot %d: batches take sponge boundaries only", i);
    if (nrec[i] < 0 || (nrec[i] > 0 && (!rec_xyz || !rec_xyz[i] || !seis || !seis[i])))
      return fail(WFD_E_ARG, "shot %d: receivers / output missing", i);
    if (!work[i] || (uintptr_t)work[i] % kAlign)
      return fail(WFD_E_ARG, "shot %d: workspace NULL or not 256-byte aligned", i);
    for (int j = 0; j < i; ++j)
      if (ctxs[j] == c) return fail(WFD_E_ARG, "shot %d: context used twice", i);
  }
  ScopedDevice sd(c0->device);
  wfd_batch *b = new (std::nothrow) wfd_batch();
  if (!b) return fail(WFD_E_NOMEM, "out of host memory");
  b->stream = c0->stream;
  b->nt = c0->grid.nt;
  b->vd = c0->vd;
  for (int i = 0; i < nshot; ++i) b->fs = b->fs || ctxs[i]->grid.free_surface != 0;
  b->variant = c0->tuning.variant;
  b->h_wins[0].resize(nshot);
  b->h_wins[1].resize(nshot);
  int offset = 0;
  for (int i = 0; i < nshot; ++i) {
    wfd_ctx *c = ctxs[i];
    Work w = work_layout(c, nrec[i], WorkKind::Forward, nullptr, 0, work[i]);
    if (work_bytes[i] < w.bytes) {
      delete b;
      return fail(WFD_E_NOMEM, "shot %d: workspace has %zu bytes, %zu needed", i, work_bytes[i],
                  w.bytes);
    }
    int64_t src_idx = 0;
    wfd_status s = prepare_shot(c, wavelet, src_xyz + 3 * (size_t)i, nrec[i],
                                nrec[i] > 0 ? rec_xyz[i] : nullptr, w, src_idx);
    if (s != WFD_OK) {
      delete b;
      return s;
    }
    if (i == 0) {
      b->d_wins[0] = w.wins;
      b->d_wins[1] = w.wins + kMaxBatch;
    }
    // Each window keeps the tile map of its own launch (z chunks sized for the
    // whole device, at least 16 planes deep when several shots share the
    // launch, 4 for a single shot); one launch then has a single tail instead
    // of one per shot.  Measured on 24 windows of 173-300 cells: sizing the
    // chunks for a 1/nshot share of the device instead makes full-depth
    // columns, whose last round leaves the device idle longer.
    wfd::Tuning tu = c->tuning;
    tu.variant = b->variant;  // one tile shape per launch
    wfd::WindowStep d{};
    d.g = step_grid(c);
    const int nb = wfd::forward_tile_map(
        d.g, tu, nshot == 1 ? wfd::kSingleMinZc : wfd::kBatchMinZc, &d.map);
    d.src = wfd::Source{src_idx, &w.scale->sigma, wavelet};
    d.rec = rec_table(w, nrec[i]);
    d.rec_scale = w.rec_scale;
    d.seis_tm = nrec[i] > 0 ? w.seis_tm : nullptr;
    d.block_begin = offset;
    d.block_end = offset + nb;
    offset += (nb + 7) / 8 * 8;
    for (int p = 0; p < 2; ++p) {
      wfd::WindowStep e = d;
      e.cur = p == 0 ? w.W1 : w.W2;
      e.prev = p == 0 ? w.W2 : w.W1;
      e.out = const_cast<float *>(e.prev);
      b->h_wins[p][i] = e;
    }
    b->ctxs.push_back(c);
    b->model_gen.push_back(c->model_gen);
    b->W1.push_back(w.W1);
    b->W2.push_back(w.W2);
    b->seis_tm.push_back(w.seis_tm);
    b->seis_out.push_back(nrec[i] > 0 ? seis[i] : nullptr);
    b->nrec.push_back(nrec[i]);
  }
  b->nblocks = offset;
  for (int p = 0; p < 2; ++p) {
    if (hipMemcpyAsync(b->d_wins[p], b->h_wins[p].data(), nshot * sizeof(wfd::WindowStep),
                       hipMemcpyHostToDevice, b->stream) != hipSuccess) {
      delete b;
      return fail(WFD_E_HIP, "descriptor upload failed");
    }
  }
  if (hipStreamSynchronize(b->stream) != hipSuccess) {  // host descriptors may go now
    delete b;
    return fail(WFD_E_HIP, "hipStreamSynchronize failed");
  }
  *out = b;
  return WFD_OK;
}

namespace {

wfd_status batch_enqueue(wfd_batch *b) {
  wfd_ctx *c0 = b->ctxs[0];
  const int nwin = (int)b->ctxs.size();
  for (int i = 0; i < nwin; ++i) {
    HIP_TRY(wfd::launch_fill_zero(b->W1[i], b->ctxs[i]->vol, b->stream));
    HIP_TRY(wfd::launch_fill_zero(b->W2[i], b->ctxs[i]->vol, b->stream));
  }
  for (int n = 0; n < b->nt; ++n) {
    Timed t(c0, WFD_K_FORWARD);
    HIP_TRY(wfd::launch_forward_multi(b->d_wins[n & 1], nwin, b->nblocks, n, b->variant, b->vd,
                                      b->fs, b->stream));
  }
  for (int i = 0; i < nwin; ++i)
    if (b->nrec[i] > 0)
      HIP_TRY(wfd::launch_transpose(b->seis_tm[i], b->seis_out[i], b->nrec[i], b->nt, b->stream));
  return WFD_OK;
}

}  // namespace

wfd_status wfd_batch_run(wfd_batch *b, int32_t use_graph) {
  if (!b) return fail(WFD_E_ARG, "batch is NULL");
  // the step descriptors (and a captured graph) hold the coefficient pointers
  // of each context's model at creation time
  for (size_t i = 0; i < b->ctxs.size(); ++i)
    if (!b->ctxs[i]->has_model || b->ctxs[i]->model_gen != b->model_gen[i])
      return fail(WFD_E_STATE, "shot %zu: the context's model changed after wfd_batch_create",
                  i);
  ScopedDevice sd(b->ctxs[0]->device);
  if (!use_graph) return batch_enqueue(b);
  if (!b->stream) return fail(WFD_E_ARG, "graph capture needs a non-default stream");
  if (b->ctxs[0]->prof) return fail(WFD_E_STATE, "profiling events cannot be captured");
  if (!b->exec) {
    HIP_TRY(hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
    wfd_status s = batch_enqueue(b);
    hipGraph_t graph = nullptr;
    const hipError_t e = hipStreamEndCapture(b->stream, &graph);
    if (s != WFD_OK) {
      if (graph) (void)hipGraphDestroy(graph);
      return s;
    }
    if (e != hipSuccess) return fail(WFD_E_HIP, "hipStreamEndCapture: %s", hipGetErrorString(e));
    b->graph = graph;
    HIP_TRY(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
  }
  HIP_TRY(hipGraphLaunch(b->exec, b->stream));
  return WFD_OK;
}

wfd_status wfd_batch_destroy(wfd_batch *b) {
  if (!b) return WFD_OK;
  ScopedDevice sd(b->ctxs[0]->device);
  if (b->exec || b->graph) (void)hipStreamSynchronize(b->stream);
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  delete b;
  return WFD_OK;
}

// A batch of shots whose whole gradients (Alg. 3 body) run together: every
// forward and adjoint step is one launch over the tiles of every shot, with
// binomial checkpointing on one plan shared by all shots.
struct wfd_gbatch {
  std::vector<wfd_ctx *> ctxs;
  std::vector<uint64_t> model_gen;
  std::vector<Work> work;
  std::vector<int> nrec;
  std::vector<const float *> dobs;
  std::vector<double *> misfit;
  std::vector<float *> grad;
  std::vector<int32_t> plan;
  wfd::GradWindow *d_wins = nullptr;  // in shot 0's workspace
  int fblocks = 0, ablocks = 0, variant = 0, adj_variant = 0, nt = 0, nsnap = 0;
  bool vd = false, fs = false, illum = false;
  hipStream_t stream = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

wfd_status wfd_gbatch_create(wfd_gbatch **out, int32_t nshot, wfd_ctx *const *ctxs,
                             const float *wavelet, const double *src_xyz, const int32_t *nrec,
                             const double *const *rec_xyz, const float *const *dobs,
                             int32_t n_snapshots, double *const *misfit_dev,
                             float *const *grad_dev, float *const *illum_dev_or_null,
                             void *const *work_dev, const size_t *work_bytes) {
  if (!out) return fail(WFD_E_ARG, "batch pointer is NULL");
  *out = nullptr;
  if (nshot < 1 || nshot > kMaxBatch)
    return fail(WFD_E_ARG, "batch size must be in [1, %d] (got %d)", kMaxBatch, nshot);
  if (!ctxs || !src_xyz || !nrec || !work_dev || !work_bytes || !wavelet || !misfit_dev ||
      !grad_dev)
    return fail(WFD_E_ARG, "NULL argument");
  if (n_snapshots < 1) return fail(WFD_E_ARG, "n_snapshots must be >= 1");
  wfd_ctx *c0 = ctxs[0];
  const bool illum = illum_dev_or_null && illum_dev_or_null[0];
  for (int i = 0; i < nshot; ++i) {
    wfd_ctx *c = ctxs[i];
    if (!c || !c->has_model) return fail(WFD_E_STATE, "shot %d: context without a model", i);
    if (c->device != c0->device) return fail(WFD_E_ARG, "shot %d: other device", i);
    if (c->stream != c0->stream) return fail(WFD_E_ARG, "shot %d: contexts must share one stream", i);
    if (c->grid.nt != c0->grid.nt) return fail(WFD_E_ARG, "shot %d: nt differs", i);
    if (c->vd != c0->vd) return fail(WFD_E_ARG, "shot %d: density mode differs", i);
    if (c->cpml) return fail(WFD_E_ARG, "shot %d: batches take sponge boundaries only", i);
    if (nrec[i] < 0 || (nrec[i] > 0 && (!rec_xyz || !rec_xyz[i] || !dobs || !dobs[i])))
      return fail(WFD_E_ARG, "shot %d: receivers / observed data missing", i);
    if (!misfit_dev[i] || !grad_dev[i]) return fail(WFD_E_ARG, "shot %d: misfit / gradient output is NULL", i);
    if (illum != (illum_dev_or_null && illum_dev_or_null[i]))
      return fail(WFD_E_ARG, "shot %d: illumination outputs must be given for all shots or none", i);
    if (!work_dev[i] || (uintptr_t)work_dev[i] % kAlign)
      return fail(WFD_E_ARG, "shot %d: workspace NULL or not 256-byte aligned", i);
    for (int j = 0; j < i; ++j)
      if (ctxs[j] == c) return fail(WFD_E_ARG, "shot %d: context used twice", i);
  }
  ScopedDevice sd(c0->device);
  wfd_gbatch *b = new (std::nothrow) wfd_gbatch();
  if (!b) return fail(WFD_E_NOMEM, "out of host memory");
  b->stream = c0->stream;
  b->nt = c0->grid.nt;
  b->nsnap = n_snapshots;
  b->vd = c0->vd;
  b->illum = illum;
  b->variant = c0->tuning.variant;
  b->adj_variant = c0->tuning.adj_variant;
  for (int i = 0; i < nshot; ++i) b->fs = b->fs || ctxs[i]->grid.free_surface != 0;
  int64_t nsteps = 0;
  wfd::build_checkpoint_plan(b->nt, n_snapshots, b->plan, nsteps);
  wfd_ckpt ck{};
  ck.mode = WFD_CKPT_REVOLVE;
  ck.n_snapshots = n_snapshots;
  std::vector<wfd::GradWindow> h((size_t)nshot);
  int foff = 0, aoff = 0;
  for (int i = 0; i < nshot; ++i) {
    wfd_ctx *c = ctxs[i];
    Work w = work_layout(c, nrec[i], WorkKind::Gradient, &ck, n_snapshots, work_dev[i]);
    if (work_bytes[i] < w.bytes) {
      delete b;
      return fail(WFD_E_NOMEM, "shot %d: workspace has %zu bytes, %zu needed", i, work_bytes[i],
                  w.bytes);
    }
    int64_t src_idx = 0;
    wfd_status s = prepare_shot(c, wavelet, src_xyz + 3 * (size_t)i, nrec[i],
                                nrec[i] > 0 ? rec_xyz[i] : nullptr, w, src_idx);
    if (s != WFD_OK) {
      delete b;
      return s;
    }
    wfd::Tuning tu = c->tuning;
    tu.variant = b->variant;  // one tile shape per launch
    tu.adj_variant = b->adj_variant;
    wfd::GradWindow &d = h[(size_t)i];
    d.g = step_grid(c);
    const int min_zc = nshot == 1 ? wfd::kSingleMinZc : wfd::kBatchMinZc;
    const int nf = wfd::forward_tile_map(d.g, tu, min_zc, &d.fmap);
    const int na = wfd::adjoint_tile_map(d.g, tu, illum, min_zc, &d.amap);
    d.src = wfd::Source{src_idx, &w.scale->sigma, wavelet};
    d.rec = rec_table(w, nrec[i]);
    d.rec_scale = w.rec_scale;
    d.seis_tm = w.seis_tm;
    d.res_tm = w.res_tm;
    d.W1 = w.W1;
    d.W2 = w.W2;
    d.store = w.store;
    d.vol = c->vol;
    d.P1 = w.P1;
    d.P2 = w.P2;
    d.gimg = w.g;
    d.il = wfd::IllumOut{illum ? illum_dev_or_null[i] : nullptr, c->grid.border, c->grid.nx,
                         c->grid.ny, c->grid.nz, w.scale, 0};
    d.fblock_begin = foff;
    d.fblock_end = foff + nf;
    d.ablock_begin = aoff;
    d.ablock_end = aoff + na;
    foff += (nf + 7) / 8 * 8;  // ranges start at multiples of 8: XCD-aware order
    aoff += (na + 7) / 8 * 8;
    b->ctxs.push_back(c);
    b->model_gen.push_back(c->model_gen);
    b->work.push_back(w);
    b->nrec.push_back(nrec[i]);
    b->dobs.push_back(nrec[i] > 0 ? dobs[i] : nullptr);
    b->misfit.push_back(misfit_dev[i]);
    b->grad.push_back(grad_dev[i]);
  }
  b->fblocks = foff;
  b->ablocks = aoff;
  b->d_wins = b->work[0].gwins;
  if (hipMemcpyAsync(b->d_wins, h.data(), (size_t)nshot * sizeof(wfd::GradWindow),
                     hipMemcpyHostToDevice, b->stream) != hipSuccess ||
      hipStreamSynchronize(b->stream) != hipSuccess) {  // the host descriptors may go now
    delete b;
    return fail(WFD_E_HIP, "descriptor upload failed");
  }
  *out = b;
  return WFD_OK;
}

namespace {

// The whole batched gradient on the stream: clears, the shared checkpoint plan
// (one launch per forward step and per adjoint step over every shot's
// tiles), residuals and misfits after the forward sweep, then the fold.
wfd_status gbatch_enqueue(wfd_gbatch *b) {
  wfd_ctx *c0 = b->ctxs[0];
  const int nwin = (int)b->ctxs.size();
  const int nt = b->nt;
  hipStream_t st = b->stream;
  auto pool = [&](int i, int k) -> float * {
    const Work &w = b->work[(size_t)i];
    return k == 0 ? w.W1 : (k == 1 ? w.W2 : w.store + (size_t)(k - 2) * (size_t)b->ctxs[i]->vol);
  };
  for (int i = 0; i < nwin; ++i) {
    const Work &w = b->work[(size_t)i];
    for (float *p : {w.W1, w.W2, w.P1, w.P2, w.g})
      HIP_TRY(wfd::launch_fill_zero(p, b->ctxs[i]->vol, st));
  }
  const int nbuf = 2 + 2 * b->nsnap;
  std::vector<int> pins((size_t)nbuf, 0);
  struct Slot {
    int state = -1, a = -1, b = -1;
  };
  std::vector<Slot> slots((size_t)b->nsnap);
  int cur_state = -1, cur = -1, prev = -1, reached = 0, parity = 0;
  bool residual_done = false;
  auto slot_of = [&](int state) -> Slot * {
    for (auto &sl : slots)
      if (sl.state == state) return &sl;
    return nullptr;
  };
  auto free_buffer = [&](int not1, int not2) -> int {
    for (int i = 0; i < nbuf; ++i)
      if (pins[(size_t)i] == 0 && i != not1 && i != not2) return i;
    return -1;
  };
  for (size_t i = 0; i + 3 <= b->plan.size(); i += 3) {
    const int op = b->plan[i], a = b->plan[i + 1], bb = b->plan[i + 2];
    if (op == wfd::kAdvance) {
      if (cur_state != a) {
        if (a == 0) {
          cur = free_buffer(-1, -1);
          prev = free_buffer(cur, -1);
          if (cur < 0 || prev < 0) return fail(WFD_E_STATE, "checkpoint pool exhausted");
          for (int s = 0; s < nwin; ++s) {
            HIP_TRY(wfd::launch_fill_zero(pool(s, cur), b->ctxs[s]->vol, st));
            HIP_TRY(wfd::launch_fill_zero(pool(s, prev), b->ctxs[s]->vol, st));
          }
        } else {
          Slot *sl = slot_of(a);
          if (!sl) return fail(WFD_E_STATE, "checkpoint plan: state %d not stored", a);
          cur = sl->a;
          prev = sl->b;
        }
      }
      for (int n = a; n < bb; ++n) {
        const int o = pins[(size_t)prev] == 0 ? prev : free_buffer(cur, prev);
        if (o < 0) return fail(WFD_E_STATE, "checkpoint pool exhausted");
        {
          Timed t(c0, WFD_K_FORWARD);
          HIP_TRY(wfd::launch_forward_pool(b->d_wins, nwin, b->fblocks, n, cur, prev, o,
                                           n >= reached ? 1 : 0, b->variant, b->vd, b->fs, st));
        }
        if (n >= reached) reached = n + 1;
        prev = cur;
        cur = o;
      }
      cur_state = bb;
    } else if (op == wfd::kStore) {
      if (cur_state != a) return fail(WFD_E_STATE, "checkpoint plan: store of non-current state");
      Slot &sl = slots[(size_t)bb];
      sl.state = a;
      sl.a = cur;
      sl.b = prev;
      ++pins[(size_t)cur];
      ++pins[(size_t)prev];
    } else if (op == wfd::kVisit) {
      if (!residual_done) {
        residual_done = true;
        for (int s = 0; s < nwin; ++s) {
          if (b->nrec[(size_t)s] == 0) continue;
          const Work &w = b->work[(size_t)s];
          int np = 0;
          Timed t(c0, WFD_K_OTHER);
          HIP_TRY(wfd::launch_residual(w.seis_tm, b->dobs[(size_t)s], w.rec_adj, w.scale,
                                       b->nrec[(size_t)s], nt, w.res_tm, w.partial, &np, st));
          HIP_TRY(wfd::launch_sum_partials(w.partial, np, b->misfit[(size_t)s], st));
        }
      }
      int wk = -1;
      if (cur_state == a)
        wk = cur;
      else if (Slot *sl = slot_of(a))
        wk = sl->a;
      else if (cur_state == a + 1)
        wk = prev;
      if (wk < 0) return fail(WFD_E_STATE, "checkpoint plan: state %d unavailable", a);
      {
        Timed t(c0, WFD_K_ADJOINT);
        HIP_TRY(wfd::launch_adjoint_multi(b->d_wins, nwin, b->ablocks, a, parity, wk,
                                          b->adj_variant, b->vd, b->illum, b->fs, st));
      }
      parity ^= 1;
    } else if (op == wfd::kFree) {
      Slot &sl = slots[(size_t)bb];
      --pins[(size_t)sl.a];
      --pins[(size_t)sl.b];
      sl = Slot{};
    }
  }
  for (int s = 0; s < nwin; ++s) {
    wfd_ctx *c = b->ctxs[(size_t)s];
    const Work &w = b->work[(size_t)s];
    Timed t(c0, WFD_K_OTHER);
    HIP_TRY(wfd::launch_grad_fold(w.g, c->k, c->pitch, c->Ny, c->grid.border, c->grid.nx,
                                  c->grid.ny, c->grid.nz, c->grid.dt, w.scale, 0,
                                  b->grad[(size_t)s], st));
  }
  return WFD_OK;
}

}  // namespace

wfd_status wfd_gbatch_run(wfd_gbatch *b, int32_t use_graph) {
  if (!b) return fail(WFD_E_ARG, "batch is NULL");
  for (size_t i = 0; i < b->ctxs.size(); ++i)
    if (!b->ctxs[i]->has_model || b->ctxs[i]->model_gen != b->model_gen[i])
      return fail(WFD_E_STATE, "shot %zu: the context's model changed after wfd_gbatch_create",
                  i);
  ScopedDevice sd(b->ctxs[0]->device);
  if (!use_graph) return gbatch_enqueue(b);
  if (!b->stream) return fail(WFD_E_ARG, "graph capture needs a non-default stream");
  if (b->ctxs[0]->prof) return fail(WFD_E_STATE, "profiling events cannot be captured");
  if (!b->exec) {
    HIP_TRY(hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
    wfd_status s = gbatch_enqueue(b);
    hipGraph_t graph = nullptr;
    const hipError_t e = hipStreamEndCapture(b->stream, &graph);
    if (s != WFD_OK) {
      if (graph) (void)hipGraphDestroy(graph);
      return s;
    }
    if (e != hipSuccess) return fail(WFD_E_HIP, "hipStreamEndCapture: %s", hipGetErrorString(e));
    b->graph = graph;
    HIP_TRY(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
  }
  HIP_TRY(hipGraphLaunch(b->exec, b->stream));
  return WFD_OK;
}

wfd_status wfd_gbatch_destroy(wfd_gbatch *b) {
  if (!b) return WFD_OK;
  ScopedDevice sd(b->ctxs[0]->device);
  if (b->exec || b->graph) (void)hipStreamSynchronize(b->stream);
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  delete b;
  return WFD_OK;
}


wfd_status wfd_map_position(const wfd_grid *grid, const double xyz[3], int32_t ijk[3]) {
  wfd_status s = check_grid(grid);
  if (s != WFD_OK) return s;
  if (!xyz || !ijk) return fail(WFD_E_ARG, "NULL argument");
  if (!wfd::map_position(*grid, xyz, ijk))
    return fail(WFD_E_RANGE, "position (%g, %g, %g) is outside the model", xyz[0], xyz[1], xyz[2]);
  return WFD_OK;
}

wfd_status wfd_cfl_ratio(const wfd_grid *grid, double vmax, double m2max, double *ratio) {
  wfd_status s = check_grid(grid);
  if (s != WFD_OK) return s;
  if (!ratio) return fail(WFD_E_ARG, "ratio is NULL");
  *ratio = wfd::cfl_ratio(*grid, vmax, m2max);
  return WFD_OK;
}

wfd_status wfd_checkpoint_plan(int32_t nt, int32_t n_snapshots, int32_t *actions,
                               int64_t capacity, int64_t *n_actions, int64_t *n_forward_steps) {
  if (nt < 1) return fail(WFD_E_ARG, "nt must be >= 1");
  if (n_snapshots < 1) return fail(WFD_E_ARG, "n_snapshots must be >= 1");
  if (!n_actions || !n_forward_steps) return fail(WFD_E_ARG, "NULL argument");
  std::vector<int32_t> plan;
  int64_t steps = 0;
  wfd::build_checkpoint_plan(nt, n_snapshots, plan, steps);
  *n_actions = (int64_t)plan.size() / 3;
  *n_forward_steps = steps;
  if (actions) {
    if (capacity < *n_actions) return fail(WFD_E_NOMEM, "action buffer too small");
    std::memcpy(actions, plan.data(), plan.size() * sizeof(int32_t));
  }
  return WFD_OK;
}

wfd_status wfd_set_profiling(wfd_ctx *c, int32_t enable) {
  if (!c) return fail(WFD_E_ARG, "ctx is NULL");
  ScopedDevice sd(c->device);
  if (enable) {
    wfd_status s = drain_profile(c);
    if (s != WFD_OK) return s;
    for (int i = 0; i < WFD_K_COUNT; ++i) {
      c->launches[i] = 0;
      c->ms[i] = 0.0;
    }
  }
  c->prof = enable != 0;
  return WFD_OK;
}

wfd_status wfd_kernel_stats(wfd_ctx *c, int32_t kernel_class, int64_t *launches, double *total_ms) {
  if (!c || !launches || !total_ms) return fail(WFD_E_ARG, "NULL argument");
  if (kernel_class < 0 || kernel_class >= WFD_K_COUNT)
    return fail(WFD_E_ARG, "unknown kernel class %d", kernel_class);
  ScopedDevice sd(c->device);
  wfd_status s = drain_profile(c);
  if (s != WFD_OK) return s;
  *launches = c->launches[kernel_class];
  *total_ms = c->ms[kernel_class];
  return WFD_OK;
}

// ---- learned gradient preconditioner ---------------------------------------

wfd_status wfd_cnn_packed_elems(int32_t cin, int32_t cout, int32_t flip, int64_t *elems) {
  if (!elems) return fail(WFD_E_ARG, "NULL argument");
  const bool layer = (cin == 2 && cout == 16) || (cin == 16 && cout == 16) ||
                     (cin == 16 && cout == 1);
  if (!layer || (flip != 0 && flip != 1))
    return fail(WFD_E_ARG, "no network layer %d -> %d (flip %d)", cin, cout, flip);
  const int rows_in = flip ? cout : cin;
  *elems = 16LL * ((27 * rows_in + 31) / 32 * 32);
  return WFD_OK;
}

wfd_status wfd_cnn_pack_weights(const float *w, int32_t cin, int32_t cout, int32_t flip,
                                uint16_t *apk, void *stream) {
  int64_t n = 0;
  wfd_status s = wfd_cnn_packed_elems(cin, cout, flip, &n);
  if (s != WFD_OK) return s;
  if (!w || !apk) return fail(WFD_E_ARG, "NULL argument");
  HIP_TRY(wfd::launch_pack_weights(w, cin, cout, flip, apk, (hipStream_t)stream));
  return WFD_OK;
}

namespace {
// The CNN kernels tile a volume into 64 x 4 x 16-voxel marches and index
// tiles with 32-bit integers: the tile count must stay below 2^31.
bool cnn_volume_ok(int32_t nx, int32_t ny, int32_t nz) {
  if (nx < 1 || ny < 1 || nz < 1) return false;
  const int64_t a = ((int64_t)nx + 63) / 64, b = ((int64_t)ny + 3) / 4, c = ((int64_t)nz + 15) / 16;
  return a * b <= INT32_MAX && a * b * c <= INT32_MAX;
}
}  // namespace

wfd_status wfd_cnn_conv(const uint16_t *in, int32_t nx, int32_t ny, int32_t nz, int32_t cin,
                        int32_t cout, const uint16_t *apk, const float *bias, int32_t relu,
                        const uint16_t *mask, const uint16_t *residual, int32_t residual_channels,
                        uint16_t *out_bf16, float *out_f32, void *stream) {
  const bool shape = (cin == 2 && cout == 16) || (cin == 16 && cout == 16) ||
                     (cin == 16 && cout == 1) || (cin == 1 && cout == 16);
  if (!shape) return fail(WFD_E_ARG, "no convolution %d -> %d channels", cin, cout);
  if (!cnn_volume_ok(nx, ny, nz))
    return fail(WFD_E_ARG, "volume %d x %d x %d empty or too large", nx, ny, nz);
  if ((int64_t)nx * ny > (int64_t(1) << 24))
    return fail(WFD_E_ARG, "an x-y plane of %d x %d voxels exceeds 2^24", nx, ny);
  if (!in || !apk) return fail(WFD_E_ARG, "NULL input or weights");
  if (mask && cout == 16 && (uintptr_t)mask % 8)
    return fail(WFD_E_ARG, "a 16-channel mask must be 8-byte aligned");
  if (!out_bf16 && !out_f32) return fail(WFD_E_ARG, "no output");
  if (residual && (cout != 1 || residual_channels < 1 || residual_channels > 16))
    return fail(WFD_E_ARG, "a residual needs a single-output convolution and 1 to 16 channels");
  if ((uintptr_t)in % 16 || (uintptr_t)apk % 16 || (uintptr_t)out_bf16 % 16 ||
      (uintptr_t)out_f32 % 16)
    return fail(WFD_E_ARG, "buffers must be 16-byte aligned");
  HIP_TRY(wfd::launch_conv(cin, cout, in, nx, ny, nz, apk, bias, relu, mask, residual,
                           residual_channels, out_bf16, out_f32, (hipStream_t)stream));
  return WFD_OK;
}

wfd_status wfd_cnn_wgrad_workspace_bytes(int32_t nx, int32_t ny, int32_t nz, size_t *bytes) {
  if (!bytes) return fail(WFD_E_ARG, "NULL argument");
  if (!cnn_volume_ok(nx, ny, nz))
    return fail(WFD_E_ARG, "volume %d x %d x %d empty or too large", nx, ny, nz);
  *bytes = wfd::cnn_wgrad_workspace_floats(nx, ny, nz) * sizeof(float);
  return WFD_OK;
}

wfd_status wfd_cnn_wgrad(const uint16_t *in, const uint16_t *dz, int32_t nx, int32_t ny,
                         int32_t nz, int32_t cin, int32_t cout, float *dw, float *db,
                         void *work, size_t work_bytes, void *stream) {
  const bool layer = (cin == 2 && cout == 16) || (cin == 16 && cout == 16) ||
                     (cin == 16 && cout == 1);
  if (!layer) return fail(WFD_E_ARG, "no network layer %d -> %d", cin, cout);
  if (!cnn_volume_ok(nx, ny, nz))
    return fail(WFD_E_ARG, "volume %d x %d x %d empty or too large", nx, ny, nz);
  if ((int64_t)nx * ny > (int64_t(1) << 24))
    return fail(WFD_E_ARG, "an x-y plane of %d x %d voxels exceeds 2^24", nx, ny);
  if (!in || !dz || !dw || !work) return fail(WFD_E_ARG, "NULL argument");
  if ((uintptr_t)in % 16) return fail(WFD_E_ARG, "input must be 16-byte aligned");
  if (cout == 16 && (uintptr_t)dz % 16)
    return fail(WFD_E_ARG, "a 16-channel output gradient must be 16-byte aligned");
  const size_t need = wfd::cnn_wgrad_workspace_floats(nx, ny, nz) * sizeof(float);
  if (work_bytes < need)
    return fail(WFD_E_NOMEM, "workspace has %zu bytes, %zu needed", work_bytes, need);
  HIP_TRY(wfd::launch_wgrad(cin, cout, in, dz, nx, ny, nz, static_cast<float *>(work), dw, db,
                            (hipStream_t)stream));
  return WFD_OK;
}

wfd_status wfd_cnn_mse(const float *y, const float *t, int64_t n, uint16_t *dy, double *loss,
                       void *work, size_t work_bytes, void *stream) {
  if (!y || !t || !dy || !loss || !work) return fail(WFD_E_ARG, "NULL argument");
  if (n < 1) return fail(WFD_E_ARG, "n must be >= 1");
  if (work_bytes < WFD_CNN_REDUCE_BYTES)
    return fail(WFD_E_NOMEM, "workspace must hold %d bytes", WFD_CNN_REDUCE_BYTES);
  HIP_TRY(wfd::launch_mse(y, t, n, dy, static_cast<double *>(work), wfd::kCnnReduceBlocks, loss,
                          (hipStream_t)stream));
  return WFD_OK;
}

wfd_status wfd_cnn_adam(float *w, const float *g, float *m, float *v, int32_t n, float lr,
                        float beta1, float beta2, float eps, int32_t step, void *stream) {
  if (!w || !g || !m || !v) return fail(WFD_E_ARG, "NULL argument");
  if (n < 1 || step < 1) return fail(WFD_E_ARG, "n and step must be >= 1");
  if (!(lr > 0.0f) || !(beta1 >= 0.0f && beta1 < 1.0f) || !(beta2 >= 0.0f && beta2 < 1.0f))
    return fail(WFD_E_ARG, "bad Adam hyper-parameters");
  HIP_TRY(wfd::launch_adam(w, g, m, v, n, lr, beta1, beta2, eps, step, (hipStream_t)stream));
  return WFD_OK;
}

wfd_status wfd_cnn_pack_input(const float *grad, const float *illum, int64_t n, float eps,
                              uint16_t *out, void *work, size_t work_bytes, void *stream) {
  if (!grad || !illum || !out || !work) return fail(WFD_E_ARG, "NULL argument");
  if (n < 1) return fail(WFD_E_ARG, "n must be >= 1");
  if (!(eps > 0.0f)) return fail(WFD_E_ARG, "eps must be > 0");
  if (work_bytes < WFD_CNN_REDUCE_BYTES)
    return fail(WFD_E_NOMEM, "workspace must hold %d bytes", WFD_CNN_REDUCE_BYTES);
  HIP_TRY(wfd::launch_pack_input(grad, illum, n, eps, static_cast<float *>(work),
                                 wfd::kCnnReduceBlocks, out, (hipStream_t)stream));
  return WFD_OK;
}

// ---- gradient smoothing ------------------------------------------------------

namespace {
constexpr int kSmoothPartials = 512;

size_t smooth_bytes(int mode, int nx, int ny, int nz) {
  const size_t vol = (size_t)nx * ny * nz;
  if (mode == WFD_SMOOTH_LAPLACE) return align_up(2 * (size_t)(nx + ny + nz) * sizeof(double));
  return align_up(3 * vol * sizeof(float)) + align_up(kSmoothPartials * sizeof(double));
}

double sum_partials_host(const double *dev, std::vector<double> &host, hipStream_t s,
                         hipError_t &err) {
  err = hipMemcpyAsync(host.data(), dev, host.size() * sizeof(double), hipMemcpyDeviceToHost, s);
  if (err == hipSuccess) err = hipStreamSynchronize(s);
  double t = 0.0;
  for (double v : host) t += v;
  return t;
}
}  // namespace

wfd_status wfd_smooth_workspace_bytes(int32_t mode, int32_t nx, int32_t ny, int32_t nz,
                                      size_t *bytes) {
  if (!bytes) return fail(WFD_E_ARG, "NULL argument");
  if (mode != WFD_SMOOTH_LAPLACE && mode != WFD_SMOOTH_BESSEL)
    return fail(WFD_E_ARG, "unknown smoothing mode %d", mode);
  if (nx < 1 || ny < 1 || nz < 1) return fail(WFD_E_ARG, "empty volume");
  *bytes = smooth_bytes(mode, nx, ny, nz);
  return WFD_OK;
}

wfd_status wfd_smooth(int32_t mode, const float *in, float *out, int32_t nx, int32_t ny,
                      int32_t nz, const double lengths[3], const double spacing[3], double tol,
                      int32_t max_iter, void *work, size_t work_bytes, int32_t *iterations,
                      void *stream_) {
  if (mode != WFD_SMOOTH_LAPLACE && mode != WFD_SMOOTH_BESSEL)
    return fail(WFD_E_ARG, "unknown smoothing mode %d", mode);
  if (!in || !out || !lengths || !spacing || !work) return fail(WFD_E_ARG, "NULL argument");
  if (nx < 1 || ny < 1 || nz < 1) return fail(WFD_E_ARG, "empty volume");
  for (int d = 0; d < 3; ++d) {
    if (!(lengths[d] >= 0.0) || !std::isfinite(lengths[d]))
      return fail(WFD_E_ARG, "lengths must be finite and >= 0");
    if (!(spacing[d] > 0.0) || !std::isfinite(spacing[d]))
      return fail(WFD_E_ARG, "spacing must be finite and > 0");
  }
  const size_t need = smooth_bytes(mode, nx, ny, nz);
  if (work_bytes < need)
    return fail(WFD_E_NOMEM, "workspace has %zu bytes, %zu needed", work_bytes, need);
  hipStream_t st = (hipStream_t)stream_;
  const int64_t n = (int64_t)nx * ny * nz;
  if (mode == WFD_SMOOTH_LAPLACE) {
    if (out != in) HIP_TRY(hipMemcpyAsync(out, in, n * sizeof(float), hipMemcpyDeviceToDevice, st));
    const int len[3] = {nx, ny, nz};
    const int64_t lines[3] = {(int64_t)ny * nz, (int64_t)nx * nz, (int64_t)nx * ny};
    double *dev = static_cast<double *>(work);
    std::vector<double> host(2 * (size_t)(nx + ny + nz), 0.0);
    size_t off = 0;
    double a_of[3];
    size_t off_of[3];
    for (int d = 0; d < 3; ++d) {
      const int m = len[d];
      const double a = lengths[d] > 0.0 ? std::exp(-spacing[d] / lengths[d]) : 0.0;
      a_of[d] = a;
      off_of[d] = off;
      double *cp = host.data() + off, *inv = host.data() + off + m;
      for (int i = 0; i < m; ++i) {
        double b = 1.0 + a * a;
        if (m == 1) b = (1.0 - a) * (1.0 - a);
        else if (i == 0 || i == m - 1) b = 1.0 + a * a - a;  // zero-flux ends
        const double den = i == 0 ? b : b + a * cp[i - 1];
        inv[i] = 1.0 / den;
        cp[i] = -a / den;
      }
      off += 2 * (size_t)m;
    }
    HIP_TRY(hipMemcpyAsync(dev, host.data(), host.size() * sizeof(double), hipMemcpyHostToDevice,
                           st));
    for (int d = 0; d < 3; ++d) {
      if (lengths[d] <= 0.0) continue;
      const double a = a_of[d];
      HIP_TRY(wfd::launch_tri_lines(out, d, len[d], lines[d], nx, ny, dev + off_of[d],
                                    dev + off_of[d] + len[d], a, (1.0 - a) * (1.0 - a), st));
    }
    HIP_TRY(hipStreamSynchronize(st));  // the host coefficients may go now
    if (iterations) *iterations = 0;
    return WFD_OK;
  }
  // Bessel: conjugate gradients on B u = g from u = 0
  if (out == in) return fail(WFD_E_ARG, "the Bessel filter needs out != in");
  if (max_iter < 1) return fail(WFD_E_ARG, "max_iter must be >= 1");
  if (!(tol > 0.0)) return fail(WFD_E_ARG, "tol must be > 0");
  char *base = static_cast<char *>(work);
  float *r = reinterpret_cast<float *>(base);
  float *p = r + n;
  float *ap = p + n;
  double *part = reinterpret_cast<double *>(base + align_up(3 * (size_t)n * sizeof(float)));
  const float cx = (float)(lengths[0] * lengths[0] / (spacing[0] * spacing[0]));
  const float cy = (float)(lengths[1] * lengths[1] / (spacing[1] * spacing[1]));
  const float cz = (float)(lengths[2] * lengths[2] / (spacing[2] * spacing[2]));
  std::vector<double> hp(kSmoothPartials);
  hipError_t e = hipSuccess;
  HIP_TRY(wfd::launch_cg_start(in, r, out, n, part, kSmoothPartials, st));
  const double gg = sum_partials_host(part, hp, st, e);
  if (e != hipSuccess) return fail(WFD_E_HIP, "smoothing: %s", hipGetErrorString(e));
  if (iterations) *iterations = 0;
  if (gg == 0.0) return WFD_OK;
  HIP_TRY(wfd::launch_cg_direction(p, r, n, 0.0f, kSmoothPartials, st));
  double rr = gg;
  int it = 0;
  while (it < max_iter && rr > tol * tol * gg) {
    HIP_TRY(wfd::launch_bessel_apply(p, ap, nx, ny, nz, cx, cy, cz, part, kSmoothPartials, st));
    const double pap = sum_partials_host(part, hp, st, e);
    if (e != hipSuccess) return fail(WFD_E_HIP, "smoothing: %s", hipGetErrorString(e));
    const double alpha = rr / pap;
    HIP_TRY(wfd::launch_cg_update(out, r, p, ap, n, (float)alpha, part, kSmoothPartials, st));
    const double rr_new = sum_partials_host(part, hp, st, e);
    if (e != hipSuccess) return fail(WFD_E_HIP, "smoothing: %s", hipGetErrorString(e));
    ++it;
    if (rr_new <= tol * tol * gg) {
      rr = rr_new;
      break;
    }
    HIP_TRY(wfd::launch_cg_direction(p, r, n, (float)(rr_new / rr), kSmoothPartials, st));
    rr = rr_new;
  }
  if (iterations) *iterations = it;
  if (rr > tol * tol * gg)
    return fail(WFD_E_RANGE, "smoothing: no convergence in %d iterations (residual %.3g)", it,
                std::sqrt(rr / gg));
  return WFD_OK;
}

wfd_status wfd_resample(int32_t mode, const float *in, int32_t nrec, int32_t nt_in, double dt_in,
                        float *out, int32_t nt_out, double dt_out, void *stream) {
  if (mode != WFD_RESAMPLE_NEAREST && mode != WFD_RESAMPLE_SINC)
    return fail(WFD_E_ARG, "unknown resampling mode %d", mode);
  if (nrec < 0 || nt_in < 1 || nt_out < 1) return fail(WFD_E_ARG, "bad trace sizes");
  if (!(dt_in > 0.0) || !(dt_out > 0.0) || !std::isfinite(dt_in) || !std::isfinite(dt_out))
    return fail(WFD_E_ARG, "sample steps must be finite and > 0");
  if (nrec == 0) return WFD_OK;
  if (!in || !out) return fail(WFD_E_ARG, "NULL argument");
  if (in == out) return fail(WFD_E_ARG, "in and out must differ");
  HIP_TRY(wfd::launch_resample(in, nrec, nt_in, dt_in, out, nt_out, dt_out,
                               mode == WFD_RESAMPLE_SINC, (hipStream_t)stream));
  return WFD_OK;
}

}  // extern "C"



