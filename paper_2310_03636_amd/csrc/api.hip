// C ABI of the spin-1 split-step library: validation, workspace layout,
// shell index tables, and the host-side order of the passes.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>

#include <algorithm>
#include <cmath>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "spin1.h"
#include "internal.hpp"

using namespace spin1;

namespace {

thread_local std::string g_err = "no error";

int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

int hip_fail(hipError_t e, const char* what) {
  return fail(SPIN1_EHIP, "%s: %s", what, hipGetErrorString(e));
}

bool is_pow2(int64_t v) { return v > 0 && (v & (v - 1)) == 0; }

}  // namespace

// ---------------------------------------------------------------------------
// Static scratch of spin1_observables_noalloc: partial sums in a device array
// of the library itself, so that the call needs no workspace region and
// allocates nothing.  Each device holds its own copy (from the load of the
// code object until the process ends).  Host code uses the address that
// hipGetSymbolAddress returns per device, never the array's name.
// ---------------------------------------------------------------------------
static constexpr size_t kNoAllocScratchBytes = size_t(32) << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace {

constexpr int kMaxDevices = 64;

std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};
hipError_t g_scratch_err[kMaxDevices] = {};

// Once per device, with that device current (spin1_create): the device
// address of its copy of the scratch array.
void scratch_setup(int dev) {
  if (dev < 0 || dev >= kMaxDevices) return;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[dev]) return;
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e == hipSuccess && ptr) {
    g_scratch_ptr[dev] = ptr;
    g_scratch_err[dev] = hipSuccess;
  } else {
    g_scratch_err[dev] = e != hipSuccess ? e : hipErrorInvalidSymbol;
  }
}

// the scratch address of device dev, or null with *err set
void* scratch_of(int dev, hipError_t* err) {
  if (dev < 0 || dev >= kMaxDevices) {
    *err = hipErrorInvalidDevice;
    return nullptr;
  }
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  *err = g_scratch_ptr[dev] ? hipSuccess : g_scratch_err[dev];
  if (*err == hipSuccess && !g_scratch_ptr[dev]) *err = hipErrorNotInitialized;
  return g_scratch_ptr[dev];
}

size_t align_up(size_t v) { return (v + 255) & ~size_t(255); }

int validate_grid(const spin1_grid* g, int32_t dtype) {
  if (!g) return fail(SPIN1_EINVAL, "grid pointer is NULL");
  if (dtype != SPIN1_C64 && dtype != SPIN1_C128) return fail(SPIN1_EINVAL, "dtype %d is not SPIN1_C64/SPIN1_C128", dtype);
  if (g->dim < 1 || g->dim > 3) return fail(SPIN1_EINVAL, "dim must be 1, 2 or 3 (got %d)", g->dim);
  if (!(g->dx > 0.0) || !isfinite(g->dx)) return fail(SPIN1_EINVAL, "dx must be finite and > 0");
  if (g->samples < 1) return fail(SPIN1_EINVAL, "samples must be >= 1 (got %d)", g->samples);
  for (int a = 0; a < 3; ++a) {
    const int n = g->n[a];
    if (a >= g->dim) {
      if (n != 1) return fail(SPIN1_EINVAL, "n[%d] must be 1 for a %d-dimensional grid (got %d)", a, g->dim, n);
      continue;
    }
    if (!is_pow2(n)) return fail(SPIN1_EINVAL, "n[%d] = %d is not a power of two", a, n);
    if (n < 8) return fail(SPIN1_EINVAL, "n[%d] = %d is below the minimum 8", a, n);
    if (a == 0) {
      if (n > 4096) return fail(SPIN1_EUNSUPPORTED, "Nx = %d exceeds 4096", n);
      if (g->dim > 1 && n < 16) return fail(SPIN1_EUNSUPPORTED, "Nx = %d: 2D/3D grids need Nx >= 16", n);
    } else if (n > 1024) {
      return fail(SPIN1_EUNSUPPORTED, "n[%d] = %d: strided axes support at most 1024 points", a, n);
    }
  }
  const int64_t sites = int64_t(g->n[0]) * g->n[1] * g->n[2];
  if (sites * g->samples * 3 > (int64_t(1) << 40)) return fail(SPIN1_EUNSUPPORTED, "field too large");
  // one component of one sample is addressed with 32-bit byte offsets inside a pass
  if (sites * (dtype == SPIN1_C128 ? 16 : 8) >= (int64_t(1) << 32))
    return fail(SPIN1_EUNSUPPORTED, "one component of one sample exceeds 4 GiB");
  return SPIN1_OK;
}

Geom geom_of(const spin1_grid* g) {
  Geom r;
  r.dim = g->dim;
  for (int a = 0; a < 3; ++a) r.n[a] = g->n[a];
  r.dx = g->dx;
  r.S = g->samples;
  r.sites = int64_t(g->n[0]) * g->n[1] * g->n[2];
  r.rows = r.sites / g->n[0];
  return r;
}

double cell_of(const Geom& g) {
  double c = 1.0;
  for (int a = 0; a < g.dim; ++a) c *= g.dx;
  return c;
}

int64_t isqrt64(int64_t v) {
  int64_t s = int64_t(sqrt(double(v)));
  while (s > 0 && s * s > v) --s;
  while ((s + 1) * (s + 1) <= v) ++s;
  return s;
}

// shell of integer |j'|^2 = J: the b with 4J < (2b+1)^2 and (2b-1)^2 <= 4J for b >= 1
int shell_of(int64_t J) { return int((isqrt64(4 * J) + 1) / 2); }

int nmax_of(const Geom& g) {
  int m = 1;
  for (int a = 0; a < g.dim; ++a) m = std::max(m, g.n[a]);
  return m;
}

int64_t mode_J(const Geom& g, int64_t site) {
  const int nm = nmax_of(g);
  int64_t J = 0;
  int64_t rest = site;
  for (int a = 0; a < g.dim; ++a) {
    const int n = g.n[a];
    const int64_t j = rest % n;
    rest /= n;
    const int64_t js = (j < n / 2 ? j : j - n) * (nm / n);
    J += js * js;
  }
  return J;
}

int num_bins_of(const Geom& g) {
  const int64_t h = nmax_of(g) / 2;
  return shell_of(int64_t(g.dim) * h * h) + 1;
}

struct Layout {
  size_t ph[3] = {0, 0, 0}, tw[3] = {0, 0, 0}, part[3] = {0, 0, 0};
  int64_t nblk[3] = {0, 0, 0};  // partial entries (y, z: one per workgroup)
  size_t sff = 0, pow = 0, perm = 0, offs = 0, end = 0;
};

// spass geometry for axis a (1 = y, 2 = z)
void spass_geom(const Geom& g, int a, int64_t* sa, int64_t* inner, int64_t* outer, int64_t* outer_stride) {
  const int64_t nx = g.n[0], ny = g.n[1];
  if (a == 1) {
    *sa = nx;
    *inner = nx;
    *outer = g.dim == 3 ? g.n[2] : 1;
    *outer_stride = nx * ny;
  } else {
    *sa = nx * ny;
    *inner = nx * ny;
    *outer = 1;
    *outer_stride = 0;
  }
}

size_t layout_group(const Geom& g, bool dbl, size_t base, Layout* L) {
  const size_t cb = dbl ? 16 : 8, rb = dbl ? 8 : 4;
  const size_t tb = 16;  // table entry: complex128, or hi + lo complex64
  size_t off = base;
  for (int a = 0; a < g.dim; ++a) {
    L->ph[a] = off;
    off = align_up(off + size_t(a == 0 ? 3 : 1) * g.n[a] * tb);
    L->tw[a] = off;
    off = align_up(off + size_t(g.n[a]) * tb);
  }
  L->part[0] = off;
  off = align_up(off + size_t(g.S) * g.rows * 4 * sizeof(double));
  for (int a = 1; a < g.dim; ++a) {
    int64_t sa, inner, outer, os;
    spass_geom(g, a, &sa, &inner, &outer, &os);
    const int tx = spass_tx(g.n[a], dbl);
    L->nblk[a] = int64_t(3) * g.S * outer * (inner / tx);
    L->part[a] = off;
    off = align_up(off + size_t(L->nblk[a]) * sizeof(double));
  }
  L->sff = off;  // complex spectrum scratch (also the reverse-mode seed in 1D)
  off = align_up(off + size_t(g.S) * g.sites * cb);
  L->pow = off;
  off = align_up(off + size_t(g.S) * g.sites * rb);
  L->perm = off;
  off = align_up(off + size_t(g.sites) * sizeof(int32_t));
  L->offs = off;
  off = align_up(off + size_t(num_bins_of(g) + 1) * sizeof(int32_t));
  L->end = off;
  return off;
}

struct GroupState {
  spin1_grid grid;
  Geom geo;
  void* psi;
  Layout lay;
  int nbins;
  const double* pot = nullptr;  // trap potential [sites] (borrowed), or null
};

}  // namespace

struct ProfRecord {
  int kind;
  hipEvent_t start, stop;
};

struct GraphEntry {
  int64_t n;
  double dt;
  uint64_t version;
  uint64_t last_use;
  hipGraphExec_t exec;
};
constexpr size_t kMaxGraphs = 8;

struct spin1_ctx {
  int dtype = SPIN1_C64;
  bool dbl = false;
  hipStream_t stream = nullptr;
  int device = 0;
  bool bound = false;
  spin1_params p{};
  std::vector<GroupState> groups;
  char* ws = nullptr;
  bool tab_valid = false;
  double tab_dt = 0.0, tab_q = 0.0;
  // profiling
  bool prof = false;
  std::vector<hipEvent_t> ev_pool;  // created events, reused
  std::vector<ProfRecord> rec;      // records since the last read
  size_t ev_used = 0;
  // captured step sequences: (steps, dt) of the current binding and couplings
  bool use_graphs = true;
  int64_t graph_max_steps = 1024;
  int steps_per_launch_1d = 0;  // 0: automatic (see spin1.h)
  bool grouped_x = false;
  int kernel_1d = 0;  // 0 automatic, 1 one thread group per sample, 2 component groups
  int scheme = SPIN1_SCHEME_STRANG;
  bool dithered_tables = true;  // FP32 streaming passes: dithered float tables
  int stores = SPIN1_STORES_AUTO;  // field stores of the streaming step passes
  // groups outside the grouped x-pass run on streams of their own (default
  // priority), forked from and joined back into the caller's stream per call
  bool concurrent = true;
  static constexpr int kSideStreams = 3;  // with the caller's: four hardware queues
  hipStream_t side[kSideStreams] = {};
  hipEvent_t join_ev[kSideStreams] = {};
  hipEvent_t fork_ev = nullptr;
  uint64_t version = 0;  // bumped whenever a captured graph could go stale
  uint64_t use_clock = 0;
  std::vector<GraphEntry> graphs;
  // step-pass variants chosen by the autotuner: [pass 0 = x, 1 = strided][double][log2 N]
  int8_t variant[2][2][13] = {};
  void drop_graphs() {
    for (GraphEntry& g : graphs) (void)hipGraphExecDestroy(g.exec);
    graphs.clear();
  }
  ~spin1_ctx() {
    drop_graphs();
    for (hipEvent_t e : ev_pool) (void)hipEventDestroy(e);
    if (fork_ev) (void)hipEventDestroy(fork_ev);
    for (int i = 0; i < kSideStreams; ++i) {
      if (join_ev[i]) (void)hipEventDestroy(join_ev[i]);
      if (side[i]) (void)hipStreamDestroy(side[i]);
    }
  }
};

LaunchTiming& spin1::launch_timing() {
  static thread_local LaunchTiming lt;
  return lt;
}

namespace {

int check_ctx(spin1_ctx* ctx, bool need_bound) {
  if (!ctx) return fail(SPIN1_EINVAL, "context is NULL");
  if (need_bound && !ctx->bound) return fail(SPIN1_ESTATE, "no field bound: call spin1_bind or spin1_init_wigner first");
  return SPIN1_OK;
}

int validate_params(const spin1_params* p) {
  if (!p) return fail(SPIN1_EINVAL, "params pointer is NULL");
  const double v[5] = {p->c0, p->c1, p->q, p->n0, p->wigner_var};
  for (double x : v)
    if (!isfinite(x)) return fail(SPIN1_EINVAL, "params must be finite");
  if (p->n0 < 0.0) return fail(SPIN1_EINVAL, "n0 must be >= 0");
  if (p->wigner_var < 0.0) return fail(SPIN1_EINVAL, "wigner_var must be >= 0");
  return SPIN1_OK;
}

char* at(spin1_ctx* ctx, size_t off) { return ctx->ws + off; }

hipEvent_t next_event(spin1_ctx* ctx) {
  if (ctx->ev_used == ctx->ev_pool.size()) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    ctx->ev_pool.push_back(e);
  }
  return ctx->ev_pool[ctx->ev_used++];
}

// Times the launches of its scope when profiling is on.  A scope with one
// kernel launch is timed by the kernel's own begin and end (the events handed
// to launch_kernel); a scope with several by events recorded on the stream
// before and after it.  ONE: the scope launches exactly one kernel (the step
// passes), so no events go on the stream, which keeps the profiled steps'
// launch gaps close to those of unprofiled ones.
struct Prof {
  spin1_ctx* ctx;
  int kind;
  bool one;
  hipEvent_t a = nullptr, b = nullptr, ka = nullptr, kb = nullptr;
  int64_t first = 0;
  bool on = false, nested = false;
  LaunchTiming outer;
  Prof(spin1_ctx* c, int k, bool one_launch = false) : ctx(c), kind(k), one(one_launch) {
    if (!ctx->prof) return;
    // inside another scope (not done today) this one is timed on the stream,
    // and the outer scope's launch events are put back at its end
    if (launch_timing().start) {
      one = false;
      a = next_event(ctx);
      b = next_event(ctx);
      if (!a || !b) return;
      on = true;
      nested = true;
      outer = launch_timing();
      launch_timing().start = launch_timing().stop = nullptr;
      (void)hipEventRecord(a, ctx->stream);
      return;
    }
    ka = next_event(ctx);
    kb = next_event(ctx);
    if (!one) {
      a = next_event(ctx);
      b = next_event(ctx);
    }
    if (!ka || !kb || (!one && (!a || !b))) return;
    on = true;
    if (!one) (void)hipEventRecord(a, ctx->stream);
    LaunchTiming& lt = launch_timing();
    lt.start = ka;
    lt.stop = kb;
    first = lt.launches;
  }
  ~Prof() {
    if (!on) return;
    if (nested) {
      (void)hipEventRecord(b, ctx->stream);
      ctx->rec.push_back(ProfRecord{kind, a, b});
      launch_timing().start = outer.start;
      launch_timing().stop = outer.stop;
      return;
    }
    LaunchTiming& lt = launch_timing();
    const int64_t n = lt.launches - first;
    lt.start = lt.stop = nullptr;  // unused when the scope launched nothing
    if (!one) (void)hipEventRecord(b, ctx->stream);
    if (n == 1)
      ctx->rec.push_back(ProfRecord{kind, ka, kb});
    else if (n > 1 && !one)
      ctx->rec.push_back(ProfRecord{kind, a, b});
  }
};

int make_tables(spin1_ctx* ctx, double dt) {
  for (auto& G : ctx->groups) {
    for (int a = 0; a < G.geo.dim; ++a) {
      Prof pr(ctx, SPIN1_K_OTHER);
      const hipError_t e = launch_tables(ctx->stream, ctx->dbl, at(ctx, G.lay.ph[a]), at(ctx, G.lay.tw[a]), G.geo.n[a],
                                         a == 0 ? 3 : 1, dt, ctx->p.q, G.geo.dx);
      if (e != hipSuccess) return hip_fail(e, "table kernel");
    }
  }
  ctx->tab_valid = true;
  ctx->tab_dt = dt;
  ctx->tab_q = ctx->p.q;
  return SPIN1_OK;
}

int upload_shells(spin1_ctx* ctx, GroupState& G) {
  const Geom& g = G.geo;
  const int nb = G.nbins;
  std::vector<int32_t> offs(size_t(nb) + 1, 0), perm;
  std::vector<int32_t> shell;
  try {
    perm.resize(size_t(g.sites));
    shell.resize(size_t(g.sites));
  } catch (const std::bad_alloc&) {
    return fail(SPIN1_ENOMEM, "host allocation of shell tables failed");
  }
  for (int64_t s = 0; s < g.sites; ++s) {
    const int b = shell_of(mode_J(g, s));
    shell[size_t(s)] = b;
    offs[size_t(b) + 1]++;
  }
  for (int b = 0; b < nb; ++b) offs[size_t(b) + 1] += offs[size_t(b)];
  std::vector<int32_t> fill(offs.begin(), offs.end() - 1);
  for (int64_t s = 0; s < g.sites; ++s) perm[size_t(fill[size_t(shell[size_t(s)])]++)] = int32_t(s);
  hipError_t e = hipMemcpy(at(ctx, G.lay.perm), perm.data(), perm.size() * sizeof(int32_t), hipMemcpyHostToDevice);
  if (e != hipSuccess) return hip_fail(e, "upload of shell permutation");
  e = hipMemcpy(at(ctx, G.lay.offs), offs.data(), offs.size() * sizeof(int32_t), hipMemcpyHostToDevice);
  if (e != hipSuccess) return hip_fail(e, "upload of shell offsets");
  return SPIN1_OK;
}

// Non-temporal field stores in the streaming step passes: forced by the
// option, else when the bound fields together exceed 512 MiB (complex64) or
// 768 MiB (complex128).  Measured on 2D 512^2 batches (MI355X, 256 MB
// last-level cache), split-step time with non-temporal against ordinary
// stores: complex64 +3 to +4% up to 64 samples (403 MB: the next pass reads
// part of the field from the cache), +1.2% at 80 (503 MB), level at 96
// (604 MB), -3 to -5% from 128 (805 MB) to 384 samples (2.4 GB); complex128
// +3% up to 48 samples (604 MB), level to +3% at 64 (805 MB), -1.4 to -2.2%
// from 96 (1.2 GB) to 192 samples (2.4 GB).
constexpr double kStreamingStoreBytesC64 = double(size_t(512) << 20);
constexpr double kStreamingStoreBytesC128 = double(size_t(768) << 20);
bool streaming_stores(const spin1_ctx* ctx) {
  if (ctx->stores != SPIN1_STORES_AUTO) return ctx->stores == SPIN1_STORES_STREAMING;
  double bytes = 0.0;
  for (const GroupState& G : ctx->groups)
    bytes += 3.0 * double(G.geo.S) * double(G.geo.sites) * (ctx->dbl ? 16.0 : 8.0);
  return bytes > (ctx->dbl ? kStreamingStoreBytesC128 : kStreamingStoreBytesC64);
}

XPassArgs xargs(spin1_ctx* ctx, const GroupState& G) {
  XPassArgs a{};
  a.nt = streaming_stores(ctx) ? 1 : 0;
  a.psi = G.psi;
  a.pot = G.pot;
  a.tw = at(ctx, G.lay.tw[0]);
  a.ph = at(ctx, G.lay.ph[0]);
  a.rows = G.geo.rows;
  a.sites = G.geo.sites;
  a.S = G.geo.S;
  a.c0 = ctx->p.c0;
  a.c1 = ctx->p.c1;
  a.q = ctx->p.q;
  a.kscale = 2.0 * M_PI / (double(G.geo.n[0]) * G.geo.dx);
  a.power_scale = 1.0 / double(G.geo.sites);
  return a;
}

SPassArgs sargs(spin1_ctx* ctx, const GroupState& G, int axis, void* field, int64_t nfield) {
  SPassArgs a{};
  a.nt = streaming_stores(ctx) ? 1 : 0;
  a.psi = field;
  a.tw = at(ctx, G.lay.tw[axis]);
  a.ph = at(ctx, G.lay.ph[axis]);
  spass_geom(G.geo, axis, &a.sa, &a.inner, &a.outer, &a.outer_stride);
  a.nfield = nfield;
  a.field_stride = G.geo.sites;
  a.kscale = 2.0 * M_PI / (double(G.geo.n[axis]) * G.geo.dx);
  a.power_scale = 1.0 / double(G.geo.sites);
  return a;
}

// The passes of step i of an n-step sequence of dt on one field: step 0 opens
// with R(dt/2), later steps merge the previous closing half with their own
// opening half into R(dt); the last step closes with R(dt/2) (x-pass epilogue
// in 1D, k_local otherwise).  tau_open = tau_close = 0 gives the kinetic +
// Zeeman passes alone, which the reverse sweep applies to the adjoint field.
int log2_of(int n) {
  int r = 0;
  while ((1 << (r + 1)) <= n) ++r;
  return r;
}

int twiddle_offset(const spin1_ctx* ctx) { return ctx->dithered_tables && !ctx->dbl ? kPlainTwiddles : 0; }

int variant_of(spin1_ctx* ctx, int pass, int n) {
  return ctx->variant[pass][ctx->dbl ? 1 : 0][log2_of(n)] + twiddle_offset(ctx);
}

// Direction of the streaming step pass with index k in the sequence of passes
// (dim per step): every other pass walks its work items backwards, so that it
// starts on the data the pass before it wrote last (still in the last-level
// cache).
int pass_reverse(int64_t k) { return int(k & 1); }

// the passes of a step after the x-pass: y/z passes, closing half step (2D/3D);
// step: index of the step in the call (sets the pass directions)
int enqueue_group_rest(spin1_ctx* ctx, const GroupState& G, void* field, double tau_close, int64_t step = 0) {
  hipError_t e;
  for (int a = 1; a < G.geo.dim; ++a) {
    SPassArgs sa = sargs(ctx, G, a, field, int64_t(3) * G.geo.S);
    sa.reverse = pass_reverse(step * G.geo.dim + a);
    sa.tick = step;
    {
      Prof pr(ctx, a == 1 ? SPIN1_K_YPASS : SPIN1_K_ZPASS, true);
      e = launch_spass(ctx->stream, ctx->dbl, MODE_STEP, G.geo.n[a], sa, variant_of(ctx, 1, G.geo.n[a]));
    }
    if (e != hipSuccess) return hip_fail(e, a == 1 ? "y-pass" : "z-pass");
  }
  if (G.geo.dim > 1 && tau_close != 0.0) {
    {
      Prof pr(ctx, SPIN1_K_LOCAL, true);
      e = launch_local(ctx->stream, ctx->dbl, field, G.geo.S, G.geo.sites, tau_close, ctx->p.c0, ctx->p.c1, G.pot);
    }
    if (e != hipSuccess) return hip_fail(e, "closing local update");
  }
  return SPIN1_OK;
}

// one step of group G on field (read from src instead when src is given: out of
// place); step: index of the step in the call (sets the pass directions)
int enqueue_group_step(spin1_ctx* ctx, const GroupState& G, void* field, double tau_open, double tau_close,
                       const void* src = nullptr, int64_t step = 0) {
  XPassArgs xa = xargs(ctx, G);
  xa.psi = field;
  xa.src = src;
  xa.reverse = pass_reverse(step * G.geo.dim);
  xa.tick = step;
  xa.tau_pre = tau_open;
  xa.tau_post = G.geo.dim == 1 ? tau_close : 0.0;
  hipError_t e;
  {
    Prof pr(ctx, SPIN1_K_XPASS, true);
    e = launch_xpass(ctx->stream, ctx->dbl, MODE_STEP, G.geo.n[0], xa, variant_of(ctx, 0, G.geo.n[0]));
  }
  if (e != hipSuccess) return hip_fail(e, "x-pass");
  return enqueue_group_rest(ctx, G, field, tau_close, step);
}

// 1D groups with more than one step per launch: consecutive chunks of up to
// steps_per_launch_1d steps, the first opening with R(dt/2), the last closing
// with R(dt/2), exactly the sequence of the per-step passes.
int steps_per_launch(const spin1_ctx* ctx, const GroupState& G) {
  if (G.geo.dim != 1 || G.pot) return 1;  // the multi-step kernels take no trap potential
  if (ctx->steps_per_launch_1d > 0) return ctx->steps_per_launch_1d;
  return 64;
}

bool multi_1d(const spin1_ctx* ctx, const GroupState& G) { return steps_per_launch(ctx, G) > 1; }

// The component-group form of the 1D multi-step kernel unless chosen
// otherwise (it was faster at every measured size and sample count; where its
// LDS does not fit, Nx = 4096, the launcher takes the pencil form, which holds
// a sample in the registers of 512 threads).
bool split_1d(const spin1_ctx* ctx, const GroupState&) { return ctx->kernel_1d != 1; }

int enqueue_group_multi(spin1_ctx* ctx, const GroupState& G, int64_t n, double dt) {
  XPassArgs xa = xargs(ctx, G);
  const int per = steps_per_launch(ctx, G);
  for (int64_t i0 = 0; i0 < n; i0 += per) {
    const int k = int(n - i0 < per ? n - i0 : per);
    hipError_t e;
    {
      Prof pr(ctx, SPIN1_K_XPASS, true);
      e = launch_x1d_multi(ctx->stream, ctx->dbl, G.geo.n[0], xa, k, dt, i0 == 0, i0 + k == n, split_1d(ctx, G));
    }
    if (e != hipSuccess) return hip_fail(e, "1D multi-step pass");
  }
  return SPIN1_OK;
}

// Groups whose step x-passes share one grouped launch: stepped one launch
// per step, pencil lengths the grouped kernel takes; at least two of them.
std::vector<size_t> grouped_x_set(const spin1_ctx* ctx) {
  std::vector<size_t> out;
  if (!ctx->grouped_x) return out;
  for (size_t g = 0; g < ctx->groups.size() && out.size() < size_t(kMaxGroupedX); ++g) {
    const GroupState& G = ctx->groups[g];
    if (!multi_1d(ctx, G) && !G.pot && G.geo.n[0] >= 16 && G.geo.n[0] <= grouped_x_max_n(ctx->dbl))
      out.push_back(g);
  }
  if (out.size() < 2) out.clear();
  return out;
}

int enqueue_grouped_x(spin1_ctx* ctx, const std::vector<size_t>& set, double tau_open, double tau_close,
                      int64_t step) {
  XGroupArgs ga{};
  int64_t items = 0;
  for (size_t j = 0; j < set.size(); ++j) {
    const GroupState& G = ctx->groups[set[j]];
    XGroupEntry& e = ga.g[j];
    e.psi = G.psi;
    e.tw = at(ctx, G.lay.tw[0]);
    e.ph = at(ctx, G.lay.ph[0]);
    e.rows = G.geo.rows;
    e.sites = G.geo.sites;
    e.pencils = int64_t(G.geo.S) * G.geo.rows;
    e.item_begin = items;
    e.tau_post = G.geo.dim == 1 ? tau_close : 0.0;
    e.n = G.geo.n[0];
    e.lg_rows = log2_of(int(G.geo.rows));
    items += grouped_x_items(e.n, e.pencils);
  }
  ga.item_end = items;
  ga.ngroups = int(set.size());
  ga.tau_pre = tau_open;
  ga.c0 = ctx->p.c0;
  ga.c1 = ctx->p.c1;
  ga.dither = twiddle_offset(ctx) != 0;
  ga.tick = step;
  hipError_t e;
  {
    Prof pr(ctx, SPIN1_K_XPASS, true);
    e = launch_xpass_grouped(ctx->stream, ctx->dbl, ga);
  }
  if (e != hipSuccess) return hip_fail(e, "grouped x-pass");
  return SPIN1_OK;
}

// The paper's Lie scheme, psi <- O D K psi per step (K without q): the D, O
// of step i run in the x-pass prologue of step i + 1 (2D/3D) or in the
// x-pass epilogue (1D); after the last step a local pass applies them.
int enqueue_steps_paper(spin1_ctx* ctx, int64_t n, double dt) {
  for (int64_t i = 0; i < n; ++i)
    for (auto& G : ctx->groups) {
      XPassArgs xa = xargs(ctx, G);
      xa.tau_pre = G.geo.dim > 1 && i > 0 ? dt : 0.0;
      xa.tau_post = G.geo.dim == 1 ? dt : 0.0;
      hipError_t e;
      {
        Prof pr(ctx, SPIN1_K_XPASS);
        e = launch_xpass(ctx->stream, ctx->dbl, MODE_PAPER, G.geo.n[0], xa);
      }
      if (e != hipSuccess) return hip_fail(e, "Lie-scheme x-pass");
      const int rc = enqueue_group_rest(ctx, G, G.psi, 0.0, i);
      if (rc) return rc;
      if (G.geo.dim > 1 && i == n - 1) {
        {
          Prof pr(ctx, SPIN1_K_LOCAL);
          e = launch_paper_local(ctx->stream, ctx->dbl, G.psi, G.geo.S, G.geo.sites, dt, ctx->p.c0, ctx->p.c1,
                                 ctx->p.q, G.pot);
        }
        if (e != hipSuccess) return hip_fail(e, "Lie-scheme local pass");
      }
    }
  return SPIN1_OK;
}

// The side streams and events, created on first use, all or nothing.
int ensure_side_streams(spin1_ctx* ctx) {
  if (ctx->side[0]) return SPIN1_OK;
  hipStream_t s[spin1_ctx::kSideStreams] = {};
  hipEvent_t j[spin1_ctx::kSideStreams] = {};
  hipEvent_t f = nullptr;
  hipError_t e = hipEventCreateWithFlags(&f, hipEventDisableTiming);
  for (int i = 0; i < spin1_ctx::kSideStreams && e == hipSuccess; ++i) {
    e = hipStreamCreateWithFlags(&s[i], hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&j[i], hipEventDisableTiming);
  }
  if (e != hipSuccess) {
    for (int i = 0; i < spin1_ctx::kSideStreams; ++i) {
      if (j[i]) (void)hipEventDestroy(j[i]);
      if (s[i]) (void)hipStreamDestroy(s[i]);
    }
    if (f) (void)hipEventDestroy(f);
    return hip_fail(e, "side streams");
  }
  for (int i = 0; i < spin1_ctx::kSideStreams; ++i) {
    ctx->side[i] = s[i];
    ctx->join_ev[i] = j[i];
  }
  ctx->fork_ev = f;
  return SPIN1_OK;
}

// All n steps of one group outside the grouped x-pass: multi-step 1D chunks,
// or one launch sequence per step.
int enqueue_group_steps(spin1_ctx* ctx, const GroupState& G, int64_t n, double dt) {
  if (multi_1d(ctx, G)) return enqueue_group_multi(ctx, G, n, dt);
  for (int64_t i = 0; i < n; ++i) {
    const int rc = enqueue_group_step(ctx, G, G.psi, i == 0 ? 0.5 * dt : dt, i == n - 1 ? 0.5 * dt : 0.0, nullptr, i);
    if (rc) return rc;
  }
  return SPIN1_OK;
}

// The steps of the grouped x-pass set: one grouped x-pass launch per step,
// then the other passes of each group in the set.
int enqueue_grouped_steps(spin1_ctx* ctx, const std::vector<size_t>& set, int64_t n, double dt) {
  for (int64_t i = 0; i < n && !set.empty(); ++i) {
    const double pre = i == 0 ? 0.5 * dt : dt;
    const double close = i == n - 1 ? 0.5 * dt : 0.0;
    int rc = enqueue_grouped_x(ctx, set, pre, close, i);
    for (size_t g : set)
      if (!rc) rc = enqueue_group_rest(ctx, ctx->groups[g], ctx->groups[g].psi, close, i);
    if (rc) return rc;
  }
  return SPIN1_OK;
}

// The independent sequences of a call: the grouped x-pass set (if any) and
// every other group.  Sequences share no data, so with concurrent groups each
// runs on a stream of its own (the caller's stream and up to three side
// streams, forked from and joined back into the caller's stream; round robin
// beyond four sequences), which lets the passes of small groups fill the GPU
// together.
int enqueue_steps(spin1_ctx* ctx, int64_t n, double dt) {
  if (ctx->scheme == SPIN1_SCHEME_PAPER) return enqueue_steps_paper(ctx, n, dt);
  const std::vector<size_t> set = grouped_x_set(ctx);
  std::vector<char> in_set(ctx->groups.size(), 0);
  for (size_t g : set) in_set[g] = 1;
  // sequence k: -1 = the grouped set, else a group index
  std::vector<int> seqs;
  if (!set.empty()) seqs.push_back(-1);
  for (size_t g = 0; g < ctx->groups.size(); ++g)
    if (!in_set[g]) seqs.push_back(int(g));
  auto enqueue_seq = [&](int q) {
    return q < 0 ? enqueue_grouped_steps(ctx, set, n, dt) : enqueue_group_steps(ctx, ctx->groups[size_t(q)], n, dt);
  };
  // side streams are not used while profiling (its events time the caller's
  // stream) or on the NULL stream
  const bool overlap = ctx->concurrent && seqs.size() > 1 && !ctx->prof && ctx->stream != nullptr;
  if (!overlap) {
    for (int q : seqs) {
      const int rc = enqueue_seq(q);
      if (rc) return rc;
    }
    return SPIN1_OK;
  }
  int rc = ensure_side_streams(ctx);
  if (rc) return rc;
  const int nside = int(std::min<size_t>(seqs.size() - 1, spin1_ctx::kSideStreams));
  hipError_t e = hipEventRecord(ctx->fork_ev, ctx->stream);
  for (int i = 0; i < nside && e == hipSuccess; ++i) e = hipStreamWaitEvent(ctx->side[i], ctx->fork_ev, 0);
  if (e != hipSuccess) return hip_fail(e, "stream fork");
  hipStream_t main = ctx->stream;
  for (size_t k = 0; k < seqs.size() && !rc; ++k) {
    const int lane = int(k % size_t(nside + 1));  // 0: the caller's stream
    ctx->stream = lane == 0 ? main : ctx->side[lane - 1];
    rc = enqueue_seq(seqs[k]);
  }
  ctx->stream = main;
  // join every side stream, also after a failed enqueue, so that a capture stays well formed
  for (int i = 0; i < nside; ++i) {
    hipError_t je = hipEventRecord(ctx->join_ev[i], ctx->side[i]);
    if (je == hipSuccess) je = hipStreamWaitEvent(ctx->stream, ctx->join_ev[i], 0);
    if (je != hipSuccess && !rc) rc = hip_fail(je, "stream join");
  }
  return rc;
}

// Replay (capturing on first use) the graph of n steps of dt.
int launch_graph(spin1_ctx* ctx, int64_t n, double dt) {
  GraphEntry* hit = nullptr;
  for (GraphEntry& g : ctx->graphs)
    if (g.n == n && g.dt == dt && g.version == ctx->version) hit = &g;
  if (!hit) {
    hipGraph_t graph = nullptr;
    hipError_t e = hipStreamBeginCapture(ctx->stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return hip_fail(e, "hipStreamBeginCapture");
    const int rc = enqueue_steps(ctx, n, dt);
    e = hipStreamEndCapture(ctx->stream, &graph);
    if (rc) {
      if (graph) (void)hipGraphDestroy(graph);
      return rc;
    }
    if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
    hipGraphExec_t exec = nullptr;
    e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) return hip_fail(e, "hipGraphInstantiate");
    if (ctx->graphs.size() >= kMaxGraphs) {  // evict the least recently used
      size_t lru = 0;
      for (size_t i = 1; i < ctx->graphs.size(); ++i)
        if (ctx->graphs[i].last_use < ctx->graphs[lru].last_use) lru = i;
      (void)hipGraphExecDestroy(ctx->graphs[lru].exec);
      ctx->graphs.erase(ctx->graphs.begin() + long(lru));
    }
    ctx->graphs.push_back(GraphEntry{n, dt, ctx->version, 0, exec});
    hit = &ctx->graphs.back();
  }
  hit->last_use = ++ctx->use_clock;
  const hipError_t e = hipGraphLaunch(hit->exec, ctx->stream);
  if (e != hipSuccess) return hip_fail(e, "hipGraphLaunch");
  return SPIN1_OK;
}

int bind_impl(spin1_ctx* ctx, const spin1_grid* groups, int32_t n_groups, const spin1_params* p,
              void* const* psi_dev, void* ws) {
  int rc = check_ctx(ctx, false);
  if (rc) return rc;
  if (n_groups < 1 || !groups) return fail(SPIN1_EINVAL, "need at least one group");
  if (!psi_dev) return fail(SPIN1_EINVAL, "psi_dev is NULL");
  if (!ws) return fail(SPIN1_EINVAL, "workspace pointer is NULL");
  if ((rc = validate_params(p))) return rc;
  for (int i = 0; i < n_groups; ++i) {
    if ((rc = validate_grid(&groups[i], ctx->dtype))) return rc;
    if (!psi_dev[i]) return fail(SPIN1_EINVAL, "psi_dev[%d] is NULL", i);
    if (reinterpret_cast<uintptr_t>(psi_dev[i]) % (ctx->dbl ? 16 : 8))
      return fail(SPIN1_EINVAL, "psi_dev[%d] is not aligned to the complex size", i);
  }
  if (reinterpret_cast<uintptr_t>(ws) % 256) return fail(SPIN1_EINVAL, "workspace must be 256-byte aligned");
  std::vector<GroupState> gs(static_cast<size_t>(n_groups));
  size_t off = 0;
  for (int i = 0; i < n_groups; ++i) {
    gs[size_t(i)].grid = groups[i];
    gs[size_t(i)].geo = geom_of(&groups[i]);
    gs[size_t(i)].psi = psi_dev[i];
    gs[size_t(i)].nbins = num_bins_of(gs[size_t(i)].geo);
    off = layout_group(gs[size_t(i)].geo, ctx->dbl, off, &gs[size_t(i)].lay);
  }
  ctx->groups.swap(gs);
  ctx->ws = static_cast<char*>(ws);
  ctx->p = *p;
  ctx->bound = true;
  ctx->tab_valid = false;
  ctx->version++;
  ctx->drop_graphs();
  for (auto& G : ctx->groups)
    if ((rc = upload_shells(ctx, G))) {
      ctx->bound = false;
      return rc;
    }
  if ((rc = make_tables(ctx, 0.0))) {
    ctx->bound = false;
    return rc;
  }
  return SPIN1_OK;
}

}  // namespace

extern "C" {

const char* spin1_last_error(void) { return g_err.c_str(); }

int spin1_check_grid(const spin1_grid* g, int32_t dtype) { return validate_grid(g, dtype); }

size_t spin1_field_bytes(const spin1_grid* g, int32_t dtype) {
  if (validate_grid(g, dtype)) return 0;
  const Geom G = geom_of(g);
  return size_t(G.S) * 3 * size_t(G.sites) * (dtype == SPIN1_C128 ? 16 : 8);
}

size_t spin1_workspace_bytes(const spin1_grid* groups, int32_t n_groups, int32_t dtype) {
  if (!groups || n_groups < 1) {
    fail(SPIN1_EINVAL, "need at least one group");
    return 0;
  }
  size_t off = 0;
  for (int i = 0; i < n_groups; ++i) {
    if (validate_grid(&groups[i], dtype)) return 0;
    Layout L;
    off = layout_group(geom_of(&groups[i]), dtype == SPIN1_C128, off, &L);
  }
  return off;
}

int32_t spin1_num_bins(const spin1_grid* g) {
  const int rc = validate_grid(g, SPIN1_C64);
  if (rc) return rc;
  return num_bins_of(geom_of(g));
}

int spin1_bin_counts(const spin1_grid* g, int64_t* counts) {
  int rc = validate_grid(g, SPIN1_C64);
  if (rc) return rc;
  if (!counts) return fail(SPIN1_EINVAL, "counts pointer is NULL");
  const Geom G = geom_of(g);
  const int nb = num_bins_of(G);
  for (int b = 0; b < nb; ++b) counts[b] = 0;
  for (int64_t s = 0; s < G.sites; ++s) counts[shell_of(mode_J(G, s))]++;
  return SPIN1_OK;
}

int spin1_create(spin1_ctx** out, int32_t dtype, void* stream) {
  if (!out) return fail(SPIN1_EINVAL, "out pointer is NULL");
  if (dtype != SPIN1_C64 && dtype != SPIN1_C128) return fail(SPIN1_EINVAL, "dtype %d is not SPIN1_C64/SPIN1_C128", dtype);
  int dev = 0;
  const hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  spin1_ctx* c = new (std::nothrow) spin1_ctx;
  if (!c) return fail(SPIN1_ENOMEM, "context allocation failed");
  c->dtype = dtype;
  c->dbl = dtype == SPIN1_C128;
  c->stream = static_cast<hipStream_t>(stream);
  c->device = dev;
  scratch_setup(dev);  // the no-allocation observables' scratch on this device
  *out = c;
  return SPIN1_OK;
}

int spin1_destroy(spin1_ctx* ctx) {
  if (!ctx) return fail(SPIN1_EINVAL, "context is NULL");
  delete ctx;
  return SPIN1_OK;
}

int spin1_bind(spin1_ctx* ctx, const spin1_grid* groups, int32_t n_groups, const spin1_params* p,
               void* const* psi_dev, void* workspace_dev) {
  return bind_impl(ctx, groups, n_groups, p, psi_dev, workspace_dev);
}

int spin1_init_wigner_shard(spin1_ctx* ctx, uint64_t seed, const spin1_grid* groups, int32_t n_groups,
                            const int64_t* first_sample, const spin1_params* p, void* const* psi_dev,
                            void* workspace_dev) {
  int rc = check_ctx(ctx, false);
  if (rc) return rc;
  if (first_sample && n_groups > 0 && groups)  // checked before the bind changes any state
    for (int32_t i = 0; i < n_groups; ++i)
      if (first_sample[i] < 0 || first_sample[i] > (int64_t(1) << 62) - groups[i].samples)
        return fail(SPIN1_EINVAL, "first_sample[%d] = %lld is out of range", i, (long long)first_sample[i]);
  rc = bind_impl(ctx, groups, n_groups, p, psi_dev, workspace_dev);
  if (rc) return rc;
  for (size_t i = 0; i < ctx->groups.size(); ++i) {
    const GroupState& G = ctx->groups[i];
    Prof pr(ctx, SPIN1_K_OTHER);
    const uint64_t first = first_sample ? uint64_t(first_sample[i]) : 0;
    const hipError_t e =
        launch_init(ctx->stream, ctx->dbl, G.psi, G.geo, seed, uint64_t(i), first, ctx->p.n0, ctx->p.wigner_var);
    if (e != hipSuccess) return hip_fail(e, "init kernel");
  }
  return SPIN1_OK;
}

int spin1_init_wigner(spin1_ctx* ctx, uint64_t seed, const spin1_grid* groups, int32_t n_groups,
                      const spin1_params* p, void* const* psi_dev, void* workspace_dev) {
  return spin1_init_wigner_shard(ctx, seed, groups, n_groups, nullptr, p, psi_dev, workspace_dev);
}

int spin1_set_params(spin1_ctx* ctx, const spin1_params* p) {
  int rc = check_ctx(ctx, true);
  if (rc) return rc;
  if ((rc = validate_params(p))) return rc;
  ctx->p = *p;
  ctx->tab_valid = false;
  ctx->version++;
  return SPIN1_OK;
}

int spin1_sync_field(spin1_ctx* ctx) { return check_ctx(ctx, true); }

int spin1_step(spin1_ctx* ctx, int64_t n, double dt) {
  int rc = check_ctx(ctx, true);
  if (rc) return rc;
  if (n < 0) return fail(SPIN1_EINVAL, "n must be >= 0");
  if (!isfinite(dt)) return fail(SPIN1_EINVAL, "dt must be finite");
  if (n == 0 || dt == 0.0) return SPIN1_OK;
  if (!ctx->tab_valid || ctx->tab_dt != dt || ctx->tab_q != ctx->p.q)
    if ((rc = make_tables(ctx, dt))) return rc;
  const bool graphs = ctx->use_graphs && !ctx->prof && ctx->stream != nullptr;
  if (!graphs) return enqueue_steps(ctx, n, dt);
  // calls longer than the graph limit run as consecutive synchronised chunks
  while (n > 0) {
    const int64_t m = n < ctx->graph_max_steps ? n : ctx->graph_max_steps;
    if ((rc = launch_graph(ctx, m, dt))) return rc;
    n -= m;
  }
  return SPIN1_OK;
}

int spin1_local_update(spin1_ctx* ctx, double tau) {
  int rc = check_ctx(ctx, true);
  if (rc) return rc;
  if (!isfinite(tau)) return fail(SPIN1_EINVAL, "tau must be finite");
  for (auto& G : ctx->groups) {
    Prof pr(ctx, SPIN1_K_LOCAL);
    const hipError_t e = launch_local(ctx->stream, ctx->dbl, G.psi, G.geo.S, G.geo.sites, tau, ctx->p.c0, ctx->p.c1, G.pot);
    if (e != hipSuccess) return hip_fail(e, "local update");
  }
  return SPIN1_OK;
}

int spin1_structure_factor(spin1_ctx* ctx, int32_t group, double* bins_dev) {
  int rc = check_ctx(ctx, true);
  if (rc) return rc;
  if (group < 0 || size_t(group) >= ctx->groups.size()) return fail(SPIN1_EINVAL, "group %d out of range", group);
  if (!bins_dev) return fail(SPIN1_EINVAL, "bins_dev is NULL");
  const GroupState& G = ctx->groups[size_t(group)];
  XPassArgs xa = xargs(ctx, G);
  hipError_t e;
  {
    Prof pr(ctx, SPIN1_K_SPECTRUM);
    if (G.geo.dim == 1) {
      xa.out = at(ctx, G.lay.pow);
      e = launch_xpass(ctx->stream, ctx->dbl, MODE_SF_POWER, G.geo.n[0], xa);
    } else {
      xa.out = at(ctx, G.lay.sff);
      e = launch_xpass(ctx->stream, ctx->dbl, MODE_SF, G.geo.n[0], xa);
    }
  }
  if (e != hipSuccess) return hip_fail(e, "spectrum x-pass");
  for (int a = 1; a < G.geo.dim; ++a) {
    SPassArgs sa = sargs(ctx, G, a, at(ctx, G.lay.sff), G.geo.S);
    const bool last = a == G.geo.dim - 1;
    sa.out = at(ctx, G.lay.pow);
    {
      Prof pr(ctx, SPIN1_K_SPECTRUM);
      e = launch_spass(ctx->stream, ctx->dbl, last ? MODE_SF_POWER : MODE_SF, G.geo.n[a], sa);
    }
    if (e != hipSuccess) return hip_fail(e, "spectrum strided pass");
  }
  Prof pr(ctx, SPIN1_K_SHELLS);
  e = launch_bin(ctx->stream, ctx->dbl, at(ctx, G.lay.pow), G.geo.S, G.geo.sites,
                 reinterpret_cast<const int32_t*>(at(ctx, G.lay.perm)),
                 reinterpret_cast<const int32_t*>(at(ctx, G.lay.offs)), G.nbins, bins_dev);
  if (e != hipSuccess) return hip_fail(e, "shell kernel");
  return SPIN1_OK;
}

// The observables of group G: MEASURE passes writing FP64 partials to
// part_x ([S*rows][4]), part_y and part_z (one per strided-pass workgroup,
// nblk[1] and nblk[2] of them), then the per-sample finish into obs.
static int enqueue_observables(spin1_ctx* ctx, const GroupState& G, double* part_x, double* part_y, double* part_z,
                               double* obs) {
  XPassArgs xa = xargs(ctx, G);
  xa.part = part_x;
  Prof pr(ctx, SPIN1_K_OBSERVABLES);
  hipError_t e = launch_xpass(ctx->stream, ctx->dbl, MODE_MEASURE, G.geo.n[0], xa);
  if (e != hipSuccess) return hip_fail(e, "energy x-pass");
  for (int a = 1; a < G.geo.dim; ++a) {
    SPassArgs sa = sargs(ctx, G, a, G.psi, int64_t(3) * G.geo.S);
    sa.part = a == 1 ? part_y : part_z;
    e = launch_spass(ctx->stream, ctx->dbl, MODE_MEASURE, G.geo.n[a], sa);
    if (e != hipSuccess) return hip_fail(e, "energy strided pass");
  }
  e = launch_obs_finish(ctx->stream, G.geo.S, part_x, G.geo.rows, G.geo.dim > 1 ? part_y : nullptr,
                        G.lay.nblk[1] / G.geo.S, G.geo.dim > 2 ? part_z : nullptr, G.lay.nblk[2] / G.geo.S,
                        cell_of(G.geo), obs);
  if (e != hipSuccess) return hip_fail(e, "observables finish");
  return SPIN1_OK;
}

int spin1_observables(spin1_ctx* ctx, int32_t group, double* obs_dev) {
  int rc = check_ctx(ctx, true);
  if (rc) return rc;
  if (group < 0 || size_t(group) >= ctx->groups.size()) return fail(SPIN1_EINVAL, "group %d out of range", group);
  if (!obs_dev) return fail(SPIN1_EINVAL, "obs_dev is NULL");
  const GroupState& G = ctx->groups[size_t(group)];
  auto part = [&](int a) { return reinterpret_cast<double*>(at(ctx, G.lay.part[a])); };
  return enqueue_observables(ctx, G, part(0), part(1), part(2), obs_dev);
}

int spin1_observables_noalloc(spin1_ctx* ctx, int32_t group, double* obs_dev) {
  int rc = check_ctx(ctx, true);
  if (rc) return rc;
  if (group < 0 || size_t(group) >= ctx->groups.size()) return fail(SPIN1_EINVAL, "group %d out of range", group);
  if (!obs_dev) return fail(SPIN1_EINVAL, "obs_dev is NULL");
  const GroupState& G = ctx->groups[size_t(group)];
  // the same partials as the workspace layout, packed into the static scratch
  const size_t ox = 0;
  const size_t oy = align_up(ox + size_t(G.geo.S) * size_t(G.geo.rows) * 4 * sizeof(double));
  const size_t oz = align_up(oy + size_t(G.lay.nblk[1]) * sizeof(double));
  const size_t end = align_up(oz + size_t(G.lay.nblk[2]) * sizeof(double));
  if (end > kNoAllocScratchBytes)
    return fail(SPIN1_EUNSUPPORTED,
                "group %d needs %zu bytes of partial sums; the static scratch of spin1_observables_noalloc holds %zu "
                "(use spin1_observables)",
                group, end, kNoAllocScratchBytes);
  hipError_t e = hipSuccess;
  char* base = static_cast<char*>(scratch_of(ctx->device, &e));
  if (!base) return hip_fail(e, "address of the static scratch");
  return enqueue_observables(ctx, G, reinterpret_cast<double*>(base + ox), reinterpret_cast<double*>(base + oy),
                             reinterpret_cast<double*>(base + oz), obs_dev);
}

int spin1_transverse_spin(spin1_ctx* ctx, int32_t group, void* fperp_dev) {
  int rc = check_ctx(ctx, true);
  if (rc) return rc;
  if (group < 0 || size_t(group) >= ctx->groups.size()) return fail(SPIN1_EINVAL, "group %d out of range", group);
  if (!fperp_dev) return fail(SPIN1_EINVAL, "fperp_dev is NULL");
  const GroupState& G = ctx->groups[size_t(group)];
  Prof pr(ctx, SPIN1_K_OBSERVABLES);
  const hipError_t e = launch_f_perp(ctx->stream, ctx->dbl, G.psi, G.geo.S, G.geo.sites, fperp_dev);
  if (e != hipSuccess) return hip_fail(e, "transverse spin");
  return SPIN1_OK;
}

int spin1_spin_texture(spin1_ctx* ctx, int32_t group, double* out_dev) {
  int rc = check_ctx(ctx, true);
  if (rc) return rc;
  if (group < 0 || size_t(group) >= ctx->groups.size()) return fail(SPIN1_EINVAL, "group %d out of range", group);
  if (!out_dev) return fail(SPIN1_EINVAL, "out_dev is NULL");
  const GroupState& G = ctx->groups[size_t(group)];
  Prof pr(ctx, SPIN1_K_OBSERVABLES);
  // the x-pass partials ([S*rows][4] doubles) hold the [S*rows][3] row sums
  const hipError_t e = launch_texture(ctx->stream, ctx->dbl, G.psi, G.geo.S, G.geo.rows, G.geo.sites, G.geo.n[0],
                                      reinterpret_cast<double*>(at(ctx, G.lay.part[0])), out_dev);
  if (e != hipSuccess) return hip_fail(e, "spin texture");
  return SPIN1_OK;
}

// One step of group G with the observables of the state its kinetic sub-step
// starts from summed inside the passes and finished into obs (S x 3).
static int enqueue_group_step_logged(spin1_ctx* ctx, const GroupState& G, double dt, double tau_open,
                                     double tau_close, double* obs) {
  XPassArgs xa = xargs(ctx, G);
  xa.tau_pre = tau_open;
  xa.tau_post = G.geo.dim == 1 ? tau_close : 0.0;
  xa.part = reinterpret_cast<double*>(at(ctx, G.lay.part[0]));
  hipError_t e;
  {
    Prof pr(ctx, SPIN1_K_XPASS);
    e = launch_xpass(ctx->stream, ctx->dbl, MODE_STEP_LOG, G.geo.n[0], xa);
  }
  if (e != hipSuccess) return hip_fail(e, "logged x-pass");
  for (int a = 1; a < G.geo.dim; ++a) {
    SPassArgs sa = sargs(ctx, G, a, G.psi, int64_t(3) * G.geo.S);
    sa.part = reinterpret_cast<double*>(at(ctx, G.lay.part[a]));
    {
      Prof pr(ctx, a == 1 ? SPIN1_K_YPASS : SPIN1_K_ZPASS);
      e = launch_spass(ctx->stream, ctx->dbl, MODE_STEP_LOG, G.geo.n[a], sa);
    }
    if (e != hipSuccess) return hip_fail(e, "logged strided pass");
  }
  {
    const double* py = G.geo.dim > 1 ? reinterpret_cast<const double*>(at(ctx, G.lay.part[1])) : nullptr;
    const double* pz = G.geo.dim > 2 ? reinterpret_cast<const double*>(at(ctx, G.lay.part[2])) : nullptr;
    Prof pr(ctx, SPIN1_K_OBSERVABLES);
    e = launch_obs_finish(ctx->stream, G.geo.S, reinterpret_cast<const double*>(at(ctx, G.lay.part[0])), G.geo.rows,
                          py, G.lay.nblk[1] / G.geo.S, pz, G.lay.nblk[2] / G.geo.S, cell_of(G.geo), obs);
  }
  if (e != hipSuccess) return hip_fail(e, "logged observables finish");
  if (G.geo.dim > 1 && tau_close != 0.0) {
    {
      Prof pr(ctx, SPIN1_K_LOCAL);
      e = launch_local(ctx->stream, ctx->dbl, G.psi, G.geo.S, G.geo.sites, tau_close, ctx->p.c0, ctx->p.c1, G.pot);
    }
    if (e != hipSuccess) return hip_fail(e, "closing local update");
  }
  return SPIN1_OK;
}

int spin1_step_observed(spin1_ctx* ctx, int64_t n, double dt, int32_t group, double* obs_dev) {
  int rc = check_ctx(ctx, true);
  if (rc) return rc;
  if (group < 0 || size_t(group) >= ctx->groups.size()) return fail(SPIN1_EINVAL, "group %d out of range", group);
  if (!obs_dev) return fail(SPIN1_EINVAL, "obs_dev is NULL");
  if (ctx->scheme != SPIN1_SCHEME_STRANG) return fail(SPIN1_EUNSUPPORTED, "the step log takes the Strang scheme");
  if (n < 0) return fail(SPIN1_EINVAL, "n must be >= 0");
  if (!isfinite(dt)) return fail(SPIN1_EINVAL, "dt must be finite");
  if (n == 0) return SPIN1_OK;
  if (!ctx->tab_valid || ctx->tab_dt != dt || ctx->tab_q != ctx->p.q)
    if ((rc = make_tables(ctx, dt))) return rc;
  const int64_t S = ctx->groups[size_t(group)].geo.S;
  for (int64_t i = 0; i < n; ++i) {
    const double pre = i == 0 ? 0.5 * dt : dt;
    const double close = i == n - 1 ? 0.5 * dt : 0.0;
    for (size_t g = 0; g < ctx->groups.size(); ++g) {
      const GroupState& G = ctx->groups[g];
      rc = int64_t(g) == group ? enqueue_group_step_logged(ctx, G, dt, pre, close, obs_dev + i * S * 3)
                               : enqueue_group_step(ctx, G, G.psi, pre, close, nullptr, i);
      if (rc) return rc;
    }
  }
  return SPIN1_OK;
}

// ---------------------------------------------------------------------------
// reverse mode
// ---------------------------------------------------------------------------
static size_t adj_layout(const Geom& g, bool dbl, int64_t every, size_t* seg, size_t* hbuf, size_t* part,
                         size_t* acc) {
  const size_t fb = size_t(g.S) * 3 * size_t(g.sites) * (dbl ? 16 : 8);
  size_t off = 0;
  *seg = off;
  off = align_up(off + size_t(every + 1) * fb);
  *hbuf = off;
  off = align_up(off + fb);
  *part = off;
  off = align_up(off + size_t(adj_local_blocks(g.S, g.sites)) * 2 * sizeof(double));
  *acc = off;
  off = align_up(off + 2 * sizeof(double));
  return off;
}

size_t spin1_adjoint_workspace_bytes(const spin1_grid* g, int32_t dtype, int64_t every) {
  if (validate_grid(g, dtype)) return 0;
  if (every < 1) {
    fail(SPIN1_EINVAL, "checkpoint interval must be >= 1");
    return 0;
  }
  size_t a, b, c, d;
  return adj_layout(geom_of(g), dtype == SPIN1_C128, every, &a, &b, &c, &d);
}

static int check_adjoint_args(spin1_ctx* ctx, int64_t n, double dt, int64_t every) {
  int rc = check_ctx(ctx, true);
  if (rc) return rc;
  if (ctx->groups.size() != 1) return fail(SPIN1_EUNSUPPORTED, "reverse mode supports one bound group");
  if (ctx->scheme != SPIN1_SCHEME_STRANG) return fail(SPIN1_EUNSUPPORTED, "reverse mode takes the Strang scheme");
  if (ctx->groups[0].pot) return fail(SPIN1_EUNSUPPORTED, "reverse mode takes no trap potential");
  if (n < 1) return fail(SPIN1_EINVAL, "n must be >= 1");
  if (every < 1) return fail(SPIN1_EINVAL, "checkpoint interval must be >= 1");
  if (!isfinite(dt) || dt == 0.0) return fail(SPIN1_EINVAL, "dt must be finite and nonzero");
  return SPIN1_OK;
}

int spin1_forward_ckpt(spin1_ctx* ctx, int64_t n, double dt, int64_t every, void* ckpt_dev) {
  int rc = check_adjoint_args(ctx, n, dt, every);
  if (rc) return rc;
  if (!ckpt_dev) return fail(SPIN1_EINVAL, "ckpt_dev is NULL");
  const GroupState& G = ctx->groups[0];
  const size_t fb = size_t(G.geo.S) * 3 * size_t(G.geo.sites) * (ctx->dbl ? 16 : 8);
  const int64_t nck = (n + every - 1) / every;
  for (int64_t c = 0; c < nck; ++c) {
    const hipError_t e = hipMemcpyAsync(static_cast<char*>(ckpt_dev) + size_t(c) * fb, G.psi, fb,
                                        hipMemcpyDeviceToDevice, ctx->stream);
    if (e != hipSuccess) return hip_fail(e, "checkpoint copy");
    const int64_t m = (n - c * every) < every ? (n - c * every) : every;
    if ((rc = spin1_step(ctx, m, dt))) return rc;
  }
  return SPIN1_OK;
}

int spin1_adjoint(spin1_ctx* ctx, int64_t n, double dt, int64_t every, const void* ckpt_dev,
                  const double* dl_dbins_dev, void* adj_ws_dev, void* grad_psi0_dev, double* grad_qc1_dev) {
  int rc = check_adjoint_args(ctx, n, dt, every);
  if (rc) return rc;
  if (!ckpt_dev || !dl_dbins_dev || !adj_ws_dev || !grad_psi0_dev || !grad_qc1_dev)
    return fail(SPIN1_EINVAL, "a device pointer argument is NULL");
  if (reinterpret_cast<uintptr_t>(adj_ws_dev) % 256) return fail(SPIN1_EINVAL, "adjoint workspace must be 256-byte aligned");
  if (!ctx->tab_valid || ctx->tab_dt != dt || ctx->tab_q != ctx->p.q)
    if ((rc = make_tables(ctx, dt))) return rc;
  const GroupState& G = ctx->groups[0];
  const Geom& g = G.geo;
  const size_t fb = size_t(g.S) * 3 * size_t(g.sites) * (ctx->dbl ? 16 : 8);
  size_t oseg, oh, opart, oacc;
  adj_layout(g, ctx->dbl, every, &oseg, &oh, &opart, &oacc);
  char* ws = static_cast<char*>(adj_ws_dev);
  char* seg = ws + oseg;
  void* H = ws + oh;
  double* part = reinterpret_cast<double*>(ws + opart);
  double* acc = reinterpret_cast<double*>(ws + oacc);
  const int nblk = adj_local_blocks(g.S, g.sites);
  hipStream_t st = ctx->stream;
  hipError_t e;
  void* sff = at(ctx, G.lay.sff);

  // 1. spectrum Fhat of the final field
  XPassArgs xa = xargs(ctx, G);
  xa.out = sff;
  if ((e = launch_xpass(st, ctx->dbl, MODE_SF, g.n[0], xa)) != hipSuccess) return hip_fail(e, "adjoint spectrum x");
  for (int a = 1; a < g.dim; ++a) {
    const SPassArgs sa = sargs(ctx, G, a, sff, g.S);
    if ((e = launch_spass(st, ctx->dbl, MODE_SF, g.n[a], sa)) != hipSuccess) return hip_fail(e, "adjoint spectrum");
  }
  // 2. seed in spectral space and back to real space (H(F_perp) = DFT(H(Fhat)))
  if ((e = launch_adj_spectrum(st, ctx->dbl, sff, g, reinterpret_cast<const int32_t*>(at(ctx, G.lay.offs)), G.nbins,
                               dl_dbins_dev)) != hipSuccess)
    return hip_fail(e, "adjoint spectral seed");
  if ((e = launch_fft1_x(st, ctx->dbl, g.n[0], sff, at(ctx, G.lay.tw[0]), int64_t(g.S) * g.rows)) != hipSuccess)
    return hip_fail(e, "adjoint x transform");
  for (int a = 1; a < g.dim; ++a) {
    const SPassArgs sa = sargs(ctx, G, a, sff, g.S);
    if ((e = launch_spass(st, ctx->dbl, MODE_SF, g.n[a], sa)) != hipSuccess) return hip_fail(e, "adjoint transform");
  }
  // 3. H(psi_T) from H(F_perp)
  if ((e = launch_adj_seed(st, ctx->dbl, G.psi, sff, H, g.S, g.sites)) != hipSuccess) return hip_fail(e, "adjoint seed");
  if ((e = hipMemsetAsync(acc, 0, 2 * sizeof(double), st)) != hipSuccess) return hip_fail(e, "clear accumulators");

  // 4. segments in reverse: recompute the states, then walk the steps backwards.
  //    Backwards, the local-update VJPs run at psi_n (closing half of the last
  //    step), then after each step's kinetic pass at psi_i: the opening half of
  //    step i fused with the closing half of step i - 1, and at psi_0 the
  //    opening half alone.
  const int64_t nck = (n + every - 1) / every;
  const double half = 0.5 * dt;
  auto local_vjp = [&](int kind, const void* state) -> int {
    hipError_t le = launch_adj_local(st, ctx->dbl, kind, state, H, g.S, g.sites, half, ctx->p.c0, ctx->p.c1, dt, part);
    if (le != hipSuccess) return hip_fail(le, "local-update VJP");
    if ((le = launch_adj_accum(st, part, nblk, acc)) != hipSuccess) return hip_fail(le, "adjoint accumulate");
    return SPIN1_OK;
  };
  for (int64_t c = nck - 1; c >= 0; --c) {
    const int64_t len = (n - c * every) < every ? (n - c * every) : every;
    e = hipMemcpyAsync(seg, static_cast<const char*>(ckpt_dev) + size_t(c) * fb, fb, hipMemcpyDeviceToDevice, st);
    if (e != hipSuccess) return hip_fail(e, "segment copy");
    for (int64_t j = 0; j < len; ++j)  // state j + 1 from state j, out of place
      if ((rc = enqueue_group_step(ctx, G, seg + size_t(j + 1) * fb, half, half, seg + size_t(j) * fb))) return rc;
    if (c == nck - 1 && (rc = local_vjp(ADJ_CLOSE, seg + size_t(len) * fb))) return rc;
    for (int64_t j = len - 1; j >= 0; --j) {
      if ((rc = enqueue_group_step(ctx, G, H, 0.0, 0.0))) return rc;
      if ((rc = local_vjp(c == 0 && j == 0 ? ADJ_OPEN : ADJ_OPEN_CLOSE, seg + size_t(j) * fb))) return rc;
    }
  }
  // 5. outputs in the real-gradient convention
  if ((e = launch_conj(st, ctx->dbl, H, grad_psi0_dev, int64_t(g.S) * 3 * g.sites)) != hipSuccess)
    return hip_fail(e, "gradient output");
  if ((e = hipMemcpyAsync(grad_qc1_dev, acc, 2 * sizeof(double), hipMemcpyDeviceToDevice, st)) != hipSuccess)
    return hip_fail(e, "gradient output");
  return SPIN1_OK;
}

// ---------------------------------------------------------------------------
// autotuning of the step passes
// ---------------------------------------------------------------------------
int32_t spin1_num_variants(void) { return step_variants(); }

static int check_variant_args(spin1_ctx* ctx, int32_t pass, int32_t n) {
  int rc = check_ctx(ctx, false);
  if (rc) return rc;
  if (pass != 0 && pass != 1) return fail(SPIN1_EINVAL, "pass must be 0 (x) or 1 (strided)");
  if (!is_pow2(n) || n < 8 || n > (pass == 0 ? 4096 : 1024)) return fail(SPIN1_EINVAL, "no kernel for n = %d", n);
  return SPIN1_OK;
}

int spin1_get_variant(spin1_ctx* ctx, int32_t pass, int32_t n, int32_t* variant) {
  int rc = check_variant_args(ctx, pass, n);
  if (rc) return rc;
  if (!variant) return fail(SPIN1_EINVAL, "variant pointer is NULL");
  *variant = ctx->variant[pass][ctx->dbl ? 1 : 0][log2_of(n)];
  return SPIN1_OK;
}

int spin1_set_variant(spin1_ctx* ctx, int32_t pass, int32_t n, int32_t variant) {
  int rc = check_variant_args(ctx, pass, n);
  if (rc) return rc;
  if (variant < 0 || variant >= step_variants()) return fail(SPIN1_EINVAL, "variant %d out of range", variant);
  ctx->variant[pass][ctx->dbl ? 1 : 0][log2_of(n)] = int8_t(variant);
  ctx->version++;
  return SPIN1_OK;
}

int spin1_autotune(spin1_ctx* ctx, void* scratch_dev, size_t scratch_bytes, int32_t reps) {
  int rc = check_ctx(ctx, true);
  if (rc) return rc;
  if (!scratch_dev) return fail(SPIN1_EINVAL, "scratch pointer is NULL");
  if (reps < 1 || reps > 1000) return fail(SPIN1_EINVAL, "reps must be in 1..1000");
  const double dt = ctx->tab_dt != 0.0 ? ctx->tab_dt : 0.01;
  if (!ctx->tab_valid || ctx->tab_dt != dt || ctx->tab_q != ctx->p.q)
    if ((rc = make_tables(ctx, dt))) return rc;
  hipEvent_t ev[2];
  if (hipEventCreate(&ev[0]) != hipSuccess) return fail(SPIN1_EHIP, "hipEventCreate");
  if (hipEventCreate(&ev[1]) != hipSuccess) {
    (void)hipEventDestroy(ev[0]);
    return fail(SPIN1_EHIP, "hipEventCreate");
  }
  // fastest timed sweep per (pass, log2 n, variant)
  double best_ms[2][13][8];
  for (auto& a : best_ms)
    for (auto& b : a)
      for (double& c : b) c = 1e300;
  bool seen[2][13] = {};
  const int nv = step_variants();
  rc = SPIN1_OK;
  for (auto& G : ctx->groups) {
    const size_t fb = size_t(G.geo.S) * 3 * size_t(G.geo.sites) * (ctx->dbl ? 16 : 8);
    if (fb > scratch_bytes) {
      rc = fail(SPIN1_EINVAL, "scratch of %zu bytes is smaller than a field (%zu bytes)", scratch_bytes, fb);
      break;
    }
    hipError_t e = hipMemcpyAsync(scratch_dev, G.psi, fb, hipMemcpyDeviceToDevice, ctx->stream);
    if (e != hipSuccess) {
      rc = hip_fail(e, "autotune copy");
      break;
    }
    for (int axis = 0; axis < G.geo.dim && !rc; ++axis) {
      const int pass = axis == 0 ? 0 : 1;
      const int lg = log2_of(G.geo.n[axis]);
      seen[pass][lg] = true;
      // sweep 0 brings the clocks up and is not counted; sweeps 1..3 are
      // timed, the variants taking turns, and each variant keeps its fastest
      // (one sweep disturbed by anything else on the GPU changes no choice)
      for (int sweep = 0; sweep < 4 && !rc; ++sweep)
      for (int v = 0; v < nv && !rc; ++v) {
        auto launch = [&]() {
          if (pass == 0) {
            XPassArgs xa = xargs(ctx, G);
            xa.psi = scratch_dev;
            xa.tau_pre = dt;
            return launch_xpass(ctx->stream, ctx->dbl, MODE_STEP, G.geo.n[0], xa, v + twiddle_offset(ctx));
          }
          const SPassArgs sa = sargs(ctx, G, axis, scratch_dev, int64_t(3) * G.geo.S);
          return launch_spass(ctx->stream, ctx->dbl, MODE_STEP, G.geo.n[axis], sa, v + twiddle_offset(ctx));
        };
        e = launch();  // warm-up (also loads the code object)
        if (e == hipSuccess) e = hipEventRecord(ev[0], ctx->stream);
        for (int r = 0; r < reps && e == hipSuccess; ++r) e = launch();
        if (e == hipSuccess) e = hipEventRecord(ev[1], ctx->stream);
        if (e == hipSuccess) e = hipEventSynchronize(ev[1]);
        float ms = 0.0f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, ev[0], ev[1]);
        if (e != hipSuccess) {
          rc = hip_fail(e, "autotune timing");
          break;
        }
        if (sweep > 0 && double(ms) < best_ms[pass][lg][v]) best_ms[pass][lg][v] = double(ms);
      }
    }
    if (rc) break;
  }
  if (!rc)
    for (int pass = 0; pass < 2; ++pass)
      for (int lg = 0; lg < 13; ++lg) {
        if (!seen[pass][lg]) continue;
        int best = 0;
        for (int v = 1; v < nv; ++v)
          if (best_ms[pass][lg][v] < best_ms[pass][lg][best]) best = v;
        ctx->variant[pass][ctx->dbl ? 1 : 0][lg] = int8_t(best);
      }
  // Refinement in context: a pass variant interacts with the passes around
  // it (what the last-level cache holds when it starts, the direction the
  // previous pass walked), so each choice of a 2D/3D group is retried, one
  // (pass, n) at a time, by timing whole split steps of the groups that use
  // it, each on its scratch copy; the variant with the least total time stays.
  const bool prof = ctx->prof;
  ctx->prof = false;
  for (int pass = 0; pass < 2 && !rc; ++pass)
    for (int lg = 0; lg < 13 && !rc; ++lg) {
      if (!seen[pass][lg]) continue;
      const int n = 1 << lg;
      std::vector<const GroupState*> users;
      for (const GroupState& G : ctx->groups) {
        if (G.geo.dim < 2) continue;
        bool uses = pass == 0 && G.geo.n[0] == n;
        for (int a = 1; a < G.geo.dim && pass == 1; ++a) uses = uses || G.geo.n[a] == n;
        if (uses) users.push_back(&G);
      }
      if (users.empty()) continue;
      int8_t& slot = ctx->variant[pass][ctx->dbl ? 1 : 0][lg];
      int best = slot;
      double best_total = 1e300;
      for (int v = 0; v < nv && !rc; ++v) {
        slot = int8_t(v);
        double total = 0.0;
        for (const GroupState* G : users) {
          const size_t fb = size_t(G->geo.S) * 3 * size_t(G->geo.sites) * (ctx->dbl ? 16 : 8);
          hipError_t e = hipMemcpyAsync(scratch_dev, G->psi, fb, hipMemcpyDeviceToDevice, ctx->stream);
          if (e != hipSuccess) {
            rc = hip_fail(e, "autotune copy");
            break;
          }
          // one step to warm up, three timed
          rc = enqueue_group_step(ctx, *G, scratch_dev, dt, 0.0, nullptr, 0);
          if (!rc && (e = hipEventRecord(ev[0], ctx->stream)) != hipSuccess) rc = hip_fail(e, "autotune timing");
          for (int i = 1; i <= 3 && !rc; ++i) rc = enqueue_group_step(ctx, *G, scratch_dev, dt, 0.0, nullptr, i);
          if (rc) break;
          float ms = 0.0f;
          e = hipEventRecord(ev[1], ctx->stream);
          if (e == hipSuccess) e = hipEventSynchronize(ev[1]);
          if (e == hipSuccess) e = hipEventElapsedTime(&ms, ev[0], ev[1]);
          if (e != hipSuccess) {
            rc = hip_fail(e, "autotune timing");
            break;
          }
          total += double(ms);
        }
        if (!rc && total < best_total) {
          best_total = total;
          best = v;
        }
      }
      slot = int8_t(best);
    }
  ctx->prof = prof;
  (void)hipEventDestroy(ev[0]);
  (void)hipEventDestroy(ev[1]);
  if (rc) return rc;
  ctx->version++;
  return SPIN1_OK;
}

int spin1_set_potential(spin1_ctx* ctx, int32_t group, const double* v_dev) {
  int rc = check_ctx(ctx, true);
  if (rc) return rc;
  if (group < 0 || size_t(group) >= ctx->groups.size()) return fail(SPIN1_EINVAL, "group %d out of range", group);
  if (reinterpret_cast<uintptr_t>(v_dev) % sizeof(double))
    return fail(SPIN1_EINVAL, "the potential must be aligned to 8 bytes");
  ctx->groups[size_t(group)].pot = v_dev;
  ctx->version++;  // captured graphs hold the old kernel arguments and launch pattern
  return SPIN1_OK;
}

int spin1_set_option(spin1_ctx* ctx, int32_t option, int64_t value) {
  int rc = check_ctx(ctx, false);
  if (rc) return rc;
  switch (option) {
    case SPIN1_OPT_GRAPHS:
      ctx->use_graphs = value != 0;
      return SPIN1_OK;
    case SPIN1_OPT_GRAPH_MAX_STEPS:
      if (value < 1) return fail(SPIN1_EINVAL, "graph step limit must be >= 1");
      ctx->graph_max_steps = value;
      return SPIN1_OK;
    case SPIN1_OPT_SCHEME:
      if (value != SPIN1_SCHEME_STRANG && value != SPIN1_SCHEME_PAPER) return fail(SPIN1_EINVAL, "unknown scheme");
      ctx->scheme = int(value);
      ctx->version++;
      return SPIN1_OK;
    case SPIN1_OPT_1D_KERNEL:
      if (value < 0 || value > 2) return fail(SPIN1_EINVAL, "1D kernel choice must be 0, 1 or 2");
      ctx->kernel_1d = int(value);
      ctx->version++;
      return SPIN1_OK;
    case SPIN1_OPT_CONCURRENT_GROUPS:
      ctx->concurrent = value != 0;
      ctx->version++;
      return SPIN1_OK;
    case SPIN1_OPT_FP32_TWIDDLES:
      if (value != SPIN1_TWIDDLES_COMPENSATED && value != SPIN1_TWIDDLES_DITHERED)
        return fail(SPIN1_EINVAL, "unknown twiddle precision");
      ctx->dithered_tables = value == SPIN1_TWIDDLES_DITHERED;
      ctx->version++;
      return SPIN1_OK;
    case SPIN1_OPT_STREAMING_STORES:
      if (value != SPIN1_STORES_AUTO && value != SPIN1_STORES_CACHED && value != SPIN1_STORES_STREAMING)
        return fail(SPIN1_EINVAL, "unknown store form");
      ctx->stores = int(value);
      ctx->version++;
      return SPIN1_OK;
    case SPIN1_OPT_GROUPED_X:
      ctx->grouped_x = value != 0;
      ctx->version++;
      return SPIN1_OK;
    case SPIN1_OPT_STEPS_PER_LAUNCH_1D:
      if (value < 0 || value > 1024) return fail(SPIN1_EINVAL, "1D steps per launch must be in 0..1024");
      ctx->steps_per_launch_1d = int(value);
      ctx->version++;  // captured graphs hold the old launch pattern
      return SPIN1_OK;
  }
  return fail(SPIN1_EINVAL, "unknown option %d", option);
}

int spin1_profile_enable(spin1_ctx* ctx, int32_t enable) {
  int rc = check_ctx(ctx, false);
  if (rc) return rc;
  ctx->prof = enable != 0;
  return SPIN1_OK;
}

int spin1_profile_read(spin1_ctx* ctx, double* ms, int64_t* launches, int32_t n_kinds) {
  int rc = check_ctx(ctx, false);
  if (rc) return rc;
  if (!ms || !launches || n_kinds < 1 || n_kinds > SPIN1_K_COUNT)
    return fail(SPIN1_EINVAL, "need output arrays of 1..%d entries", int(SPIN1_K_COUNT));
  for (int k = 0; k < n_kinds; ++k) {
    ms[k] = 0.0;
    launches[k] = 0;
  }
  hipError_t e = hipStreamSynchronize(ctx->stream);
  if (e != hipSuccess) return hip_fail(e, "stream synchronize");
  for (const ProfRecord& r : ctx->rec) {
    float t = 0.0f;
    e = hipEventElapsedTime(&t, r.start, r.stop);
    if (e != hipSuccess) return hip_fail(e, "event elapsed time");
    if (r.kind < n_kinds) {
      ms[r.kind] += double(t);
      launches[r.kind] += 1;
    }
  }
  ctx->rec.clear();
  ctx->ev_used = 0;
  return SPIN1_OK;
}

}  // extern "C"
