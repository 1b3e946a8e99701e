// icr_api.hip -- host side of the C-ABI declared in include/icarus_hip.h.
//
// Owns argument validation, the device workspace layout, unit conversion of
// the API's SI inputs, the device-resident step loop and its HIP-graph
// replay.  All numerics run in the kernels of icr_kernels.hip.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "icarus_hip.h"
#include "icr_ensemble.hpp"
#include "icr_kernels.hpp"

using namespace icr;

namespace {

thread_local std::string g_err;

int fail(int code, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

#define HIP_TRY(expr)                                                              \
  do {                                                                             \
    hipError_t e_ = (expr);                                                        \
    if (e_ != hipSuccess)                                                          \
      return fail(ICR_ERR_HIP, "%s failed: %s", #expr, hipGetErrorString(e_));     \
  } while (0)

// ---- units: code value = SI value / unit ----------------------------------
constexpr double kAU = 1.495978707e11;
constexpr double kV = 1.0e5;
constexpr double kMp = 1.67262192369e-27;
constexpr double kKb = 1.380649e-23;
constexpr double kMu0 = 4.0e-7 * 3.14159265358979323846;
constexpr double kGM = 1.32712440018e20;
constexpr double kPi = 3.14159265358979323846;

struct Units {
  double t, len, rho, p, b, v;
  Units() {
    len = kAU;
    v = kV;
    t = kAU / kV;
    rho = kMp * 1.0e6;
    p = rho * kV * kV;
    b = std::sqrt(kMu0 * rho) * kV;
  }
  Scale scale() const {
    Scale s;
    const double c[NV] = {rho, v, v, v, p, b, b, b};
    for (int q = 0; q < NV; ++q) s.s[q] = c[q];
    s.t = t;
    s.len = len;
    return s;
  }
};

// Captured graphs of 16, 8, 4, 2 and 1 steps for each starting state buffer:
// a call of n steps replays at most n / 16 + 4 graphs.
constexpr int NGRAPH = 5;
constexpr int GRAPH_STEPS[NGRAPH] = {16, 8, 4, 2, 1};
// Host <-> device copies of states, tracers and divergences go through a
// staging region of the workspace in chunks of this many cells (8 doubles
// each): no call after creation allocates device memory.
constexpr long long STAGE_CELLS = 65536;

size_t align_up(size_t x) { return (x + 255) & ~size_t(255); }

struct Layout {
  size_t u[3], g[2], m64, mr, maps, tau, cme, traj, plog, pout, clock, partials, stage, total;
  long long stage_cells;  // cells per host-transfer chunk
  size_t t[3], fm, frout, ftend, tg[2];  // passive tracer (0 when off)
  long long max_blocks;
};

Layout make_layout(const icr_grid& g, const icr_phys& p) {
  Layout L{};
  const size_t rs = p.precision == ICR_PREC_F32 ? 4 : 8;
  const size_t ncell = (size_t)g.n_r * g.n_theta * g.n_phi;
  const size_t plane = (size_t)g.n_theta * g.n_phi;
  // partial slots: the largest grid of any stage-kernel launch configuration
  long long mb = 0;
  for (int tr : {64, 128, 256}) {
    const long long b = (long long)((g.n_r + tr - 1) / tr) *
                        ((g.n_theta + 256 / tr - 1) / (256 / tr)) * g.n_phi;
    mb = b > mb ? b : mb;
  }
  for (int tr : {32, 64}) {
    const long long b = stage_lds_blocks(g.n_r, g.n_theta, g.n_phi, tr, 1);
    mb = b > mb ? b : mb;
  }
  {
    const long long b = stage_w5_blocks(g.n_r, g.n_theta, g.n_phi, 1);
    mb = b > mb ? b : mb;
  }
  L.max_blocks = mb;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off += align_up(bytes);
    return o;
  };
  for (int q = 0; q < 3; ++q) L.u[q] = take(NV * ncell * rs);
  for (int q = 0; q < 2; ++q) L.g[q] = take(NV * plane * rs);
  L.m64 = take(sizeof(double) * METRIC64_LEN(g.n_r, g.n_theta));
  L.mr = take(rs * METRICR_LEN(g.n_r, g.n_theta));
  L.maps = take(sizeof(double) * (size_t)g.max_maps * NV * plane);
  L.tau = take(sizeof(double) * (size_t)g.max_maps);
  L.cme = take(sizeof(double) * 8 * (size_t)(g.max_cmes > 0 ? g.max_cmes : 1));
  L.traj = take(sizeof(double) * 4 * (size_t)(g.max_probes > 0 ? g.max_probes : 1) *
                (size_t)(g.max_traj_pts > 0 ? g.max_traj_pts : 1));
  L.plog = take(sizeof(double) * 12 * (size_t)(g.max_probes > 0 ? g.max_probes : 1) *
                (size_t)(g.probe_log_rows > 0 ? g.probe_log_rows : 1));
  L.pout = take(sizeof(double) * 12 * (size_t)(g.max_probes > 0 ? g.max_probes : 1));
  L.clock = take(sizeof(DevClock));
  L.partials = take(sizeof(double) * 4 * (size_t)L.max_blocks);
  // staging: the boundary / shell outputs ([8][nt][np] doubles at most) and
  // host-transfer chunks of stage_cells cells x 8 doubles
  L.stage_cells = (long long)ncell < STAGE_CELLS ? (long long)ncell : STAGE_CELLS;
  const size_t sb = (size_t)L.stage_cells > plane ? (size_t)L.stage_cells : plane;
  L.stage = take(sizeof(double) * NV * sb);
  if (p.tracer) {
    for (int q = 0; q < 3; ++q) L.t[q] = take(ncell * rs);
    L.fm = take(3 * ncell * rs);
    L.frout = take(plane * rs);
    L.ftend = take((size_t)g.n_r * g.n_phi * rs);
    for (int q = 0; q < 2; ++q) L.tg[q] = take(plane * rs);
  }
  L.total = off;
  return L;
}

int validate(const icr_grid* g, const icr_phys* p) {
  if (!g || !p) return fail(ICR_ERR_ARG, "grid and phys must not be NULL");
  if (g->n_r < 1 || g->n_theta < 1 || g->n_phi < 1)
    return fail(ICR_ERR_ARG, "cell counts must be >= 1 (got %d %d %d)", g->n_r, g->n_theta,
                g->n_phi);
  const double cells = (double)g->n_r * g->n_theta * g->n_phi;
  // the stage kernels address one variable's array with 32-bit byte offsets
  if (cells >= 536870912.0)
    return fail(ICR_ERR_ARG, "grid too large (%.0f cells, at most 2^29 - 1)", cells);
  if (!(g->r_in > 0 && g->r_out > g->r_in))
    return fail(ICR_ERR_ARG, "need 0 < r_in < r_out");
  if (!(g->th_min > 0 && g->th_max > g->th_min && g->th_max < kPi))
    return fail(ICR_ERR_ARG, "need 0 < th_min < th_max < pi");
  if (g->max_maps < 1 || g->max_cmes < 0 || g->max_probes < 0 || g->max_probes > 64 ||
      g->probe_log_rows < 0)
    return fail(ICR_ERR_ARG, "invalid capacities (max_maps >= 1, 0 <= max_probes <= 64)");
  if (g->max_probes > 0 && g->max_traj_pts < 2)
    return fail(ICR_ERR_ARG, "max_traj_pts must be >= 2 when probes are used");
  if (!(p->gamma > 1.0)) return fail(ICR_ERR_ARG, "gamma must be > 1");
  if (!(p->cfl > 0.0 && p->cfl <= 1.0)) return fail(ICR_ERR_ARG, "cfl must be in (0, 1]");
  if (!std::isfinite(p->omega)) return fail(ICR_ERR_ARG, "omega must be finite");
  if (p->flux != ICR_FLUX_TVDLF && p->flux != ICR_FLUX_HLL && p->flux != ICR_FLUX_HLLD)
    return fail(ICR_ERR_ARG, "unknown flux %d", p->flux);
  if (p->limiter != ICR_LIM_MINMOD && p->limiter != ICR_LIM_MC && p->limiter != ICR_LIM_WENO5)
    return fail(ICR_ERR_ARG, "unknown limiter %d", p->limiter);
  if (p->precision != ICR_PREC_F64 && p->precision != ICR_PREC_F32)
    return fail(ICR_ERR_ARG, "precision must be 64 or 32");
  if (p->tracer != 0 && p->tracer != 1) return fail(ICR_ERR_ARG, "tracer must be 0 or 1");
  if (p->bc_transverse != ICR_BCT_MAP && p->bc_transverse != ICR_BCT_ASYMM)
    return fail(ICR_ERR_ARG, "unknown bc_transverse %d", p->bc_transverse);
  const int ghost_width = p->limiter == ICR_LIM_WENO5 ? 3 : 2;
  if (p->bc_transverse == ICR_BCT_ASYMM && g->n_r < ghost_width)
    return fail(ICR_ERR_ARG, "asymm needs n_r >= %d (got %d)", ghost_width, g->n_r);
  return ICR_OK;
}

// ---- fixed device array of icr_step_noalloc --------------------------------
// The per-block CFL / residual / validity partials of the stage-2 kernel (4
// doubles per block) for callers that cannot allocate.  Each device holds
// its own copy from module load until the process ends; host code uses the
// address hipGetSymbolAddress returns for the current device, never the
// array's name.
constexpr int NOALLOC_MAX_BLOCKS = 32768;  // 1 MiB
static __device__ __align__(256) double scratch[4 * NOALLOC_MAX_BLOCKS];

constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[MAX_DEVICES] = {};

// Address of this device's scratch array (looked up once per device, with
// that device current).
int scratch_for_device(int dev, double** out) {
  if (dev < 0 || dev >= MAX_DEVICES) return fail(ICR_ERR_HIP, "device id %d out of range", dev);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(ICR_ERR_HIP, "hipGetSymbolAddress(scratch) failed: %s", hipGetErrorString(e));
    g_scratch_ptr[dev] = (double*)p;
  }
  *out = g_scratch_ptr[dev];
  return ICR_OK;
}

}  // namespace

namespace icr {
// The error channel of icr_last_error(), for the other host translation
// units of the library.
int set_error(int code, const char* msg) {
  g_err = msg;
  return code;
}
}  // namespace icr

struct icr_solver {
  icr_grid g;
  icr_phys p;
  Units un;
  bool f32;
  hipStream_t stream;      // caller's stream: all work and graph launches
  hipStream_t cap_stream;  // private stream used only to capture graphs
  char* ws;
  Layout L;
  int cur;                 // state buffer (0/1) holding the current state
  bool have_state, have_maps;
  int n_maps, n_cme, n_probes, n_pts;
  std::vector<double> tau_h;  // map times (code units) held on the device, ascending
  double cadence;
  double r_in, omega, gm, dph;
  int tile_r, variant, use_graphs, planes;
  hipGraphExec_t g_steps[NGRAPH][2];
  bool graphs_ok;
  int dev;                  // HIP device the solver was created on
  double* part_override;    // non-null: stage-2 partials go here (icr_step_noalloc)

  double* partials() { return part_override ? part_override : (double*)(ws + L.partials); }

  void* u(int q) { return ws + L.u[q]; }
  bool trc() const { return p.tracer != 0; }
  void* tr(int q) { return trc() ? ws + L.t[q] : nullptr; }
  void* tg(int q) { return trc() ? ws + L.tg[q] : nullptr; }
  void* ghost(int q) { return ws + L.g[q]; }
  double* m64() { return (double*)(ws + L.m64); }
  void* mr() { return ws + L.mr; }
  DevClock* clock() { return (DevClock*)(ws + L.clock); }
  long long ncell() const { return (long long)g.n_r * g.n_theta * g.n_phi; }
  // thread-per-cell launches (variant 1 and the CFL kernel)
  int v1_tile() const { return variant == 1 ? tile_r : 64; }
  dim3 block() const { return dim3(v1_tile(), 256 / v1_tile()); }
  dim3 grid() const {
    const int tr = v1_tile(), tt = 256 / tr;
    return dim3((g.n_r + tr - 1) / tr, (g.n_theta + tt - 1) / tt, g.n_phi);
  }
  int stage_blocks() const {
    if (variant == 1) {
      const dim3 gr = grid();
      return (int)(gr.x * gr.y * gr.z);
    }
    if (p.limiter == ICR_LIM_WENO5) return (int)stage_w5_blocks(g.n_r, g.n_theta, g.n_phi, planes);
    return (int)stage_lds_blocks(g.n_r, g.n_theta, g.n_phi, tile_r, planes);
  }

  BndArgs bnd() {
    BndArgs b;
    b.nt = g.n_theta;
    b.np = g.n_phi;
    b.n_maps = n_maps;
    b.tau = (const double*)(ws + L.tau);
    b.maps = (const double*)(ws + L.maps);
    b.n_cme = n_cme;
    b.cme = (const double*)(ws + L.cme);
    b.tc = m64() + OFF_TC64(g.n_r, g.n_theta);
    b.dph = dph;
    b.omega = omega;
    b.r_in = r_in;
    return b;
  }

  template <typename R>
  StageArgs<R> stage_args(int uin, int un_, int uout, int gh) {
    StageArgs<R> a;
    a.uin = (const R*)u(uin);
    a.un = (const R*)u(un_);
    a.uout = (R*)u(uout);
    a.ghost = (const R*)ghost(gh);
    a.m = metric_view<R>((const R*)mr(), g.n_r, g.n_theta, (g.th_max - g.th_min) / g.n_theta);
    a.clock = clock();
    a.partials = partials();
    a.nr = g.n_r;
    a.nt = g.n_theta;
    a.np = g.n_phi;
    a.ncell = ncell();
    a.gam = (R)p.gamma;
    a.gm1 = (R)(p.gamma - 1.0);
    a.igm1 = (R)(1.0 / (p.gamma - 1.0));
    a.omega = (R)omega;
    a.cfl = p.cfl;
    a.gravity = p.gravity ? 1 : 0;
    a.corot = p.corotation ? 1 : 0;
    a.asymm = p.bc_transverse == ICR_BCT_ASYMM ? 1 : 0;
    a.fmass = trc() ? (R*)(ws + L.fm) : nullptr;
    a.fmass_rout = trc() ? (R*)(ws + L.frout) : nullptr;
    a.fmass_tend = trc() ? (R*)(ws + L.ftend) : nullptr;
    return a;
  }

  // tracer stage: rho tau from buffer tin (density of state uin), combine
  // with tn in stage 2, into tout; inner ghost tau gh
  template <typename R>
  TracerArgs<R> tracer_args(int tin, int uin, int tn, int tout, int gh) {
    TracerArgs<R> a;
    a.tin = (const R*)tr(tin);
    a.tn = (const R*)tr(tn);
    a.tout = (R*)tr(tout);
    a.rho = (const R*)u(uin);  // variable 0 of the state is rho
    a.fm = (const R*)(ws + L.fm);
    a.frout = (const R*)(ws + L.frout);
    a.ftend = (const R*)(ws + L.ftend);
    a.gtau = (const R*)tg(gh);
    a.m = metric_view<R>((const R*)mr(), g.n_r, g.n_theta, (g.th_max - g.th_min) / g.n_theta);
    a.clock = clock();
    a.nr = g.n_r;
    a.nt = g.n_theta;
    a.np = g.n_phi;
    a.ncell = ncell();
    return a;
  }

  ProbeArgs probe_args() {
    ProbeArgs a;
    a.n = n_probes;
    a.npts = n_pts;
    a.max_probes = g.max_probes;
    a.log_rows = g.probe_log_rows;
    a.traj = (const double*)(ws + L.traj);
    a.cadence = cadence;
    a.sc = un.scale();
    a.omega = omega;
    a.gam = p.gamma;
    a.nr = g.n_r;
    a.nt = g.n_theta;
    a.np = g.n_phi;
    a.rc = m64() + 8LL * g.n_r;
    a.tc = m64() + OFF_TC64(g.n_r, g.n_theta);
    a.dph = dph;
    return a;
  }

  template <typename R>
  void enqueue_stages(int from, int to, hipStream_t st, hipEvent_t* ev) {
    const StageArgs<R> a1 = stage_args<R>(from, from, 2, 0);
    const StageArgs<R> a2 = stage_args<R>(2, from, to, 1);
    if (variant == 1)
      launch_stage<R>(a1, 1, p.flux, p.limiter, grid(), block(), st);
    else if (p.limiter == ICR_LIM_WENO5)
      launch_stage_w5<R>(a1, 1, p.flux, planes, st);
    else
      launch_stage_lds<R>(a1, 1, p.flux, p.limiter, tile_r, planes, st);
    if (trc()) launch_tracer<R>(tracer_args<R>(from, from, from, 2, 0), 1, st);
    if (ev) (void)hipEventRecord(ev[2], st);
    if (variant == 1)
      launch_stage<R>(a2, 2, p.flux, p.limiter, grid(), block(), st);
    else if (p.limiter == ICR_LIM_WENO5)
      launch_stage_w5<R>(a2, 2, p.flux, planes, st);
    else
      launch_stage_lds<R>(a2, 2, p.flux, p.limiter, tile_r, planes, st);
    if (trc()) launch_tracer<R>(tracer_args<R>(2, 2, from, to, 1), 2, st);
    if (ev) (void)hipEventRecord(ev[3], st);
    launch_finalize<R>(clock(), partials(), stage_blocks(), p.cfl, 1, logging() ? 1 : 0,
                       probe_args(), u(to), (double*)(ws + L.plog), st);
  }

  // One RK2 step from state buffer `from` into `from ^ 1`: boundary driver,
  // stage 1, stage 2, finalize (clock, dt, probe record).  ev (optional):
  // 5 events around the four kernels.
  void enqueue_step(int from, hipStream_t st, hipEvent_t* ev = nullptr) {
    const int to = from ^ 1;
    if (ev) (void)hipEventRecord(ev[0], st);
    launch_boundary(bnd(), clock(), ghost(0), ghost(1), tg(0), tg(1), f32, st);
    if (ev) (void)hipEventRecord(ev[1], st);
    if (f32)
      enqueue_stages<float>(from, to, st, ev);
    else
      enqueue_stages<double>(from, to, st, ev);
    if (ev) (void)hipEventRecord(ev[4], st);
  }

  bool logging() const { return n_probes > 0 && cadence >= 0.0 && g.probe_log_rows > 0; }

  void enqueue_cfl(hipStream_t st) {
    const dim3 gr(((unsigned)g.n_r + 63) / 64, ((unsigned)g.n_theta + 3) / 4, g.n_phi);
    const int nb = (int)(gr.x * gr.y * gr.z);
    const double* part = partials();
    if (f32) {
      launch_cfl<float>(stage_args<float>(cur, cur, cur, 0), gr, dim3(64, 4), st);
      launch_finalize<float>(clock(), part, nb, p.cfl, 0, 0, probe_args(), u(cur), nullptr, st);
    } else {
      launch_cfl<double>(stage_args<double>(cur, cur, cur, 0), gr, dim3(64, 4), st);
      launch_finalize<double>(clock(), part, nb, p.cfl, 0, 0, probe_args(), u(cur), nullptr, st);
    }
  }

  void drop_graphs() {
    if (!graphs_ok) return;
    for (int p = 0; p < NGRAPH; ++p)
      for (int q = 0; q < 2; ++q) (void)hipGraphExecDestroy(g_steps[p][q]);
    graphs_ok = false;
  }

  int capture(int from, int nsteps, hipGraphExec_t* out) {
    hipGraph_t graph;
    HIP_TRY(hipStreamBeginCapture(cap_stream, hipStreamCaptureModeThreadLocal));
    int f = from;
    for (int q = 0; q < nsteps; ++q) {
      enqueue_step(f, cap_stream);
      f ^= 1;
    }
    HIP_TRY(hipStreamEndCapture(cap_stream, &graph));
    hipError_t e = hipGraphInstantiate(out, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess)
      return fail(ICR_ERR_HIP, "hipGraphInstantiate failed: %s", hipGetErrorString(e));
    // upload now, so that the first replay does not carry the upload
    e = hipGraphUpload(*out, stream);
    if (e != hipSuccess)
      return fail(ICR_ERR_HIP, "hipGraphUpload failed: %s", hipGetErrorString(e));
    return ICR_OK;
  }

  int build_graphs() {
    if (graphs_ok) return ICR_OK;
    for (int p = 0; p < NGRAPH; ++p)
      for (int q = 0; q < 2; ++q) {
        const int rc = capture(q, GRAPH_STEPS[p], &g_steps[p][q]);
        if (rc) {  // release the graphs captured so far
          for (int pp = 0; pp <= p; ++pp)
            for (int qq = 0; qq < 2; ++qq)
              if (pp < p || qq < q) (void)hipGraphExecDestroy(g_steps[pp][qq]);
          return rc;
        }
      }
    graphs_ok = true;
    return ICR_OK;
  }

  int read_clock(DevClock* h) {
    HIP_TRY(hipMemcpyAsync(h, clock(), sizeof(DevClock), hipMemcpyDeviceToHost, stream));
    HIP_TRY(hipStreamSynchronize(stream));
    return ICR_OK;
  }
  int write_clock(const DevClock* h) {
    HIP_TRY(hipMemcpyAsync(clock(), h, sizeof(DevClock), hipMemcpyHostToDevice, stream));
    HIP_TRY(hipStreamSynchronize(stream));
    return ICR_OK;
  }
};

extern "C" {

const char* icr_last_error(void) { return g_err.c_str(); }

int icr_units(double* out) {
  if (!out) return fail(ICR_ERR_ARG, "out is NULL");
  Units u;
  out[0] = u.t;
  out[1] = u.len;
  out[2] = u.rho;
  out[3] = u.p;
  out[4] = u.b;
  out[5] = u.v;
  return ICR_OK;
}

int icr_workspace_bytes(const icr_grid* g, const icr_phys* p, size_t* bytes) {
  int rc = validate(g, p);
  if (rc) return rc;
  if (!bytes) return fail(ICR_ERR_ARG, "bytes is NULL");
  *bytes = make_layout(*g, *p).total;
  return ICR_OK;
}

int icr_create(const icr_grid* g, const icr_phys* p, void* ws, size_t ws_bytes, void* stream,
               icr_solver** out) {
  int rc = validate(g, p);
  if (rc) return rc;
  if (!out) return fail(ICR_ERR_ARG, "out is NULL");
  *out = nullptr;
  Layout L = make_layout(*g, *p);
  if (!ws || ws_bytes < L.total)
    return fail(ICR_ERR_ARG, "workspace too small: %zu < %zu bytes", ws_bytes, L.total);
  if (((uintptr_t)ws & 255) != 0) return fail(ICR_ERR_ARG, "workspace must be 256-byte aligned");
  icr_solver* s = new icr_solver();
  s->g = *g;
  s->p = *p;
  s->f32 = p->precision == ICR_PREC_F32;
  s->stream = (hipStream_t)stream;
  s->ws = (char*)ws;
  s->L = L;
  s->cur = 0;
  s->have_state = s->have_maps = false;
  s->n_maps = s->n_cme = s->n_probes = s->n_pts = 0;
  s->cadence = -1.0;
  s->r_in = g->r_in / s->un.len;
  s->omega = p->corotation ? p->omega * s->un.t : 0.0;
  s->gm = p->gravity ? kGM / (s->un.len * s->un.v * s->un.v) : 0.0;
  s->dph = 2.0 * kPi / g->n_phi;
  s->tile_r = 64;
  // WENO5 with the tracer: the thread-per-cell kernel (the WENO5 face-once
  // tile keeps no face mass fluxes)
  s->variant = (p->limiter == ICR_LIM_WENO5 && p->tracer) ? 1 : 2;
  s->planes = 8;
  s->use_graphs = 1;
  s->graphs_ok = false;
  s->part_override = nullptr;
  hipError_t e = hipGetDevice(&s->dev);
  if (e != hipSuccess) {
    delete s;
    return fail(ICR_ERR_HIP, "hipGetDevice failed: %s", hipGetErrorString(e));
  }
  {  // the fixed partials array of icr_step_noalloc on this device
    double* sp = nullptr;
    rc = scratch_for_device(s->dev, &sp);
    if (rc) {
      delete s;
      return rc;
    }
  }
  e = hipStreamCreateWithFlags(&s->cap_stream, hipStreamNonBlocking);
  if (e != hipSuccess) {
    delete s;
    return fail(ICR_ERR_HIP, "hipStreamCreate failed: %s", hipGetErrorString(e));
  }
  MetricArgs m;
  m.nr = g->n_r;
  m.nt = g->n_theta;
  m.r_in = s->r_in;
  m.r_out = g->r_out / s->un.len;
  m.q = std::pow(m.r_out / m.r_in, 1.0 / g->n_r);
  m.th_min = g->th_min;
  m.th_max = g->th_max;
  m.dph = s->dph;
  m.gm = s->gm;
  m.m64 = s->m64();
  launch_metric(m, s->mr(), s->f32, s->stream);
  DevClock c;
  std::memset(&c, 0, sizeof c);
  c.bad = BAD_NONE;
  c.t_end = -1.0;
  c.last_sample = -1;
  rc = s->write_clock(&c);
  if (rc) {
    (void)hipStreamDestroy(s->cap_stream);
    delete s;
    return rc;
  }
  e = hipGetLastError();
  if (e != hipSuccess) {
    (void)hipStreamDestroy(s->cap_stream);
    delete s;
    return fail(ICR_ERR_HIP, "metric kernel launch failed: %s", hipGetErrorString(e));
  }
  *out = s;
  return ICR_OK;
}

void icr_destroy(icr_solver* s) {
  if (!s) return;
  (void)hipStreamSynchronize(s->stream);
  s->drop_graphs();
  (void)hipStreamDestroy(s->cap_stream);
  delete s;
}

int icr_grid_edges(const icr_solver* s, double* r, double* t, double* ph) {
  if (!s) return fail(ICR_ERR_ARG, "solver is NULL");
  icr_solver* m = const_cast<icr_solver*>(s);
  const int nr = s->g.n_r, nt = s->g.n_theta, np = s->g.n_phi;
  if (r) {
    HIP_TRY(hipMemcpyAsync(r, m->m64() + OFF_REDGE64(nr, nt), sizeof(double) * (nr + 1),
                           hipMemcpyDeviceToHost, s->stream));
    HIP_TRY(hipStreamSynchronize(s->stream));
    for (int i = 0; i <= nr; ++i) r[i] *= s->un.len;
  }
  if (t)
    for (int j = 0; j <= nt; ++j)
      t[j] = s->g.th_min + (s->g.th_max - s->g.th_min) * (double)j / nt;
  if (ph)
    for (int k = 0; k <= np; ++k) ph[k] = 2.0 * kPi * (double)k / np;
  return ICR_OK;
}

namespace {
// Copy n SI maps [n][8][nt][np] (host or device) into h in code units,
// checking rho > 0, p > 0 and finiteness.
int stage_maps(icr_solver* s, int n, const double* maps, int on_device, std::vector<double>& h) {
  const size_t plane = (size_t)s->g.n_theta * s->g.n_phi;
  h.resize((size_t)n * NV * plane);
  if (on_device) {
    HIP_TRY(hipMemcpyAsync(h.data(), maps, h.size() * sizeof(double), hipMemcpyDeviceToHost,
                           s->stream));
    HIP_TRY(hipStreamSynchronize(s->stream));
  } else {
    std::memcpy(h.data(), maps, h.size() * sizeof(double));
  }
  const Scale sc = s->un.scale();
  for (int m = 0; m < n; ++m)
    for (int v = 0; v < NV; ++v)
      for (size_t q = 0; q < plane; ++q) {
        double& x = h[((size_t)m * NV + v) * plane + q];
        if ((v == 0 || v == 4) && !(x > 0.0))
          return fail(ICR_ERR_ARG, "map %d has %s <= 0 at point %zu", m, v ? "p" : "rho", q);
        if (!std::isfinite(x)) return fail(ICR_ERR_ARG, "map %d has a non-finite value", m);
        x /= sc.s[v];
      }
  return ICR_OK;
}
}  // namespace

int icr_set_boundary_maps(icr_solver* s, int n, const double* t_s, const double* maps,
                          int on_device) {
  if (!s) return fail(ICR_ERR_ARG, "solver is NULL");
  if (n < 1 || n > s->g.max_maps)
    return fail(ICR_ERR_ARG, "n_maps = %d outside [1, %d]", n, s->g.max_maps);
  if (!t_s || !maps) return fail(ICR_ERR_ARG, "t_s and maps must not be NULL");
  for (int q = 1; q < n; ++q)
    if (!(t_s[q] > t_s[q - 1])) return fail(ICR_ERR_ARG, "map times must ascend strictly");
  std::vector<double> h;
  int rc = stage_maps(s, n, maps, on_device, h);
  if (rc) return rc;
  std::vector<double> tau(n);
  for (int m = 0; m < n; ++m) tau[m] = t_s[m] / s->un.t;
  HIP_TRY(hipMemcpyAsync(s->ws + s->L.maps, h.data(), h.size() * sizeof(double),
                         hipMemcpyHostToDevice, s->stream));
  HIP_TRY(hipMemcpyAsync(s->ws + s->L.tau, tau.data(), n * sizeof(double), hipMemcpyHostToDevice,
                         s->stream));
  HIP_TRY(hipStreamSynchronize(s->stream));
  s->tau_h = tau;
  s->n_maps = n;
  s->have_maps = true;
  s->drop_graphs();
  return ICR_OK;
}

int icr_append_boundary_maps(icr_solver* s, int n, const double* t_s, const double* maps,
                             int on_device, int* n_held) {
  if (!s) return fail(ICR_ERR_ARG, "solver is NULL");
  if (!s->have_maps) return fail(ICR_ERR_STATE, "set the first maps with icr_set_boundary_maps");
  if (n < 1) return fail(ICR_ERR_ARG, "n = %d < 1", n);
  if (!t_s || !maps) return fail(ICR_ERR_ARG, "t_s and maps must not be NULL");
  const double last = s->tau_h.back() * s->un.t;
  for (int q = 0; q < n; ++q)
    if (!(t_s[q] > (q ? t_s[q - 1] : last)))
      return fail(ICR_ERR_ARG, "appended map times must ascend strictly after %.17g s", last);
  // maps strictly before the last map time <= t can no longer bracket any
  // time from the clock on
  DevClock c;
  int rc = s->read_clock(&c);
  if (rc) return rc;
  int keep = 0;
  while (keep + 1 < s->n_maps && s->tau_h[keep + 1] <= c.t) ++keep;
  const int held = s->n_maps - keep;
  if (held + n > s->g.max_maps)
    return fail(ICR_ERR_STATE,
                "map buffer full: %d maps still bracket t >= %.6g s, %d more do not fit in "
                "max_maps = %d (step further first)",
                held, c.t * s->un.t, n, s->g.max_maps);
  std::vector<double> h;
  rc = stage_maps(s, n, maps, on_device, h);
  if (rc) return rc;
  const size_t mbytes = sizeof(double) * NV * (size_t)s->g.n_theta * s->g.n_phi;
  char* base = s->ws + s->L.maps;
  for (int q = 0; q < held && keep > 0; ++q)  // slot keep + q -> q (disjoint slots)
    HIP_TRY(hipMemcpyAsync(base + q * mbytes, base + (size_t)(keep + q) * mbytes, mbytes,
                           hipMemcpyDeviceToDevice, s->stream));
  HIP_TRY(hipMemcpyAsync(base + (size_t)held * mbytes, h.data(), h.size() * sizeof(double),
                         hipMemcpyHostToDevice, s->stream));
  std::vector<double> tau(s->tau_h.begin() + keep, s->tau_h.end());
  for (int q = 0; q < n; ++q) tau.push_back(t_s[q] / s->un.t);
  HIP_TRY(hipMemcpyAsync(s->ws + s->L.tau, tau.data(), tau.size() * sizeof(double),
                         hipMemcpyHostToDevice, s->stream));
  HIP_TRY(hipStreamSynchronize(s->stream));
  s->tau_h = tau;
  s->n_maps = (int)tau.size();
  s->drop_graphs();
  if (n_held) *n_held = s->n_maps;
  return ICR_OK;
}

int icr_set_cmes(icr_solver* s, int n, const double* rows) {
  if (!s) return fail(ICR_ERR_ARG, "solver is NULL");
  if (n < 0 || n > s->g.max_cmes)
    return fail(ICR_ERR_ARG, "n = %d outside [0, %d]", n, s->g.max_cmes);
  if (n > 0 && !rows) return fail(ICR_ERR_ARG, "rows is NULL");
  std::vector<double> c((size_t)8 * (n > 0 ? n : 1));
  for (int q = 0; q < n; ++q) {
    const double* r = rows + 8 * q;
    if (!(r[1] > 0 && r[4] > 0 && r[5] > 0 && r[6] > 0 && r[7] > 0))
      return fail(ICR_ERR_ARG, "CME %d: duration, half-width, speed, density, T must be > 0", q);
    double* d = c.data() + 8 * q;
    d[0] = r[0] / s->un.t;
    d[1] = r[1] / s->un.t;
    d[2] = 0.5 * kPi - r[2];
    d[3] = r[3];
    d[4] = std::cos(r[4]);
    d[5] = r[5] / s->un.v;
    d[6] = r[6] / s->un.rho;
    d[7] = 2.0 * (r[6] / kMp) * kKb * r[7] / s->un.p;
  }
  if (n > 0) {
    HIP_TRY(hipMemcpyAsync(s->ws + s->L.cme, c.data(), 8 * n * sizeof(double),
                           hipMemcpyHostToDevice, s->stream));
    HIP_TRY(hipStreamSynchronize(s->stream));
  }
  s->n_cme = n;
  s->drop_graphs();
  return ICR_OK;
}

static int refresh_dt(icr_solver* s) {
  s->enqueue_cfl(s->stream);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipStreamSynchronize(s->stream));
  return ICR_OK;
}

int icr_init_radial(icr_solver* s) {
  if (!s) return fail(ICR_ERR_ARG, "solver is NULL");
  if (!s->have_maps) return fail(ICR_ERR_STATE, "set boundary maps first");
  if (s->f32)
    launch_init_radial<float>(s->bnd(), s->m64(), s->u(s->cur), s->g.n_r, s->p.gamma, s->stream);
  else
    launch_init_radial<double>(s->bnd(), s->m64(), s->u(s->cur), s->g.n_r, s->p.gamma,
                               s->stream);
  HIP_TRY(hipGetLastError());
  if (s->trc())
    HIP_TRY(hipMemsetAsync(s->tr(s->cur), 0, (s->f32 ? 4 : 8) * (size_t)s->ncell(), s->stream));
  DevClock c;
  int rc = s->read_clock(&c);
  if (rc) return rc;
  c.t = 0.0;
  c.step = 0;
  c.bad = BAD_NONE;
  c.counter = 0;
  c.last_dt = 0.0;
  c.resid = 0.0;
  rc = s->write_clock(&c);
  if (rc) return rc;
  s->have_state = true;
  return refresh_dt(s);
}

int icr_set_state(icr_solver* s, const double* data, int kind, int on_device) {
  if (!s) return fail(ICR_ERR_ARG, "solver is NULL");
  if (!data) return fail(ICR_ERR_ARG, "data is NULL");
  if (kind != ICR_STATE_PRIM_SI && kind != ICR_STATE_CONS_CODE)
    return fail(ICR_ERR_ARG, "unknown state kind %d", kind);
  const long long n = s->ncell();
  const Scale sc = s->un.scale();
  void* u = s->u(s->cur);
  if (on_device) {
    if (s->f32)
      launch_import<float>(data, n, u, n, 0, n, kind, sc, s->p.gamma, s->stream);
    else
      launch_import<double>(data, n, u, n, 0, n, kind, sc, s->p.gamma, s->stream);
    HIP_TRY(hipGetLastError());
  } else {
    // host data: chunks of stage_cells cells through the staging region
    double* st = (double*)(s->ws + s->L.stage);
    const long long cm = s->L.stage_cells;
    for (long long c0 = 0; c0 < n; c0 += cm) {
      const long long m = n - c0 < cm ? n - c0 : cm;
      HIP_TRY(hipMemcpy2DAsync(st, sizeof(double) * m, data + c0, sizeof(double) * n,
                               sizeof(double) * m, NV, hipMemcpyHostToDevice, s->stream));
      if (s->f32)
        launch_import<float>(st, m, u, n, c0, m, kind, sc, s->p.gamma, s->stream);
      else
        launch_import<double>(st, m, u, n, c0, m, kind, sc, s->p.gamma, s->stream);
      HIP_TRY(hipGetLastError());
    }
  }
  if (s->trc()) HIP_TRY(hipMemsetAsync(s->tr(s->cur), 0, (s->f32 ? 4 : 8) * (size_t)n, s->stream));
  hipError_t e = hipStreamSynchronize(s->stream);
  if (e != hipSuccess) return fail(ICR_ERR_HIP, "state import failed: %s", hipGetErrorString(e));
  DevClock c;
  int rc = s->read_clock(&c);
  if (rc) return rc;
  c.bad = BAD_NONE;
  c.counter = 0;
  rc = s->write_clock(&c);
  if (rc) return rc;
  s->have_state = true;
  return refresh_dt(s);
}

int icr_get_state(icr_solver* s, double* out, int kind, int on_device) {
  if (!s) return fail(ICR_ERR_ARG, "solver is NULL");
  if (!out) return fail(ICR_ERR_ARG, "out is NULL");
  if (kind != ICR_STATE_PRIM_SI && kind != ICR_STATE_CONS_CODE)
    return fail(ICR_ERR_ARG, "unknown state kind %d", kind);
  if (!s->have_state) return fail(ICR_ERR_STATE, "no state yet");
  const long long n = s->ncell();
  const Scale sc = s->un.scale();
  const void* u = s->u(s->cur);
  if (on_device) {
    if (s->f32)
      launch_export<float>(u, n, 0, n, out, n, kind, sc, s->p.gamma, s->stream);
    else
      launch_export<double>(u, n, 0, n, out, n, kind, sc, s->p.gamma, s->stream);
    HIP_TRY(hipGetLastError());
  } else {
    double* st = (double*)(s->ws + s->L.stage);
    const long long cm = s->L.stage_cells;
    for (long long c0 = 0; c0 < n; c0 += cm) {
      const long long m = n - c0 < cm ? n - c0 : cm;
      if (s->f32)
        launch_export<float>(u, n, c0, m, st, m, kind, sc, s->p.gamma, s->stream);
      else
        launch_export<double>(u, n, c0, m, st, m, kind, sc, s->p.gamma, s->stream);
      HIP_TRY(hipGetLastError());
      HIP_TRY(hipMemcpy2DAsync(out + c0, sizeof(double) * n, st, sizeof(double) * m,
                               sizeof(double) * m, NV, hipMemcpyDeviceToHost, s->stream));
    }
  }
  hipError_t e = hipStreamSynchronize(s->stream);
  if (e != hipSuccess) return fail(ICR_ERR_HIP, "state export failed: %s", hipGetErrorString(e));
  return ICR_OK;
}

int icr_get_clock(icr_solver* s, icr_clock* out) {
  if (!s || !out) return fail(ICR_ERR_ARG, "NULL argument");
  DevClock c;
  int rc = s->read_clock(&c);
  if (rc) return rc;
  out->t = c.t * s->un.t;
  out->step = c.step;
  out->last_dt = c.last_dt * s->un.t;
  out->next_dt = c.dt_cfl * s->un.t;
  out->residual = c.resid;
  out->t_code = c.t;
  return ICR_OK;
}

static int set_clock_code(icr_solver* s, double tc, long long step) {
  DevClock c;
  int rc = s->read_clock(&c);
  if (rc) return rc;
  c.t = tc;
  c.step = step;
  if (s->cadence > 0.0) c.last_sample = (long long)std::floor(tc * s->un.t / s->cadence);
  return s->write_clock(&c);
}

int icr_set_clock(icr_solver* s, double t, long long step) {
  if (!s) return fail(ICR_ERR_ARG, "solver is NULL");
  if (!std::isfinite(t) || step < 0) return fail(ICR_ERR_ARG, "invalid clock");
  return set_clock_code(s, t / s->un.t, step);
}

int icr_set_clock_code(icr_solver* s, double t_code, long long step) {
  if (!s) return fail(ICR_ERR_ARG, "solver is NULL");
  if (!std::isfinite(t_code) || step < 0) return fail(ICR_ERR_ARG, "invalid clock");
  return set_clock_code(s, t_code, step);
}

static int step_report(icr_solver* s, icr_step_info* info) {
  HIP_TRY(hipGetLastError());
  DevClock c;
  int rc = s->read_clock(&c);
  if (rc) return rc;
  if (info) {
    info->steps_taken = (int)c.taken;
    info->status = c.bad == BAD_NONE ? ICR_OK : ICR_ERR_NONPHYSICAL;
    info->bad_cell = c.bad == BAD_NONE ? -1 : c.bad;
    info->t = c.t * s->un.t;
    info->last_dt = c.last_dt * s->un.t;
    info->residual = c.resid;
  }
  if (c.bad != BAD_NONE)
    return fail(ICR_ERR_NONPHYSICAL, "non-physical cell %d after step %lld", c.bad, c.step);
  return ICR_OK;
}

int icr_step_noalloc(icr_solver* s, int n, double t_end_s, icr_step_info* info) {
  if (!s) return fail(ICR_ERR_ARG, "solver is NULL");
  if (n < 0) return fail(ICR_ERR_ARG, "n_steps must be >= 0");
  if (!s->have_maps) return fail(ICR_ERR_STATE, "set boundary maps first");
  if (!s->have_state) return fail(ICR_ERR_STATE, "initialise the state first");
  const int nb = s->stage_blocks();
  if (nb > NOALLOC_MAX_BLOCKS)
    return fail(ICR_ERR_ARG,
                "icr_step_noalloc: the stage launch has %d blocks, the fixed partials array "
                "holds %d (use more phi planes per block or icr_step)",
                nb, NOALLOC_MAX_BLOCKS);
  int dev = -1;
  HIP_TRY(hipGetDevice(&dev));
  if (dev != s->dev)
    return fail(ICR_ERR_ARG, "icr_step_noalloc: solver of device %d called with device %d "
                "current", s->dev, dev);
  double* sp = nullptr;
  int rc = scratch_for_device(s->dev, &sp);  // looked up at creation: no lookup here
  if (rc) return rc;
  const double tend = t_end_s > 0.0 ? t_end_s / s->un.t : -1.0;
  launch_clock_begin(s->clock(), tend, s->stream);
  // direct launches (no graph instantiation), partials in the fixed array;
  // every stage-2 block writes its slot before the finalize kernel reads it,
  // so nothing needs clearing between calls
  s->part_override = sp;
  for (int q = 0; q < n; ++q) {
    s->enqueue_step(s->cur, s->stream);
    s->cur ^= 1;
  }
  s->part_override = nullptr;
  return step_report(s, info);
}

int icr_step(icr_solver* s, int n, double t_end_s, icr_step_info* info) {
  if (!s) return fail(ICR_ERR_ARG, "solver is NULL");
  if (n < 0) return fail(ICR_ERR_ARG, "n_steps must be >= 0");
  if (!s->have_maps) return fail(ICR_ERR_STATE, "set boundary maps first");
  if (!s->have_state) return fail(ICR_ERR_STATE, "initialise the state first");
  const double tend = t_end_s > 0.0 ? t_end_s / s->un.t : -1.0;
  launch_clock_begin(s->clock(), tend, s->stream);
  if (s->use_graphs && n > 0) {
    int rc = s->build_graphs();
    if (rc) return rc;
    int left = n;
    for (int p = 0; p < NGRAPH; ++p)
      while (left >= GRAPH_STEPS[p] && (p == 0 || (left & GRAPH_STEPS[p]))) {
        HIP_TRY(hipGraphLaunch(s->g_steps[p][s->cur], s->stream));
        s->cur ^= GRAPH_STEPS[p] & 1;  // an even number of steps keeps the buffer
        left -= GRAPH_STEPS[p];
      }
  } else {
    for (int q = 0; q < n; ++q) {
      s->enqueue_step(s->cur, s->stream);
      s->cur ^= 1;
    }
  }
  return step_report(s, info);
}

int icr_set_probes(icr_solver* s, int n, int npts, const double* traj, double cadence) {
  if (!s) return fail(ICR_ERR_ARG, "solver is NULL");
  if (n < 0 || n > s->g.max_probes)
    return fail(ICR_ERR_ARG, "n = %d outside [0, %d]", n, s->g.max_probes);
  if (n > 0) {
    if (npts < 2 || npts > s->g.max_traj_pts)
      return fail(ICR_ERR_ARG, "n_pts = %d outside [2, %d]", npts, s->g.max_traj_pts);
    if (!traj) return fail(ICR_ERR_ARG, "traj is NULL");
    if (s->g.n_r < 2 || s->g.n_theta < 2)
      return fail(ICR_ERR_ARG, "probes need n_r >= 2 and n_theta >= 2");
    for (int q = 0; q < n; ++q)
      for (int m = 1; m < npts; ++m)
        if (!(traj[((size_t)q * npts + m) * 4] > traj[((size_t)q * npts + m - 1) * 4]))
          return fail(ICR_ERR_ARG, "trajectory %d: times must ascend strictly", q);
    HIP_TRY(hipMemcpyAsync(s->ws + s->L.traj, traj, sizeof(double) * 4 * (size_t)n * npts,
                           hipMemcpyHostToDevice, s->stream));
  }
  s->n_probes = n;
  s->n_pts = npts;
  s->cadence = cadence;
  DevClock c;
  int rc = s->read_clock(&c);
  if (rc) return rc;
  c.n_log = 0;
  c.advanced = 0;
  c.last_sample = cadence > 0.0 ? (long long)std::floor(c.t * s->un.t / cadence) : -1;
  rc = s->write_clock(&c);
  if (rc) return rc;
  s->drop_graphs();
  return ICR_OK;
}

int icr_sample_probes(icr_solver* s, double* out) {
  if (!s || !out) return fail(ICR_ERR_ARG, "NULL argument");
  if (!s->have_state) return fail(ICR_ERR_STATE, "no state yet");
  if (s->n_probes == 0) return ICR_OK;
  double* pout = (double*)(s->ws + s->L.pout);
  if (s->f32)
    launch_probe_sample<float>(s->probe_args(), s->clock(), s->u(s->cur), pout, s->stream);
  else
    launch_probe_sample<double>(s->probe_args(), s->clock(), s->u(s->cur), pout, s->stream);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipMemcpyAsync(out, pout, sizeof(double) * 12 * s->n_probes, hipMemcpyDeviceToHost,
                         s->stream));
  HIP_TRY(hipStreamSynchronize(s->stream));
  return ICR_OK;
}

int icr_read_probe_log(icr_solver* s, double* out, int cap, int* n_rec) {
  if (!s || !n_rec) return fail(ICR_ERR_ARG, "NULL argument");
  if (cap > 0 && !out) return fail(ICR_ERR_ARG, "out is NULL");
  DevClock c;
  int rc = s->read_clock(&c);
  if (rc) return rc;
  *n_rec = (int)c.n_log;
  long long rows = c.n_log;
  if (rows > s->g.probe_log_rows) rows = s->g.probe_log_rows;
  if (rows > cap) rows = cap;
  if (rows > 0 && s->n_probes > 0) {
    // log rows are [max_probes][12]; copy the first n_probes of each
    const size_t row_b = sizeof(double) * 12 * s->g.max_probes;
    std::vector<double> h((size_t)rows * 12 * s->g.max_probes);
    HIP_TRY(hipMemcpyAsync(h.data(), s->ws + s->L.plog, rows * row_b, hipMemcpyDeviceToHost,
                           s->stream));
    HIP_TRY(hipStreamSynchronize(s->stream));
    for (long long r = 0; r < rows; ++r)
      std::memcpy(out + r * 12 * s->n_probes, h.data() + r * 12 * s->g.max_probes,
                  sizeof(double) * 12 * s->n_probes);
  }
  return ICR_OK;
}

int icr_boundary_at(icr_solver* s, double t_s, double* out) {
  if (!s || !out) return fail(ICR_ERR_ARG, "NULL argument");
  if (!s->have_maps) return fail(ICR_ERR_STATE, "set boundary maps first");
  double* d = (double*)(s->ws + s->L.stage);
  launch_boundary_at(s->bnd(), t_s / s->un.t, d, s->un.scale(), s->stream);
  HIP_TRY(hipGetLastError());
  const size_t bytes = sizeof(double) * NV * s->g.n_theta * s->g.n_phi;
  HIP_TRY(hipMemcpyAsync(out, d, bytes, hipMemcpyDeviceToHost, s->stream));
  HIP_TRY(hipStreamSynchronize(s->stream));
  return ICR_OK;
}

int icr_sample_shell(icr_solver* s, double r_m, double* out) {
  if (!s || !out) return fail(ICR_ERR_ARG, "NULL argument");
  if (!s->have_state) return fail(ICR_ERR_STATE, "no state yet");
  if (!(r_m > 0.0)) return fail(ICR_ERR_ARG, "r must be > 0");
  const int nt = s->g.n_theta, np = s->g.n_phi;
  // the staging region holds [8][nt][np] doubles; the shell needs [2][nt][np]
  double* d = (double*)(s->ws + s->L.stage);
  const double* rc = s->m64() + 8LL * s->g.n_r;
  if (s->f32)
    launch_shell<float>(s->u(s->cur), rc, s->g.n_r, nt, np, r_m / s->un.len, s->p.gamma,
                        s->un.scale(), d, s->stream);
  else
    launch_shell<double>(s->u(s->cur), rc, s->g.n_r, nt, np, r_m / s->un.len, s->p.gamma,
                         s->un.scale(), d, s->stream);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipMemcpyAsync(out, d, sizeof(double) * 2 * nt * np, hipMemcpyDeviceToHost, s->stream));
  HIP_TRY(hipStreamSynchronize(s->stream));
  return ICR_OK;
}

int icr_set_tracer(icr_solver* s, const double* tau, int on_device) {
  if (!s || !tau) return fail(ICR_ERR_ARG, "NULL argument");
  if (!s->trc()) return fail(ICR_ERR_STATE, "solver created without the tracer");
  if (!s->have_state) return fail(ICR_ERR_STATE, "set the state first");
  const long long n = s->ncell();
  if (on_device) {
    if (s->f32)
      launch_tracer_io<float>(s->u(s->cur), s->tr(s->cur), (double*)tau, 0, n, 1, s->stream);
    else
      launch_tracer_io<double>(s->u(s->cur), s->tr(s->cur), (double*)tau, 0, n, 1, s->stream);
    HIP_TRY(hipGetLastError());
  } else {
    double* st = (double*)(s->ws + s->L.stage);
    const long long cm = s->L.stage_cells;
    for (long long c0 = 0; c0 < n; c0 += cm) {
      const long long m = n - c0 < cm ? n - c0 : cm;
      HIP_TRY(hipMemcpyAsync(st, tau + c0, sizeof(double) * m, hipMemcpyHostToDevice, s->stream));
      if (s->f32)
        launch_tracer_io<float>(s->u(s->cur), s->tr(s->cur), st, c0, m, 1, s->stream);
      else
        launch_tracer_io<double>(s->u(s->cur), s->tr(s->cur), st, c0, m, 1, s->stream);
      HIP_TRY(hipGetLastError());
    }
  }
  hipError_t e = hipStreamSynchronize(s->stream);
  if (e != hipSuccess) return fail(ICR_ERR_HIP, "tracer import failed: %s", hipGetErrorString(e));
  return ICR_OK;
}

int icr_get_tracer(icr_solver* s, double* tau, int on_device) {
  if (!s || !tau) return fail(ICR_ERR_ARG, "NULL argument");
  if (!s->trc()) return fail(ICR_ERR_STATE, "solver created without the tracer");
  if (!s->have_state) return fail(ICR_ERR_STATE, "no state yet");
  const long long n = s->ncell();
  if (on_device) {
    if (s->f32)
      launch_tracer_io<float>(s->u(s->cur), s->tr(s->cur), tau, 0, n, 0, s->stream);
    else
      launch_tracer_io<double>(s->u(s->cur), s->tr(s->cur), tau, 0, n, 0, s->stream);
    HIP_TRY(hipGetLastError());
  } else {
    double* st = (double*)(s->ws + s->L.stage);
    const long long cm = s->L.stage_cells;
    for (long long c0 = 0; c0 < n; c0 += cm) {
      const long long m = n - c0 < cm ? n - c0 : cm;
      if (s->f32)
        launch_tracer_io<float>(s->u(s->cur), s->tr(s->cur), st, c0, m, 0, s->stream);
      else
        launch_tracer_io<double>(s->u(s->cur), s->tr(s->cur), st, c0, m, 0, s->stream);
      HIP_TRY(hipGetLastError());
      HIP_TRY(hipMemcpyAsync(tau + c0, st, sizeof(double) * m, hipMemcpyDeviceToHost, s->stream));
    }
  }
  hipError_t e = hipStreamSynchronize(s->stream);
  if (e != hipSuccess) return fail(ICR_ERR_HIP, "tracer export failed: %s", hipGetErrorString(e));
  return ICR_OK;
}

int icr_divv(icr_solver* s, double* out, int on_device) {
  if (!s || !out) return fail(ICR_ERR_ARG, "NULL argument");
  if (!s->have_state || !s->have_maps) return fail(ICR_ERR_STATE, "maps and state first");
  const long long n = s->ncell();
  const double inv_t = 1.0 / s->un.t;
  // host output: chunks through the staging region
  const long long cm = on_device ? n : s->L.stage_cells;
  double* st = (double*)(s->ws + s->L.stage);
  for (long long c0 = 0; c0 < n; c0 += cm) {
    const long long m = n - c0 < cm ? n - c0 : cm;
    double* dst = on_device ? out : st;
    if (s->f32)
      launch_divv<float>(s->stage_args<float>(s->cur, s->cur, s->cur, 0), s->bnd(), inv_t, c0, m,
                         dst, s->stream);
    else
      launch_divv<double>(s->stage_args<double>(s->cur, s->cur, s->cur, 0), s->bnd(), inv_t, c0,
                          m, dst, s->stream);
    HIP_TRY(hipGetLastError());
    if (!on_device)
      HIP_TRY(hipMemcpyAsync(out + c0, st, sizeof(double) * m, hipMemcpyDeviceToHost, s->stream));
  }
  hipError_t e = hipStreamSynchronize(s->stream);
  if (e != hipSuccess) return fail(ICR_ERR_HIP, "divergence failed: %s", hipGetErrorString(e));
  return ICR_OK;
}

int icr_profile_steps(icr_solver* s, int n, double* avg_ms) {
  if (!s || !avg_ms) return fail(ICR_ERR_ARG, "NULL argument");
  if (n < 1) return fail(ICR_ERR_ARG, "n_steps must be >= 1");
  if (!s->have_maps || !s->have_state) return fail(ICR_ERR_STATE, "maps and state first");
  hipEvent_t ev[5];
  for (int q = 0; q < 5; ++q) HIP_TRY(hipEventCreate(&ev[q]));
  double acc[4] = {0, 0, 0, 0};
  launch_clock_begin(s->clock(), -1.0, s->stream);
  int rc = ICR_OK;
  for (int q = 0; q < n && rc == ICR_OK; ++q) {
    s->enqueue_step(s->cur, s->stream, ev);
    s->cur ^= 1;
    if (hipEventSynchronize(ev[4]) != hipSuccess) {
      rc = fail(ICR_ERR_HIP, "event synchronisation failed");
      break;
    }
    for (int k = 0; k < 4; ++k) {
      float ms = 0.f;
      (void)hipEventElapsedTime(&ms, ev[k], ev[k + 1]);
      acc[k] += ms;
    }
  }
  for (int q = 0; q < 5; ++q) (void)hipEventDestroy(ev[q]);
  for (int k = 0; k < 4; ++k) avg_ms[k] = acc[k] / n;
  return rc;
}

int icr_fast_math(const double* x, long long n, double* rcp, double* sq, void* stream) {
  if (n < 0) return fail(ICR_ERR_ARG, "n must be >= 0");
  if (n > 0 && (!x || !rcp || !sq)) return fail(ICR_ERR_ARG, "NULL argument");
  if (n == 0) return ICR_OK;
  launch_fast_math(x, n, rcp, sq, (hipStream_t)stream);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipStreamSynchronize((hipStream_t)stream));
  return ICR_OK;
}

int icr_set_launch(icr_solver* s, int variant, int tile_r, int planes, int use_graphs) {
  if (!s) return fail(ICR_ERR_ARG, "solver is NULL");
  if (variant == 0) variant = 2;
  if (s->p.limiter == ICR_LIM_WENO5) {
    // the WENO5 face-once tile is 64 x 4; with the tracer only the
    // thread-per-cell kernel runs WENO5
    if (s->trc()) variant = 1;
    if (variant == 1 && tile_r != 64 && tile_r != 128 && tile_r != 256) tile_r = 64;
    if (variant == 2) tile_r = 64;
  }
  if (variant != 1 && variant != 2) return fail(ICR_ERR_ARG, "variant must be 0, 1 or 2");
  if (tile_r == 0) tile_r = 64;
  if (variant == 1 && tile_r != 64 && tile_r != 128 && tile_r != 256)
    return fail(ICR_ERR_ARG, "variant 1 tile_r must be 64, 128 or 256 (got %d)", tile_r);
  if (variant == 2 && tile_r != 32 && tile_r != 64)
    return fail(ICR_ERR_ARG, "variant 2 tile_r must be 32 or 64 (got %d)", tile_r);
  if (planes == 0) planes = 8;
  if (planes < 1 || planes > s->g.n_phi)
    return fail(ICR_ERR_ARG, "planes must be in [1, n_phi] (got %d)", planes);
  if (variant == 2 && s->trc()) tile_r = 64;  // the tracer's flux stores exist for 64 x 4
  s->variant = variant;
  s->tile_r = tile_r;
  s->planes = planes;
  s->use_graphs = use_graphs ? 1 : 0;
  s->drop_graphs();
  return ICR_OK;
}

}  // extern "C"

// ======================================================================
// Batched ensemble
// ======================================================================
struct icr_ensemble {
  int n;
  icr_phys p;
  bool f32;
  hipStream_t stream, cap_stream;
  char* ws;
  size_t table_bytes;
  std::vector<icr_solver*> runs;
  std::vector<int> planes;
  // device tables
  void* d_runs;
  int* d_tile_off;
  int* d_bnd_off;
  int* d_trc_off;
  GridBar* d_bar;
  DevClock** d_clocks;
  DevClock* d_gather;
  int n_tiles, n_bitems, n_titems;
  int persistent, grid, use_graphs;
  long long spin_limit;
  hipGraphExec_t g_chunk;
  bool graph_ok;
  int graph_n;
};

namespace {

size_t ens_table_bytes(int n) {
  size_t b = 0;
  b += align_up(sizeof(RunDesc<double>) * n);
  b += 3 * align_up(sizeof(int) * (n + 1));
  b += align_up(sizeof(GridBar));
  b += align_up(sizeof(DevClock*) * n);
  b += align_up(sizeof(DevClock) * n);
  return b;
}

template <typename R>
RunDesc<R> make_desc(icr_solver* s, int planes) {
  RunDesc<R> d;
  for (int p = 0; p < 2; ++p) {
    d.s1[p] = s->stage_args<R>(p, p, 2, 0);
    d.s2[p] = s->stage_args<R>(2, p, p ^ 1, 1);
  }
  for (int p = 0; p < 2; ++p) {
    if (s->trc()) {
      d.t1[p] = s->tracer_args<R>(p, p, p, 2, 0);
      d.t2[p] = s->tracer_args<R>(2, 2, p, p ^ 1, 1);
    } else {
      std::memset(&d.t1[p], 0, sizeof d.t1[p]);
      std::memset(&d.t2[p], 0, sizeof d.t2[p]);
    }
  }
  d.bnd = s->bnd();
  d.ghost0 = (R*)s->ghost(0);
  d.ghost1 = (R*)s->ghost(1);
  d.tghost0 = (R*)s->tg(0);
  d.tghost1 = (R*)s->tg(1);
  d.clock = s->clock();
  d.partials = (double*)(s->ws + s->L.partials);
  // the tile grid of the run's stage kernel (WENO5: 58 cells along r)
  const int ti = s->p.limiter == ICR_LIM_WENO5 ? W5_TI : tile_cells_r(64);
  d.nbx = (s->g.n_r + ti - 1) / ti;
  d.nby = (s->g.n_theta + 3) / 4;
  d.nbz = (s->g.n_phi + planes - 1) / planes;
  d.planes = planes;
  d.par = s->cur;
  d.cfl = s->p.cfl;
  return d;
}

int ens_upload(icr_ensemble* e) {
  const int n = e->n;
  std::vector<int> toff(n + 1, 0), boff(n + 1, 0), coff(n + 1, 0);
  std::vector<char> host(sizeof(RunDesc<double>) * n);
  for (int r = 0; r < n; ++r) {
    icr_solver* s = e->runs[r];
    if (e->f32) {
      RunDesc<float> d = make_desc<float>(s, e->planes[r]);
      std::memcpy(host.data() + sizeof(RunDesc<float>) * r, &d, sizeof d);
      toff[r + 1] = toff[r] + d.nbx * d.nby * d.nbz;
    } else {
      RunDesc<double> d = make_desc<double>(s, e->planes[r]);
      std::memcpy(host.data() + sizeof(RunDesc<double>) * r, &d, sizeof d);
      toff[r + 1] = toff[r] + d.nbx * d.nby * d.nbz;
    }
    boff[r + 1] = boff[r] + (s->g.n_theta * s->g.n_phi + 255) / 256;
    coff[r + 1] = coff[r] + (s->trc() ? (int)((s->ncell() + 255) / 256) : 0);
  }
  e->n_tiles = toff[n];
  e->n_bitems = boff[n];
  e->n_titems = coff[n];
  const size_t rb = e->f32 ? sizeof(RunDesc<float>) * n : sizeof(RunDesc<double>) * n;
  HIP_TRY(hipMemcpyAsync(e->d_runs, host.data(), rb, hipMemcpyHostToDevice, e->stream));
  HIP_TRY(hipMemcpyAsync(e->d_tile_off, toff.data(), sizeof(int) * (n + 1), hipMemcpyHostToDevice,
                         e->stream));
  HIP_TRY(hipMemcpyAsync(e->d_bnd_off, boff.data(), sizeof(int) * (n + 1), hipMemcpyHostToDevice,
                         e->stream));
  HIP_TRY(hipMemcpyAsync(e->d_trc_off, coff.data(), sizeof(int) * (n + 1), hipMemcpyHostToDevice,
                         e->stream));
  HIP_TRY(hipStreamSynchronize(e->stream));
  return ICR_OK;
}

EnsLaunch ens_launch_args(icr_ensemble* e, int nsteps) {
  EnsLaunch L;
  L.runs = e->d_runs;
  L.e.n_runs = e->n;
  L.e.n_tiles = e->n_tiles;
  L.e.n_bitems = e->n_bitems;
  L.e.n_titems = e->n_titems;
  L.e.trc_off = e->d_trc_off;
  L.e.tile_off = e->d_tile_off;
  L.e.bnd_off = e->d_bnd_off;
  L.e.bar = e->d_bar;
  L.e.spin_limit = e->spin_limit;
  L.persistent = e->persistent;
  L.grid = e->grid;
  L.nsteps = nsteps;
  L.flux = e->p.flux;
  L.lim = e->p.limiter;
  L.tracer = e->p.tracer ? 1 : 0;
  return L;
}

void ens_drop_graph(icr_ensemble* e) {
  if (e->graph_ok) (void)hipGraphExecDestroy(e->g_chunk);
  e->graph_ok = false;
}

}  // namespace

extern "C" {

int icr_ens_workspace_bytes(int n, const icr_grid* grids, const icr_phys* phys, size_t* bytes) {
  if (n < 1 || !grids || !bytes) return fail(ICR_ERR_ARG, "need n >= 1, grids and bytes");
  if (phys && phys->limiter == ICR_LIM_WENO5 && phys->tracer)
    return fail(ICR_ERR_UNSUPPORTED,
                "WENO5 with the passive tracer is available for single solvers only");
  size_t total = ens_table_bytes(n);
  for (int r = 0; r < n; ++r) {
    int rc = validate(&grids[r], phys);
    if (rc) return rc;
    total += align_up(make_layout(grids[r], *phys).total);
  }
  *bytes = total;
  return ICR_OK;
}

int icr_ens_create(int n, const icr_grid* grids, const icr_phys* phys, void* ws, size_t bytes,
                   void* stream, icr_ensemble** out) {
  size_t need = 0;
  int rc = icr_ens_workspace_bytes(n, grids, phys, &need);
  if (rc) return rc;
  if (!out) return fail(ICR_ERR_ARG, "out is NULL");
  *out = nullptr;
  if (!ws || bytes < need) return fail(ICR_ERR_ARG, "workspace too small: %zu < %zu", bytes, need);
  if (((uintptr_t)ws & 255) != 0) return fail(ICR_ERR_ARG, "workspace must be 256-byte aligned");
  icr_ensemble* e = new icr_ensemble();
  e->n = n;
  e->p = *phys;
  e->f32 = phys->precision == ICR_PREC_F32;
  e->stream = (hipStream_t)stream;
  e->ws = (char*)ws;
  e->table_bytes = ens_table_bytes(n);
  char* t = e->ws;
  e->d_runs = t;
  t += align_up(sizeof(RunDesc<double>) * n);
  e->d_tile_off = (int*)t;
  t += align_up(sizeof(int) * (n + 1));
  e->d_bnd_off = (int*)t;
  t += align_up(sizeof(int) * (n + 1));
  e->d_trc_off = (int*)t;
  t += align_up(sizeof(int) * (n + 1));
  e->d_bar = (GridBar*)t;
  t += align_up(sizeof(GridBar));
  e->d_clocks = (DevClock**)t;
  t += align_up(sizeof(DevClock*) * n);
  e->d_gather = (DevClock*)t;
  e->persistent = 1;
  e->use_graphs = 1;
  e->graph_ok = false;
  e->graph_n = 0;
  e->spin_limit = 1LL << 28;
  e->planes.assign(n, 8);
  if (hipStreamCreateWithFlags(&e->cap_stream, hipStreamNonBlocking) != hipSuccess) {
    delete e;
    return fail(ICR_ERR_HIP, "hipStreamCreate failed");
  }
  char* w = e->ws + e->table_bytes;
  std::vector<DevClock*> clocks(n);
  for (int r = 0; r < n; ++r) {
    const size_t b = align_up(make_layout(grids[r], *phys).total);
    icr_solver* s = nullptr;
    rc = icr_create(&grids[r], phys, w, b, stream, &s);
    if (rc) {
      for (icr_solver* q : e->runs) icr_destroy(q);
      (void)hipStreamDestroy(e->cap_stream);
      delete e;
      return rc;
    }
    e->runs.push_back(s);
    clocks[r] = s->clock();
    if (e->planes[r] > grids[r].n_phi) e->planes[r] = grids[r].n_phi;
    w += b;
  }
  GridBar zero{};
  HIP_TRY(hipMemcpyAsync(e->d_bar, &zero, sizeof zero, hipMemcpyHostToDevice, e->stream));
  HIP_TRY(hipMemcpyAsync(e->d_clocks, clocks.data(), sizeof(DevClock*) * n,
                         hipMemcpyHostToDevice, e->stream));
  HIP_TRY(hipStreamSynchronize(e->stream));
  int dev = 0, cus = 0;
  HIP_TRY(hipGetDevice(&dev));
  HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  const int per_cu = ensemble_blocks_per_cu(e->f32, phys->flux, phys->limiter, phys->tracer != 0);
  e->grid = (per_cu > 0 ? per_cu : 1) * cus;
  e->grid -= e->grid % NXCD;
  if (e->grid < NXCD) e->grid = NXCD;
  *out = e;
  return ICR_OK;
}

void icr_ens_destroy(icr_ensemble* e) {
  if (!e) return;
  (void)hipStreamSynchronize(e->stream);
  ens_drop_graph(e);
  for (icr_solver* s : e->runs) icr_destroy(s);
  (void)hipStreamDestroy(e->cap_stream);
  delete e;
}

int icr_ens_run(icr_ensemble* e, int r, icr_solver** out) {
  if (!e || !out) return fail(ICR_ERR_ARG, "NULL argument");
  if (r < 0 || r >= e->n) return fail(ICR_ERR_ARG, "run %d outside [0, %d)", r, e->n);
  *out = e->runs[r];
  return ICR_OK;
}

int icr_ens_set_planes(icr_ensemble* e, int r, int planes) {
  if (!e) return fail(ICR_ERR_ARG, "ensemble is NULL");
  if (r < 0 || r >= e->n) return fail(ICR_ERR_ARG, "run %d outside [0, %d)", r, e->n);
  if (planes < 1 || planes > e->runs[r]->g.n_phi)
    return fail(ICR_ERR_ARG, "planes must be in [1, n_phi]");
  e->planes[r] = planes;
  ens_drop_graph(e);
  return ICR_OK;
}

int icr_ens_set_mode(icr_ensemble* e, int persistent, int grid_blocks, int use_graphs) {
  if (!e) return fail(ICR_ERR_ARG, "ensemble is NULL");
  if (grid_blocks < 0) return fail(ICR_ERR_ARG, "grid_blocks must be >= 0");
  if (grid_blocks > 0) {
    int dev = 0, cus = 0;
    HIP_TRY(hipGetDevice(&dev));
    HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    const int per_cu = ensemble_blocks_per_cu(e->f32, e->p.flux, e->p.limiter, e->p.tracer != 0);
    if (grid_blocks % NXCD != 0 || grid_blocks > per_cu * cus)
      return fail(ICR_ERR_ARG, "grid_blocks must be a multiple of 8 and <= %d resident blocks",
                  per_cu * cus);
    e->grid = grid_blocks;
  }
  e->persistent = persistent ? 1 : 0;
  e->use_graphs = use_graphs ? 1 : 0;
  ens_drop_graph(e);
  return ICR_OK;
}

int icr_ens_step(icr_ensemble* e, int n_steps, double t_end_s, icr_step_info* info) {
  if (!e) return fail(ICR_ERR_ARG, "ensemble is NULL");
  if (n_steps < 0) return fail(ICR_ERR_ARG, "n_steps must be >= 0");
  for (int r = 0; r < e->n; ++r) {
    if (!e->runs[r]->have_maps || !e->runs[r]->have_state)
      return fail(ICR_ERR_STATE, "run %d needs maps and a state", r);
  }
  int rc = ens_upload(e);
  if (rc) return rc;
  GridBar zero{};  // no ensemble kernel is in flight between calls
  HIP_TRY(hipMemcpyAsync(e->d_bar, &zero, sizeof zero, hipMemcpyHostToDevice, e->stream));
  launch_ens_clock_begin(e->d_clocks, e->n, t_end_s > 0.0 ? t_end_s / e->runs[0]->un.t : -1.0,
                         e->stream);
  // graphs replay an even chunk of steps; the parity in the tables is the
  // parity at the start of each replay
  constexpr int ECHUNK = 8;
  int left = n_steps;
  if (e->use_graphs && left >= ECHUNK) {
    if (!e->graph_ok) {
      hipGraph_t g;
      HIP_TRY(hipStreamBeginCapture(e->cap_stream, hipStreamCaptureModeThreadLocal));
      launch_ensemble(ens_launch_args(e, ECHUNK), e->f32, e->cap_stream);
      HIP_TRY(hipStreamEndCapture(e->cap_stream, &g));
      hipError_t ie = hipGraphInstantiate(&e->g_chunk, g, nullptr, nullptr, 0);
      (void)hipGraphDestroy(g);
      if (ie != hipSuccess) return fail(ICR_ERR_HIP, "hipGraphInstantiate failed");
      e->graph_ok = true;
    }
    while (left >= ECHUNK) {
      HIP_TRY(hipGraphLaunch(e->g_chunk, e->stream));
      left -= ECHUNK;
    }
  }
  if (left > 0)  // chunks keep the parity (ECHUNK is even): the tables still hold
    launch_ensemble(ens_launch_args(e, left), e->f32, e->stream);
  HIP_TRY(hipGetLastError());
  for (icr_solver* s : e->runs) s->cur ^= (n_steps & 1);
  launch_ens_gather(e->d_clocks, e->n, e->d_gather, e->stream);
  std::vector<DevClock> c(e->n);
  GridBar bar;
  HIP_TRY(hipMemcpyAsync(c.data(), e->d_gather, sizeof(DevClock) * e->n, hipMemcpyDeviceToHost,
                         e->stream));
  HIP_TRY(hipMemcpyAsync(&bar, e->d_bar, sizeof bar, hipMemcpyDeviceToHost, e->stream));
  HIP_TRY(hipStreamSynchronize(e->stream));
  if (bar.error) return fail(ICR_ERR_HIP, "ensemble grid barrier timed out (blocks not resident)");
  int status = ICR_OK;
  for (int r = 0; r < e->n; ++r) {
    const Units& u = e->runs[r]->un;
    if (info) {
      info[r].steps_taken = (int)c[r].taken;
      info[r].status = c[r].bad == BAD_NONE ? ICR_OK : ICR_ERR_NONPHYSICAL;
      info[r].bad_cell = c[r].bad == BAD_NONE ? -1 : c[r].bad;
      info[r].t = c[r].t * u.t;
      info[r].last_dt = c[r].last_dt * u.t;
      info[r].residual = c[r].resid;
    }
    if (c[r].bad != BAD_NONE) status = ICR_ERR_NONPHYSICAL;
  }
  if (status) return fail(status, "a run produced a non-physical cell");
  return ICR_OK;
}

}  // extern "C"
