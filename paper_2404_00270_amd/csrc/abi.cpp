// C ABI (include/wbpr.h): argument validation, host<->device staging and
// translation of internal status into wbpr_status codes.  Every solve runs on
// the context's engine (engine.hip).
#include <hip/hip_runtime.h>

#include <chrono>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/wbpr.h"
#include "wb_ctx.h"

namespace wb {
thread_local std::string g_err;

int check_shape(int32_t V, int64_t E, int32_t s, int32_t t) {
  if (V < 2) return fail(WBPR_EINVAL, "V must be at least 2");
  if (V >= (1 << 30)) return fail(WBPR_ETOOBIG, "V must be below 2^30");
  if (E < 0) return fail(WBPR_EINVAL, "negative E");
  if (E >= (1ll << 30)) return fail(WBPR_ETOOBIG, "E must be below 2^30");
  if (s < 0 || s >= V || t < 0 || t >= V) return fail(WBPR_EINVAL, "s or t out of range");
  if (s == t) return fail(WBPR_EINVAL, "s == t");
  return WBPR_OK;
}
}  // namespace wb

using wb::check_shape;
using wb::DevBuf;
using wb::fail;
using wb::g_err;
using wb::hip_fail;

namespace {

wb::SolveConfig to_config(const wbpr_options *o) {
  wb::SolveConfig c;
  if (!o) return c;
  c.lanes_per_vertex = o->lanes_per_vertex;
  c.split_degree = o->split_degree;
  c.block_degree = o->block_degree;
  c.gr_every_sweeps = o->gr_every_sweeps;
  c.gr_work_permille = o->gr_work_permille;
  c.max_sweeps = o->max_sweeps;
  c.max_wall_ms = o->max_wall_ms;
  c.grid_blocks = o->grid_blocks;
  c.time_kernels = o->time_kernels != 0;
  c.push_mode = o->push_mode;
  c.use_graph = o->no_graph == 0;
  c.full_scan = o->avq_mode == 1;
  c.gr_stagnation = o->gr_stagnation;
  c.wave_trace = o->wave_trace != 0;
  c.lds_max_v = o->lds_max_v;
  c.gap = o->gap >= 0;
  c.rcsr = o->layout == WBPR_LAYOUT_RCSR;
  c.batch_kernel = o->batch_kernel;
  c.debug_checks = o->debug_checks != 0;
  return c;
}

int check_options(const wbpr_options *o) {
  if (!o) return WBPR_OK;
  int P = o->lanes_per_vertex;
  if (P != 0 && P != 1 && P != 4 && P != 8 && P != 16 && P != 32 && P != 64)
    return fail(WBPR_EINVAL, "lanes_per_vertex must be 0, 1, 4, 8, 16, 32 or 64");
  if (o->avq_mode < 0 || o->avq_mode > 2) return fail(WBPR_EINVAL, "avq_mode must be 0, 1 or 2");
  if (o->split_degree < 0 || o->block_degree < 0 || o->gr_every_sweeps < 0 || o->gr_work_permille < 0 ||
      o->gr_stagnation < 0 ||
      o->max_sweeps < 0 || o->max_wall_ms < 0 || o->grid_blocks < 0)
    return fail(WBPR_EINVAL, "negative option");
  if (o->layout != WBPR_LAYOUT_AUTO && o->layout != WBPR_LAYOUT_BCSR && o->layout != WBPR_LAYOUT_RCSR)
    return fail(WBPR_EINVAL, "unknown layout");
  if (o->push_mode < 0 || o->push_mode > 2) return fail(WBPR_EINVAL, "push_mode must be 0, 1 or 2");
  if (o->batch_kernel < 0 || o->batch_kernel > 2) return fail(WBPR_EINVAL, "batch_kernel must be 0, 1 or 2");
  return WBPR_OK;
}

void fill_stats(wbpr_stats *st, const wb::EngineStats &r, const wb::SolveConfig &cfg, int64_t V, int64_t E, int64_t M,
                int32_t n, double ms_build, double ms_solve, double ms_total) {
  std::memset(st, 0, sizeof(*st));
  st->V = V;
  st->E = E;
  st->M = M;
  st->sweeps = r.sweeps;
  st->global_relabels = r.global_relabels;
  st->pushes = r.pushes;
  st->relabels = r.relabels;
  st->arc_scans = r.arc_scans;
  st->queued = r.queued;
  st->bfs_scans = r.bfs_scans;
  st->nonempty_sweeps = r.nonempty_sweeps;
  st->gr_levels = r.gr_levels;
  st->lanes_per_vertex = r.lanes;
  st->split_degree = r.split_degree;
  st->block_degree = r.block_degree;
  st->gr_every_sweeps = cfg.gr_every_sweeps;
  st->grid_blocks = cfg.grid_blocks > 0 ? cfg.grid_blocks : 1024;
  st->gr_blocks = r.gr_blocks;
  st->ms_build = ms_build;
  st->ms_phase1 = ms_solve;  // both phases, interleaved per instance
  st->ms_total = ms_total;
  for (int k = 0; k < 4; k++) {
    st->kernel_ms[k] = r.k_ms[k];
    st->kernel_launches[k] = r.k_launches[k];
    st->kernel_arc_scans[k] = r.k_scans[k];
    st->kernel_pushes[k] = r.k_pushes[k];
    st->kernel_relabels[k] = r.k_relabels[k];
    st->kernel_queued[k] = r.k_queued[k];
  }
  st->bfs_topdown_scans = r.bfs_topdown_scans;
  st->instances = n;
  st->use_graph = cfg.use_graph && !cfg.time_kernels;
  st->lds_solved = r.small_solved;
  st->gap_skipped = r.gap_skipped;
  st->lds_fallbacks = r.small_fallbacks;
  st->kernel_build_ms = r.build_ms;
  st->layout = cfg.rcsr ? WBPR_LAYOUT_RCSR : WBPR_LAYOUT_BCSR;
  st->wg_solved = r.wg_solved;
  st->wg_fallbacks = r.wg_fallbacks;
  st->debug_checked = r.debug_checked;
}

}  // namespace

extern "C" {

const char *wbpr_version(void) { return "wbpr-mi355x 0.2 (gfx950, BCSR and RCSR vertex-centric push-relabel, batched engine)"; }

const char *wbpr_last_error(void) { return g_err.c_str(); }

int wbpr_device_arch(int dev, char *buf, size_t n) {
  if (!buf || n == 0) return fail(WBPR_EINVAL, "null buffer");
  hipDeviceProp_t prop;
  hipError_t e = hipGetDeviceProperties(&prop, dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDeviceProperties");
  std::snprintf(buf, n, "%s", prop.gcnArchName);
  return WBPR_OK;
}

int wbpr_ctx_create(int device, const wbpr_options *opt, wbpr_ctx **out) {
  if (!out) return fail(WBPR_EINVAL, "null output handle");
  *out = nullptr;
  int rc = check_options(opt);
  if (rc) return rc;
  int ndev = 0;
  hipError_t e = hipGetDeviceCount(&ndev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDeviceCount");
  if (device < 0 || device >= ndev) return fail(WBPR_EINVAL, "no such device");
  e = hipSetDevice(device);
  if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
  wbpr_ctx *c = new (std::nothrow) wbpr_ctx();
  if (!c) return fail(WBPR_ENOMEM, "host allocation");
  c->device = device;
  c->cfg = to_config(opt);
  e = hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&c->ev_in, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&c->ev_out, hipEventDisableTiming);
  if (e != hipSuccess) {
    wbpr_ctx_destroy(c);
    return hip_fail(e, "stream");
  }
  c->engine.reset(new (std::nothrow) wb::Engine(device));
  if (!c->engine) {
    wbpr_ctx_destroy(c);
    return fail(WBPR_ENOMEM, "engine");
  }
  c->engine->set_config(c->cfg);
  *out = c;
  return WBPR_OK;
}

void wbpr_ctx_destroy(wbpr_ctx *c) {
  if (!c) return;
  hipSetDevice(c->device);
  if (c->stream) hipStreamSynchronize(c->stream);
  c->engine.reset();
  c->engine_na.reset();
  c->input.release();
  c->output.release();
  if (c->ev_in) hipEventDestroy(c->ev_in);
  if (c->ev_out) hipEventDestroy(c->ev_out);
  if (c->stream) hipStreamDestroy(c->stream);
  delete c;
}

int wbpr_ctx_set_options(wbpr_ctx *c, const wbpr_options *opt) {
  if (!c) return fail(WBPR_EINVAL, "null context");
  int rc = check_options(opt);
  if (rc) return rc;
  c->cfg = to_config(opt);
  c->engine->set_config(c->cfg);
  return WBPR_OK;
}

}  // extern "C"

namespace {

int ilog2(int64_t x) {
  int l = 0;
  while (x > 1) {
    x >>= 1;
    l++;
  }
  return l;
}

// Shape class of a graph for the autotuner's cache.
std::pair<int, int> shape_class(int64_t V, int64_t E) {
  return {ilog2(V), ilog2(V > 0 ? (2 * E + V - 1) / V : 1)};
}

// The context's options, with an autotuned schedule for this shape class when
// the options leave the schedule to the library.
wb::SolveConfig effective_config(wbpr_ctx *c, int64_t V, int64_t E) {
  wb::SolveConfig cfg = c->cfg;
  if (cfg.lanes_per_vertex == 0 && cfg.gr_work_permille == 0) {
    auto it = c->tuned.find(shape_class(V, E));
    if (it != c->tuned.end()) {
      cfg.lanes_per_vertex = it->second.lanes_per_vertex;
      cfg.gr_work_permille = it->second.gr_work_permille;
      cfg.gr_stagnation = it->second.gr_stagnation;
      cfg.full_scan = it->second.full_scan;
    }
  }
  return cfg;
}

bool same_schedule(const wb::SolveConfig &a, const wb::SolveConfig &b) {
  return a.lanes_per_vertex == b.lanes_per_vertex && a.gr_work_permille == b.gr_work_permille &&
         a.full_scan == b.full_scan && a.gr_stagnation == b.gr_stagnation && a.split_degree == b.split_degree &&
         a.block_degree == b.block_degree &&
         a.gr_every_sweeps == b.gr_every_sweeps && a.grid_blocks == b.grid_blocks &&
         a.time_kernels == b.time_kernels && a.push_mode == b.push_mode && a.use_graph == b.use_graph &&
         a.max_sweeps == b.max_sweeps && a.max_wall_ms == b.max_wall_ms && a.wave_trace == b.wave_trace &&
         a.lds_max_v == b.lds_max_v && a.gap == b.gap && a.rcsr == b.rcsr && a.batch_kernel == b.batch_kernel &&
         a.debug_checks == b.debug_checks;
}

// Solves a group already packed on the device, from an empty engine.
int solve_group(wbpr_ctx *c, wb::GroupInput &in, hipStream_t st, wbpr_stats *stats, wb::Engine *engine = nullptr) {
  auto t0 = std::chrono::steady_clock::now();
  int64_t Vt = 0, Et = 0;
  for (int i = 0; i < in.n; i++) {
    Vt += in.V[i];
    Et += in.E[i];
  }
  if (Vt >= (1ll << 30) || 2 * Et >= (1ll << 31) - 1) return fail(WBPR_ETOOBIG, "batch exceeds the 32-bit index limits");
  wb::Engine &eng = engine ? *engine : *c->engine;
  if (!eng.idle()) return fail(WBPR_EAGAIN, "context busy");
  wb::SolveConfig cfg = effective_config(c, Vt, Et);
  if (eng.external()) {  // nothing that creates graphs, events or trace buffers
    cfg.use_graph = false;
    cfg.time_kernels = false;
    cfg.wave_trace = false;
  }
  if (!same_schedule(cfg, eng.config())) eng.set_config(cfg);
  std::string err;
  int rc = eng.reserve(Vt, 2 * Et, Et, in.n, Vt, Et, in.n, &err);
  if (rc) return fail(rc, err);
  eng.reset_stats();
  rc = eng.admit(in, st, &err);
  if (rc) return fail(rc, err);
  const int64_t M = eng.last_build_M();
  auto t1 = std::chrono::steady_clock::now();
  std::vector<wb::Finished> done;
  rc = eng.run_to_completion(st, &done, &err);
  if (rc) {
    eng.abandon(st);  // leave the engine empty for the next call
    return fail(rc, err);
  }
  auto t2 = std::chrono::steady_clock::now();
  if (stats) {
    wb::EngineStats r;
    rc = eng.collect_stats(st, &r, &err);
    if (rc) return fail(rc, err);
    const double ms_build = std::chrono::duration<double, std::milli>(t1 - t0).count();
    const double ms_solve = std::chrono::duration<double, std::milli>(t2 - t1).count();
    const double ms_total = std::chrono::duration<double, std::milli>(t2 - t0).count();
    fill_stats(stats, r, cfg, Vt, Et, M, in.n, ms_build, ms_solve, ms_total);
    if (in.n == 1 && in.values) {
      long long v = 0;
      if (hipMemcpy(&v, in.values, sizeof(v), hipMemcpyDeviceToHost) == hipSuccess) stats->value = v;
    }
  }
  return WBPR_OK;
}

// Runs fn on the context's stream, ordered after the work already queued on
// the caller's stream (NULL: the legacy default stream) and with the
// caller's stream made to wait for everything fn queued.  The library keeps
// its own stream because it captures sweep batches into graphs there.
template <class F>
int on_caller_stream(wbpr_ctx *c, void *stream, F fn) {
  hipStream_t caller = (hipStream_t)stream;
  hipError_t e = hipEventRecord(c->ev_in, caller);
  if (e == hipSuccess) e = hipStreamWaitEvent(c->stream, c->ev_in, 0);
  if (e != hipSuccess) return hip_fail(e, "ordering after the caller's stream");
  const int rc = fn(c->stream);
  e = hipEventRecord(c->ev_out, c->stream);
  if (e == hipSuccess) e = hipStreamWaitEvent(caller, c->ev_out, 0);
  if (e != hipSuccess && rc == WBPR_OK) return hip_fail(e, "ordering the caller's stream after the solve");
  return rc;
}

}  // namespace

extern "C" {

int wbpr_solve_device(wbpr_ctx *c, const wbpr_csr *g, int32_t s, int32_t t, void *stream, int64_t *dev_value,
                      int32_t *dev_arc_flow, uint8_t *dev_cut_side, wbpr_stats *stats) {
  if (!c) return fail(WBPR_EINVAL, "null context");
  if (!g) return fail(WBPR_EINVAL, "null graph");
  int rc = check_shape(g->V, g->E, s, t);
  if (rc) return rc;
  if (!g->row_ptr || (g->E > 0 && (!g->col || !g->cap))) return fail(WBPR_EINVAL, "null CSR array");
  if (!dev_value) return fail(WBPR_EINVAL, "null value pointer");
  hipError_t e = hipSetDevice(c->device);
  if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
  int32_t V = g->V;
  int64_t E = g->E;
  wb::GroupInput in;
  in.n = 1;
  in.V = &V;
  in.E = &E;
  in.s = &s;
  in.t = &t;
  in.row_ptr = g->row_ptr;
  in.col = g->col;
  in.cap = g->cap;
  in.values = dev_value;
  in.flows = dev_arc_flow;
  in.sides = dev_cut_side;
  return on_caller_stream(c, stream, [&](hipStream_t st) { return solve_group(c, in, st, stats); });
}

}  // extern "C"

// ------------------------------------------------------- allocation-free
// Device memory of the allocation-free entry point: one static array, of
// which every device that loads this library's code holds its own copy until
// the process ends.  In host code the name `scratch` is a host-side stand-in,
// never a device address: host code only uses the address that
// hipGetSymbolAddress returns for the current device, kept per device.
static __device__ __align__(256) unsigned char scratch[WBPR_NOALLOC_SCRATCH_BYTES];

namespace {

std::mutex g_scratch_mu;
std::map<int, void *> g_scratch_ptr;  // device -> its copy of scratch

// Device address of scratch on `device`, which must be current; looked up
// once per device.
int scratch_on(int device, void **out) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  auto it = g_scratch_ptr.find(device);
  if (it != g_scratch_ptr.end()) {
    *out = it->second;
    return WBPR_OK;
  }
  void *p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return hip_fail(e, "address of the static scratch array");
  if (!p) return fail(WBPR_EDEVICE, "address of the static scratch array: null");
  g_scratch_ptr[device] = p;
  *out = p;
  return WBPR_OK;
}

}  // namespace

extern "C" {

int wbpr_solve_device_noalloc(wbpr_ctx *c, const wbpr_csr *g, int32_t s, int32_t t, void *stream,
                              int64_t *dev_value, int32_t *dev_arc_flow, uint8_t *dev_cut_side, wbpr_stats *stats) {
  if (!c) return fail(WBPR_EINVAL, "null context");
  if (!g) return fail(WBPR_EINVAL, "null graph");
  int rc = check_shape(g->V, g->E, s, t);
  if (rc) return rc;
  if (!g->row_ptr || (g->E > 0 && (!g->col || !g->cap))) return fail(WBPR_EINVAL, "null CSR array");
  if (!dev_value) return fail(WBPR_EINVAL, "null value pointer");
  hipError_t e = hipSetDevice(c->device);
  if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
  void *base = nullptr;
  rc = scratch_on(c->device, &base);
  if (rc) return rc;
  if (!c->engine_na) {  // host object only: it carves the static array, allocates nothing
    c->engine_na.reset(new (std::nothrow) wb::Engine(c->device));
    if (!c->engine_na) return fail(WBPR_ENOMEM, "engine");
    c->engine_na->set_external(base, WBPR_NOALLOC_SCRATCH_BYTES);
  }
  int32_t V = g->V;
  int64_t E = g->E;
  wb::GroupInput in;
  in.n = 1;
  in.V = &V;
  in.E = &E;
  in.s = &s;
  in.t = &t;
  in.row_ptr = g->row_ptr;
  in.col = g->col;
  in.cap = g->cap;
  in.values = dev_value;
  in.flows = dev_arc_flow;
  in.sides = dev_cut_side;
  return on_caller_stream(c, stream,
                          [&](hipStream_t st) { return solve_group(c, in, st, stats, c->engine_na.get()); });
}

int wbpr_solve(wbpr_ctx *c, const wbpr_csr *g, int32_t s, int32_t t, int64_t *value, int32_t *arc_flow,
               uint8_t *cut_side, wbpr_stats *stats) {
  if (!c) return fail(WBPR_EINVAL, "null context");
  if (!g) return fail(WBPR_EINVAL, "null graph");
  int rc = check_shape(g->V, g->E, s, t);
  if (rc) return rc;
  if (!g->row_ptr || (g->E > 0 && (!g->col || !g->cap))) return fail(WBPR_EINVAL, "null CSR array");
  if (!value) return fail(WBPR_EINVAL, "null value pointer");
  hipError_t e = hipSetDevice(c->device);
  if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
  const int64_t V = g->V, E = g->E;
  auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
  const size_t Ec = (size_t)(E > 0 ? E : 1);
  e = c->input.ensure(al(8 * (V + 1)) + 2 * al(4 * Ec));
  if (e == hipSuccess) e = c->output.ensure(al(8) + al(4 * Ec) + al((size_t)V));
  if (e != hipSuccess) return hip_fail(e, "device allocation (staging)");
  char *ip = (char *)c->input.p;
  int64_t *d_rp = (int64_t *)ip;
  int32_t *d_col = (int32_t *)(ip + al(8 * (V + 1)));
  int32_t *d_cap = (int32_t *)(ip + al(8 * (V + 1)) + al(4 * Ec));
  char *op = (char *)c->output.p;
  int64_t *d_val = (int64_t *)op;
  int32_t *d_flow = (int32_t *)(op + al(8));
  uint8_t *d_side = (uint8_t *)(op + al(8) + al(4 * Ec));
  hipStream_t st = c->stream;
  e = hipMemcpyAsync(d_rp, g->row_ptr, 8 * (V + 1), hipMemcpyHostToDevice, st);
  if (e == hipSuccess && E > 0) e = hipMemcpyAsync(d_col, g->col, 4 * E, hipMemcpyHostToDevice, st);
  if (e == hipSuccess && E > 0) e = hipMemcpyAsync(d_cap, g->cap, 4 * E, hipMemcpyHostToDevice, st);
  if (e != hipSuccess) return hip_fail(e, "host to device copy");
  wbpr_csr dg{g->V, g->E, d_rp, d_col, d_cap};
  rc = wbpr_solve_device(c, &dg, s, t, st, d_val, arc_flow ? d_flow : nullptr, cut_side ? d_side : nullptr, stats);
  if (rc) return rc;
  e = hipMemcpyAsync(value, d_val, 8, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess && arc_flow && E > 0) e = hipMemcpyAsync(arc_flow, d_flow, 4 * E, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess && cut_side) e = hipMemcpyAsync(cut_side, d_side, (size_t)V, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return hip_fail(e, "device to host copy");
  return WBPR_OK;
}

namespace {

// One instance of a packed device batch, solved alone (offsets into the
// packed arrays).
int solve_one_of(wbpr_ctx *c, int i, const int32_t *V, const int64_t *E, const int32_t *s, const int32_t *t,
                 const int64_t *rp, const int32_t *col, const int32_t *cap, hipStream_t st, int64_t *values,
                 int32_t *flows, uint8_t *sides, const std::vector<int64_t> &ro, const std::vector<int64_t> &eo,
                 const std::vector<int64_t> &vo) {
  wb::GroupInput in;
  in.n = 1;
  in.V = V + i;
  in.E = E + i;
  in.s = s + i;
  in.t = t + i;
  in.row_ptr = rp + ro[i];
  in.col = col ? col + eo[i] : nullptr;
  in.cap = cap ? cap + eo[i] : nullptr;
  in.values = values + i;
  in.flows = flows ? flows + eo[i] : nullptr;
  in.sides = sides ? sides + vo[i] : nullptr;
  return solve_group(c, in, st, nullptr);
}

}  // namespace

int wbpr_solve_batch_device(wbpr_ctx *c, int32_t n, const int32_t *V, const int64_t *E, const int32_t *s,
                            const int32_t *t, const int64_t *dev_row_ptr, const int32_t *dev_col,
                            const int32_t *dev_cap, void *stream, int64_t *dev_values, int32_t *dev_flows,
                            uint8_t *dev_sides, wbpr_stats *stats, int32_t *status) {
  if (!c) return fail(WBPR_EINVAL, "null context");
  if (n < 1) return fail(WBPR_EINVAL, "n must be at least 1");
  if (!V || !E || !s || !t || !dev_row_ptr || !dev_values) return fail(WBPR_EINVAL, "null argument");
  int64_t Et = 0;
  bool all_ok = true;
  for (int i = 0; i < n; i++)  // the packing itself needs every size
    if (V[i] < 0 || E[i] < 0) return fail(WBPR_EINVAL, "instance " + std::to_string(i) + ": negative size");
  for (int i = 0; i < n; i++) {
    int rc = check_shape(V[i], E[i], s[i], t[i]);
    if (rc) {
      if (!status) {
        g_err = "instance " + std::to_string(i) + ": " + g_err;
        return rc;
      }
      all_ok = false;
    }
    if (status) status[i] = rc;
    Et += E[i];
  }
  if (Et > 0 && (!dev_col || !dev_cap)) return fail(WBPR_EINVAL, "null CSR array");
  hipError_t e = hipSetDevice(c->device);
  if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
  return on_caller_stream(c, stream, [&](hipStream_t st) -> int {
    if (all_ok) {
      wb::GroupInput in;
      in.n = n;
      in.V = V;
      in.E = E;
      in.s = s;
      in.t = t;
      in.row_ptr = dev_row_ptr;
      in.col = dev_col;
      in.cap = dev_cap;
      in.values = dev_values;
      in.flows = dev_flows;
      in.sides = dev_sides;
      const int rc = solve_group(c, in, st, stats);
      if (!status || (rc != WBPR_EINVAL && rc != WBPR_EOVERFLOW)) return rc;
      // an instance failed the device checks: find which by solving them alone
    }
    std::vector<int64_t> ro(n), eo(n), vo(n);
    for (int i = 0, r = 0, x = 0, v = 0; i < n; i++) {
      ro[i] = r;
      eo[i] = x;
      vo[i] = v;
      r += V[i] + 1;
      x += E[i];
      v += V[i];
    }
    for (int i = 0; i < n; i++) {
      if (status[i] == WBPR_OK) {
        const int rc = solve_one_of(c, i, V, E, s, t, dev_row_ptr, dev_col, dev_cap, st, dev_values, dev_flows,
                                    dev_sides, ro, eo, vo);
        if (rc != WBPR_OK && rc != WBPR_EINVAL && rc != WBPR_EOVERFLOW) return rc;
        status[i] = rc;
      }
      if (status[i] != WBPR_OK) {
        hipError_t e2 = hipMemsetAsync(dev_values + i, 0, 8, st);
        if (e2 != hipSuccess) return hip_fail(e2, "batch output");
      }
    }
    if (stats) *stats = wbpr_stats{};
    e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_fail(e, "batch");
    return WBPR_OK;
  });
}

int wbpr_solve_batch(wbpr_ctx *c, int32_t n, const wbpr_csr *graphs, const int32_t *s, const int32_t *t,
                     int64_t *values, int32_t *const *flows, uint8_t *const *sides, wbpr_stats *stats,
                     int32_t *status) {
  if (!c) return fail(WBPR_EINVAL, "null context");
  if (n < 1 || !graphs || !s || !t || !values) return fail(WBPR_EINVAL, "null argument");
  // instances that pass the host checks are packed and solved together;
  // with a status array the others are reported there and skipped
  std::vector<int32_t> V, S, T, idx;
  std::vector<int64_t> E;
  int64_t Vt = 0, Et = 0;
  for (int i = 0; i < n; i++) {
    const wbpr_csr &g = graphs[i];
    int rc = check_shape(g.V, g.E, s[i], t[i]);
    if (!rc && (!g.row_ptr || (g.E > 0 && (!g.col || !g.cap)))) rc = fail(WBPR_EINVAL, "null CSR array");
    if (!rc && flows && !flows[i]) rc = fail(WBPR_EINVAL, "flows given but flows[i] is null");
    if (!rc && sides && !sides[i]) rc = fail(WBPR_EINVAL, "sides given but sides[i] is null");
    if (rc) {
      if (!status) {
        g_err = "instance " + std::to_string(i) + ": " + g_err;
        return rc;
      }
      status[i] = rc;
      values[i] = 0;
      continue;
    }
    idx.push_back(i);
    V.push_back(g.V);
    E.push_back(g.E);
    S.push_back(s[i]);
    T.push_back(t[i]);
    Vt += g.V;
    Et += g.E;
  }
  const int m = (int)idx.size();
  if (m == 0) {
    if (stats) *stats = wbpr_stats{};
    return WBPR_OK;
  }
  if (Vt + m >= (1ll << 30) || 2 * Et >= (1ll << 31) - 1) return fail(WBPR_ETOOBIG, "batch exceeds the index limits");
  hipError_t e = hipSetDevice(c->device);
  if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
  auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
  const size_t Ec = (size_t)(Et > 0 ? Et : 1);
  e = c->input.ensure(al(8 * (size_t)(Vt + m)) + 2 * al(4 * Ec));
  if (e == hipSuccess) e = c->output.ensure(al(8 * (size_t)m) + al(4 * Ec) + al((size_t)Vt));
  if (e != hipSuccess) return hip_fail(e, "device allocation (staging)");
  char *ip = (char *)c->input.p;
  int64_t *d_rp = (int64_t *)ip;
  int32_t *d_col = (int32_t *)(ip + al(8 * (size_t)(Vt + m)));
  int32_t *d_cap = (int32_t *)(ip + al(8 * (size_t)(Vt + m)) + al(4 * Ec));
  char *op = (char *)c->output.p;
  int64_t *d_val = (int64_t *)op;
  int32_t *d_flow = (int32_t *)(op + al(8 * (size_t)m));
  uint8_t *d_side = (uint8_t *)(op + al(8 * (size_t)m) + al(4 * Ec));
  hipStream_t st = c->stream;
  int64_t ro = 0, eo = 0;
  for (int k = 0; k < m && e == hipSuccess; k++) {
    const wbpr_csr &g = graphs[idx[k]];
    e = hipMemcpyAsync(d_rp + ro, g.row_ptr, 8 * ((size_t)g.V + 1), hipMemcpyHostToDevice, st);
    if (e == hipSuccess && g.E > 0) e = hipMemcpyAsync(d_col + eo, g.col, 4 * (size_t)g.E, hipMemcpyHostToDevice, st);
    if (e == hipSuccess && g.E > 0) e = hipMemcpyAsync(d_cap + eo, g.cap, 4 * (size_t)g.E, hipMemcpyHostToDevice, st);
    ro += g.V + 1;
    eo += g.E;
  }
  if (e != hipSuccess) return hip_fail(e, "host to device copy");
  std::vector<int32_t> sub(m, 0);
  int rc = wbpr_solve_batch_device(c, m, V.data(), E.data(), S.data(), T.data(), d_rp, d_col, d_cap, st, d_val,
                                   flows ? d_flow : nullptr, sides ? d_side : nullptr, stats,
                                   status ? sub.data() : nullptr);
  if (rc) return rc;
  std::vector<int64_t> hv(m);
  e = hipMemcpyAsync(hv.data(), d_val, 8 * (size_t)m, hipMemcpyDeviceToHost, st);
  int64_t vo = 0;
  eo = 0;
  for (int k = 0; k < m && e == hipSuccess; k++) {
    const int i = idx[k];
    if (sub[k] == WBPR_OK) {
      if (flows && E[k] > 0) e = hipMemcpyAsync(flows[i], d_flow + eo, 4 * (size_t)E[k], hipMemcpyDeviceToHost, st);
      if (e == hipSuccess && sides) e = hipMemcpyAsync(sides[i], d_side + vo, (size_t)V[k], hipMemcpyDeviceToHost, st);
    }
    vo += V[k];
    eo += E[k];
  }
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return hip_fail(e, "device to host copy");
  for (int k = 0; k < m; k++) {
    values[idx[k]] = hv[k];
    if (status) status[idx[k]] = sub[k];
  }
  return WBPR_OK;
}

}  // extern "C"

struct wbpr_graph {
  int device = 0;
  hipStream_t stream = nullptr;
  wb::SolveConfig cfg;
  std::unique_ptr<wb::Engine> engine;
  int gid = -1;
  bool broken = false;
  int32_t V = 0;
  int64_t E = 0, M = 0;
  DevBuf output;
};

extern "C" {

int wbpr_graph_upload(wbpr_ctx *c, const wbpr_csr *g, wbpr_graph **out) {
  if (!c || !g || !out) return fail(WBPR_EINVAL, "null argument");
  *out = nullptr;
  if (g->V < 2) return fail(WBPR_EINVAL, "V must be at least 2");
  int rc = check_shape(g->V, g->E, 0, 1);
  if (rc) return rc;
  if (!g->row_ptr || (g->E > 0 && (!g->col || !g->cap))) return fail(WBPR_EINVAL, "null CSR array");
  hipError_t e = hipSetDevice(c->device);
  if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
  std::unique_ptr<wbpr_graph> G(new (std::nothrow) wbpr_graph());
  if (!G) return fail(WBPR_ENOMEM, "host allocation");
  G->device = c->device;
  G->cfg = c->cfg;
  G->V = g->V;
  G->E = g->E;
  e = hipStreamCreateWithFlags(&G->stream, hipStreamNonBlocking);
  if (e != hipSuccess) return hip_fail(e, "stream");
  auto cleanup = [&](int code) {
    if (G->stream) hipStreamSynchronize(G->stream);
    G->engine.reset();
    G->output.release();
    if (G->stream) hipStreamDestroy(G->stream);
    G->stream = nullptr;
    return code;
  };
  G->engine.reset(new (std::nothrow) wb::Engine(G->device));
  if (!G->engine) return cleanup(fail(WBPR_ENOMEM, "engine"));
  G->engine->set_config(G->cfg);
  const int64_t V = g->V, E = g->E;
  std::string err;
  rc = G->engine->reserve(V, 2 * E, E, 1, V, E, 1, &err);
  if (rc) return cleanup(fail(rc, err));
  // stage the CSR on the device (temporary)
  auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
  const size_t Ec = (size_t)(E > 0 ? E : 1);
  DevBuf input;
  e = input.ensure(al(8 * (V + 1)) + 2 * al(4 * Ec));
  if (e != hipSuccess) return cleanup(hip_fail(e, "device allocation (staging)"));
  char *ip = (char *)input.p;
  int64_t *d_rp = (int64_t *)ip;
  int32_t *d_col = (int32_t *)(ip + al(8 * (V + 1)));
  int32_t *d_cap = (int32_t *)(ip + al(8 * (V + 1)) + al(4 * Ec));
  e = hipMemcpyAsync(d_rp, g->row_ptr, 8 * (V + 1), hipMemcpyHostToDevice, G->stream);
  if (e == hipSuccess && E > 0) e = hipMemcpyAsync(d_col, g->col, 4 * E, hipMemcpyHostToDevice, G->stream);
  if (e == hipSuccess && E > 0) e = hipMemcpyAsync(d_cap, g->cap, 4 * E, hipMemcpyHostToDevice, G->stream);
  if (e != hipSuccess) {
    input.release();
    return cleanup(hip_fail(e, "host to device copy"));
  }
  int32_t Vi = g->V, s0 = 0, t0 = 1;
  int64_t Ei = g->E;
  wb::GroupInput in;
  in.n = 1;
  in.V = &Vi;
  in.E = &Ei;
  in.s = &s0;
  in.t = &t0;
  in.row_ptr = d_rp;
  in.col = d_col;
  in.cap = d_cap;
  in.keep = true;
  in.start = false;
  in.group_out = &G->gid;
  rc = G->engine->admit(in, G->stream, &err);  // synchronises the stream
  input.release();
  if (rc) return cleanup(fail(rc, err));
  G->M = G->engine->last_build_M();
  *out = G.release();
  return WBPR_OK;
}

int wbpr_graph_solve(wbpr_graph *G, int32_t s, int32_t t, int64_t *value, int32_t *arc_flow, uint8_t *cut_side,
                     wbpr_stats *stats) {
  if (!G || !value) return fail(WBPR_EINVAL, "null argument");
  if (G->broken) return fail(WBPR_EINVAL, "graph handle unusable after an earlier failure");
  if (s < 0 || s >= G->V || t < 0 || t >= G->V) return fail(WBPR_EINVAL, "s or t out of range");
  if (s == t) return fail(WBPR_EINVAL, "s == t");
  hipError_t e = hipSetDevice(G->device);
  if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
  auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
  const size_t Ec = (size_t)(G->E > 0 ? G->E : 1);
  e = G->output.ensure(al(8) + al(4 * Ec) + al((size_t)G->V));
  if (e != hipSuccess) return hip_fail(e, "device allocation (outputs)");
  char *op = (char *)G->output.p;
  int64_t *d_val = (int64_t *)op;
  int32_t *d_flow = (int32_t *)(op + al(8));
  uint8_t *d_side = (uint8_t *)(op + al(8) + al(4 * Ec));
  wb::Engine &eng = *G->engine;
  auto t0 = std::chrono::steady_clock::now();
  eng.reset_stats();
  std::string err;
  int rc = eng.start_instance(G->gid, s, t, d_val, arc_flow ? d_flow : nullptr, cut_side ? d_side : nullptr, 0,
                              G->stream, &err);
  if (rc) return fail(rc, err);
  std::vector<wb::Finished> done;
  rc = eng.run_to_completion(G->stream, &done, &err);
  if (rc) {
    eng.abandon(G->stream);
    G->broken = true;
    return fail(rc, err);
  }
  auto t1 = std::chrono::steady_clock::now();
  e = hipMemcpyAsync(value, d_val, 8, hipMemcpyDeviceToHost, G->stream);
  if (e == hipSuccess && arc_flow && G->E > 0)
    e = hipMemcpyAsync(arc_flow, d_flow, 4 * (size_t)G->E, hipMemcpyDeviceToHost, G->stream);
  if (e == hipSuccess && cut_side) e = hipMemcpyAsync(cut_side, d_side, (size_t)G->V, hipMemcpyDeviceToHost, G->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(G->stream);
  if (e != hipSuccess) return hip_fail(e, "device to host copy");
  if (stats) {
    wb::EngineStats r;
    rc = eng.collect_stats(G->stream, &r, &err);
    if (rc) return fail(rc, err);
    const double ms = std::chrono::duration<double, std::milli>(t1 - t0).count();
    fill_stats(stats, r, G->cfg, G->V, G->E, G->M, 1, 0.0, ms, ms);
    stats->value = *value;
  }
  return WBPR_OK;
}

void wbpr_graph_free(wbpr_graph *G) {
  if (!G) return;
  hipSetDevice(G->device);
  if (G->stream) hipStreamSynchronize(G->stream);
  G->engine.reset();
  G->output.release();
  if (G->stream) hipStreamDestroy(G->stream);
  delete G;
}


int wbpr_autotune(wbpr_ctx *c, const wbpr_csr *g, int32_t s, int32_t t, int32_t max_trials, int32_t include_full_scan,
                  wbpr_options *best, double *best_ms) {
  if (!c || !g || !best) return fail(WBPR_EINVAL, "null argument");
  if (max_trials < 0) return fail(WBPR_EINVAL, "negative max_trials");
  int rc = check_shape(g->V, g->E, s, t);
  if (rc) return rc;
  struct Cand {
    int lanes, permille, stag;
    bool full_scan;
  };
  std::vector<Cand> cands;
  // most promising first, so a small max_trials keeps the likely winners
  const int lanes_order[] = {8, 16, 4};
  const int stag_order[] = {0, 4, 32};
  const int permille_order[] = {1000, 300};
  for (int pm : permille_order)
    for (int sg : stag_order)
      for (int l : lanes_order) cands.push_back({l, pm, sg, false});
  if (include_full_scan)
    for (int l : {8, 16}) cands.push_back({l, 1000, 0, true});
  if (max_trials > 0 && (size_t)max_trials < cands.size()) cands.resize((size_t)max_trials);
  wbpr_graph *G = nullptr;
  rc = wbpr_graph_upload(c, g, &G);
  if (rc) return rc;
  std::vector<int32_t> flow((size_t)(g->E > 0 ? g->E : 1));
  std::vector<uint8_t> side((size_t)g->V);
  double bms = 1e300;
  int bi = -1;
  int64_t value0 = -1;
  for (size_t i = 0; i < cands.size(); i++) {
    wb::SolveConfig cfg = c->cfg;
    cfg.lanes_per_vertex = cands[i].lanes;
    cfg.gr_work_permille = cands[i].permille;
    cfg.gr_stagnation = cands[i].stag;
    cfg.full_scan = cands[i].full_scan;
    cfg.time_kernels = false;
    G->cfg = cfg;
    G->engine->set_config(cfg);
    double ms = 0;
    for (int rep = 0; rep < 2; rep++) {  // warm-up (graph capture), then timed
      int64_t v = 0;
      auto t0 = std::chrono::steady_clock::now();
      rc = wbpr_graph_solve(G, s, t, &v, flow.data(), side.data(), nullptr);
      ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
      if (rc) {
        const std::string msg = g_err;
        wbpr_graph_free(G);
        return fail(rc, msg);
      }
      if (value0 < 0) value0 = v;
      if (v != value0) {
        wbpr_graph_free(G);
        return fail(WBPR_EINTERNAL, "schedules disagree on the flow value");
      }
    }
    if (ms < bms) {
      bms = ms;
      bi = (int)i;
    }
  }
  wbpr_graph_free(G);
  wb::SolveConfig win = c->cfg;
  win.lanes_per_vertex = cands[bi].lanes;
  win.gr_work_permille = cands[bi].permille;
  win.gr_stagnation = cands[bi].stag;
  win.full_scan = cands[bi].full_scan;
  c->tuned[shape_class(g->V, g->E)] = win;
  std::memset(best, 0, sizeof(*best));
  best->layout = WBPR_LAYOUT_BCSR;
  best->lanes_per_vertex = win.lanes_per_vertex;
  best->split_degree = win.split_degree;
  best->gr_every_sweeps = win.gr_every_sweeps;
  best->max_sweeps = win.max_sweeps;
  best->max_wall_ms = win.max_wall_ms;
  best->grid_blocks = win.grid_blocks;
  best->time_kernels = win.time_kernels ? 1 : 0;
  best->push_mode = win.push_mode;
  best->block_degree = win.block_degree;
  best->gr_work_permille = win.gr_work_permille;
  best->no_graph = win.use_graph ? 0 : 1;
  best->avq_mode = win.full_scan ? 1 : 0;
  best->gr_stagnation = win.gr_stagnation;
  if (best_ms) *best_ms = bms;
  return WBPR_OK;
}

int wbpr_wave_trace(wbpr_ctx *c, int32_t *records, int64_t cap, int64_t *count) {
  if (!c || !count) return fail(WBPR_EINVAL, "null argument");
  if (cap < 0 || (cap > 0 && !records)) return fail(WBPR_EINVAL, "records must hold cap records");
  hipError_t e = hipSetDevice(c->device);
  if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
  std::string err;
  const int64_t n = c->engine->read_wave_trace(c->stream, records, cap, &err);
  if (n < 0) return fail(WBPR_EDEVICE, "wave trace: " + err);
  *count = n;
  return WBPR_OK;
}

}  // extern "C"
