// C ABI (include/wbpr.h): argument validation, the device arena, host<->device
// staging and translation of internal status into wbpr_status codes.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>

#include "../../include/wbpr.h"
#include "wb_internal.h"
#include "wb_solver.h"

namespace {

thread_local std::string g_err;

int fail(int code, const std::string &msg) {
  g_err = msg;
  return code;
}

int hip_fail(hipError_t e, const char *what) {
  g_err = std::string(what) + ": " + hipGetErrorString(e);
  return e == hipErrorOutOfMemory ? WBPR_ENOMEM : WBPR_EDEVICE;
}

// Grow-only device buffer.
struct DevBuf {
  void *p = nullptr;
  size_t n = 0;
  hipError_t ensure(size_t bytes) {
    if (bytes == 0) bytes = 256;
    if (bytes <= n) return hipSuccess;
    if (p) hipFree(p);
    p = nullptr;
    n = 0;
    hipError_t e = hipMalloc(&p, bytes);
    if (e == hipSuccess) n = bytes;
    return e;
  }
  void release() {
    if (p) hipFree(p);
    p = nullptr;
    n = 0;
  }
};

wb::SolveConfig to_config(const wbpr_options *o) {
  wb::SolveConfig c;
  if (!o) return c;
  c.lanes_per_vertex = o->lanes_per_vertex;
  c.split_degree = o->split_degree;
  c.gr_every_sweeps = o->gr_every_sweeps;
  c.max_sweeps = o->max_sweeps;
  c.max_wall_ms = o->max_wall_ms;
  c.grid_blocks = o->grid_blocks;
  c.time_kernels = o->time_kernels != 0;
  c.push_mode = o->push_mode;
  c.block_degree = o->block_degree;
  return c;
}

int check_options(const wbpr_options *o) {
  if (!o) return WBPR_OK;
  int P = o->lanes_per_vertex;
  if (P != 0 && P != 4 && P != 8 && P != 16 && P != 32 && P != 64)
    return fail(WBPR_EINVAL, "lanes_per_vertex must be 0, 4, 8, 16, 32 or 64");
  if (o->split_degree < 0 || o->block_degree < 0 || o->gr_every_sweeps < 0 || o->max_sweeps < 0 ||
      o->max_wall_ms < 0 || o->grid_blocks < 0)
    return fail(WBPR_EINVAL, "negative option");
  if (o->layout != WBPR_LAYOUT_AUTO && o->layout != WBPR_LAYOUT_BCSR) return fail(WBPR_EINVAL, "unknown layout");
  if (o->push_mode < 0 || o->push_mode > 2) return fail(WBPR_EINVAL, "push_mode must be 0, 1 or 2");
  return WBPR_OK;
}

}  // namespace

struct wbpr_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  wb::SolveConfig cfg;
  DevBuf res, scratch, state, input, output, status;
  long long *pinned = nullptr;  // 64 words of pinned host memory
  int gr_blocks[7] = {0, 0, 0, 0, 0, 0, 0};
  hipEvent_t (*ev)[4] = nullptr;
  hipEvent_t (*gev)[2] = nullptr;
};

extern "C" {

const char *wbpr_version(void) { return "wbpr-mi355x 0.1 (gfx950, BCSR vertex-centric push-relabel)"; }

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
  if (e == hipSuccess) e = hipHostMalloc((void **)&c->pinned, 64 * sizeof(long long), hipHostMallocDefault);
  if (e != hipSuccess) {
    wbpr_ctx_destroy(c);
    return hip_fail(e, "context setup");
  }
  for (int lg = 2; lg <= 6; lg++) c->gr_blocks[lg] = wb::gr_max_blocks(device, 1 << lg);
  *out = c;
  return WBPR_OK;
}

void wbpr_ctx_destroy(wbpr_ctx *c) {
  if (!c) return;
  hipSetDevice(c->device);
  if (c->stream) hipStreamSynchronize(c->stream);
  c->res.release();
  c->scratch.release();
  c->state.release();
  c->input.release();
  c->output.release();
  c->status.release();
  if (c->ev) {
    for (int i = 0; i < wb::State::kMaxSweeps; i++)
      for (int k = 0; k < 4; k++) hipEventDestroy(c->ev[i][k]);
    delete[] c->ev;
  }
  if (c->gev) {
    for (int i = 0; i < wb::State::kMaxGR; i++)
      for (int k = 0; k < 2; k++) hipEventDestroy(c->gev[i][k]);
    delete[] c->gev;
  }
  if (c->pinned) hipHostFree(c->pinned);
  if (c->stream) hipStreamDestroy(c->stream);
  delete c;
}

int wbpr_ctx_set_options(wbpr_ctx *c, const wbpr_options *opt) {
  if (!c) return fail(WBPR_EINVAL, "null context");
  int rc = check_options(opt);
  if (rc) return rc;
  c->cfg = to_config(opt);
  return WBPR_OK;
}

}  // extern "C"

namespace {

int check_graph_shape(const wbpr_csr *g, int32_t s, int32_t t) {
  if (!g) return fail(WBPR_EINVAL, "null graph");
  if (g->V < 2) return fail(WBPR_EINVAL, "V must be at least 2");
  if (g->V >= (1 << 30)) return fail(WBPR_ETOOBIG, "V must be below 2^30");
  if (g->E < 0) return fail(WBPR_EINVAL, "negative E");
  if (g->E >= (1ll << 30)) return fail(WBPR_ETOOBIG, "E must be below 2^30");
  if (!g->row_ptr || (g->E > 0 && (!g->col || !g->cap))) return fail(WBPR_EINVAL, "null CSR array");
  if (s < 0 || s >= g->V || t < 0 || t >= g->V) return fail(WBPR_EINVAL, "s or t out of range");
  if (s == t) return fail(WBPR_EINVAL, "s == t");
  return WBPR_OK;
}

// Device-resident solve shared by both entry points.
int solve_dev(wbpr_ctx *c, const wbpr_csr *g, int32_t s, int32_t t, hipStream_t st, int64_t *dvalue, int32_t *dflow,
              uint8_t *dside, wbpr_stats *stats) {
  auto t0 = std::chrono::steady_clock::now();
  hipError_t e = c->res.ensure(wb::residual_bytes(g->V, g->E));
  if (e == hipSuccess) e = c->scratch.ensure(wb::build_scratch_bytes(g->V, g->E));
  if (e == hipSuccess) e = c->status.ensure(sizeof(wb::BuildStatus) + 256);
  if (e != hipSuccess) return hip_fail(e, "device allocation (graph)");
  wb::Residual res;
  wb::residual_carve(&res, g->V, g->E, c->res.p);
  wb::BuildStatus *bst = (wb::BuildStatus *)c->status.p;
  e = wb::build_residual(g->row_ptr, g->col, g->cap, &res, c->scratch.p, bst, st);
  if (e == hipSuccess) e = hipMemcpyAsync(c->pinned, bst, sizeof(wb::BuildStatus), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return hip_fail(e, "residual build");
  wb::BuildStatus hb;
  std::memcpy(&hb, c->pinned, sizeof(hb));
  if (hb.bad_input) return fail(WBPR_EINVAL, "malformed CSR (row_ptr not monotone from 0 to E, col out of range, or negative cap)");
  if (hb.overflow) return fail(WBPR_EOVERFLOW, "c(u->v) + c(v->u) over parallel arcs exceeds INT32_MAX");
  res.M = hb.M;
  auto t1 = std::chrono::steady_clock::now();

  const int chunk = 1024;
  e = c->state.ensure(wb::state_bytes(g->V, res.M_cap, chunk) + wb::misc_bytes() + 4096);
  if (e != hipSuccess) return hip_fail(e, "device allocation (state)");
  wb::State S;
  wb::state_carve(&S, g->V, res.M_cap, chunk, c->state.p);
  if (c->cfg.time_kernels && !c->ev) {
    c->ev = new (std::nothrow) hipEvent_t[wb::State::kMaxSweeps][4];
    c->gev = new (std::nothrow) hipEvent_t[wb::State::kMaxGR][2];
    if (!c->ev || !c->gev) return fail(WBPR_ENOMEM, "event table");
    for (int i = 0; i < wb::State::kMaxSweeps; i++)
      for (int k = 0; k < 4; k++) hipEventCreate(&c->ev[i][k]);
    for (int i = 0; i < wb::State::kMaxGR; i++)
      for (int k = 0; k < 2; k++) hipEventCreate(&c->gev[i][k]);
  }
  S.ev = c->ev;
  S.gev = c->gev;
  S.ev_count = 0;
  S.gev_count = 0;
  wb::SolveReport rep;
  std::string err;
  int rc = wb::solve_on_device(c->cfg, res, S, s, t, c->gr_blocks, st, c->pinned, dvalue, dflow, dside, g->cap, &rep,
                               &err);
  if (rc) return fail(rc, err);
  auto t2 = std::chrono::steady_clock::now();
  if (stats) {
    std::memset(stats, 0, sizeof(*stats));
    stats->V = g->V;
    stats->E = g->E;
    stats->M = res.M;
    stats->sweeps = rep.sweeps;
    stats->phase2_sweeps = rep.phase2_sweeps;
    stats->global_relabels = rep.global_relabels;
    stats->pushes = rep.pushes;
    stats->relabels = rep.relabels;
    stats->arc_scans = rep.arc_scans;
    stats->queued = rep.queued;
    stats->bfs_scans = rep.bfs_scans;
    stats->nonempty_sweeps = rep.nonempty_sweeps;
    stats->gr_levels = rep.gr_levels;
    stats->bfs_topdown_scans = rep.bfs_topdown_scans;
    stats->lanes_per_vertex = rep.lanes;
    stats->split_degree = rep.split_degree;
    stats->block_degree = rep.block_degree;
    stats->gr_every_sweeps = c->cfg.gr_every_sweeps > 0 ? c->cfg.gr_every_sweeps : 16;
    stats->grid_blocks = c->cfg.grid_blocks > 0 ? c->cfg.grid_blocks : 1024;
    stats->gr_blocks = rep.gr_blocks;
    stats->ms_build = std::chrono::duration<double, std::milli>(t1 - t0).count();
    stats->ms_phase1 = rep.ms_phase1;
    stats->ms_phase2 = rep.ms_phase2;
    stats->ms_decode = rep.ms_decode;
    stats->ms_total = std::chrono::duration<double, std::milli>(t2 - t0).count();
    for (int k = 0; k < 4; k++) {
      stats->kernel_ms[k] = rep.k_ms[k];
      stats->kernel_launches[k] = rep.k_launches[k];
      stats->kernel_arc_scans[k] = rep.k_scans[k];
      stats->kernel_pushes[k] = rep.k_pushes[k];
      stats->kernel_relabels[k] = rep.k_relabels[k];
      stats->kernel_queued[k] = rep.k_queued[k];
    }
  }
  if (stats) {
    // value for the stats block (one extra 8-byte read)
    long long v = 0;
    if (hipMemcpy(&v, dvalue, sizeof(v), hipMemcpyDeviceToHost) == hipSuccess) stats->value = v;
  }
  return WBPR_OK;
}

}  // namespace

extern "C" {

int wbpr_solve_device(wbpr_ctx *c, const wbpr_csr *g, int32_t s, int32_t t, void *stream, int64_t *dev_value,
                      int32_t *dev_arc_flow, uint8_t *dev_cut_side, wbpr_stats *stats) {
  if (!c) return fail(WBPR_EINVAL, "null context");
  int rc = check_graph_shape(g, s, t);
  if (rc) return rc;
  if (!dev_value) return fail(WBPR_EINVAL, "null value pointer");
  hipError_t e = hipSetDevice(c->device);
  if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
  hipStream_t st = stream ? (hipStream_t)stream : c->stream;
  return solve_dev(c, g, s, t, st, dev_value, dev_arc_flow, dev_cut_side, stats);
}

int wbpr_solve(wbpr_ctx *c, const wbpr_csr *g, int32_t s, int32_t t, int64_t *value, int32_t *arc_flow,
               uint8_t *cut_side, wbpr_stats *stats) {
  if (!c) return fail(WBPR_EINVAL, "null context");
  int rc = check_graph_shape(g, s, t);
  if (rc) return rc;
  if (!value) return fail(WBPR_EINVAL, "null value pointer");
  hipError_t e = hipSetDevice(c->device);
  if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
  const int64_t V = g->V, E = g->E;
  auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
  size_t in_bytes = al(8 * (V + 1)) + 2 * al(4 * (E > 0 ? E : 1));
  size_t out_bytes = al(8) + al(4 * (E > 0 ? E : 1)) + al((size_t)V);
  e = c->input.ensure(in_bytes);
  if (e == hipSuccess) e = c->output.ensure(out_bytes);
  if (e != hipSuccess) return hip_fail(e, "device allocation (staging)");
  char *ip = (char *)c->input.p;
  int64_t *d_rp = (int64_t *)ip;
  int32_t *d_col = (int32_t *)(ip + al(8 * (V + 1)));
  int32_t *d_cap = (int32_t *)(ip + al(8 * (V + 1)) + al(4 * (E > 0 ? E : 1)));
  char *op = (char *)c->output.p;
  int64_t *d_val = (int64_t *)op;
  int32_t *d_flow = (int32_t *)(op + al(8));
  uint8_t *d_side = (uint8_t *)(op + al(8) + al(4 * (E > 0 ? E : 1)));
  hipStream_t st = c->stream;
  e = hipMemcpyAsync(d_rp, g->row_ptr, 8 * (V + 1), hipMemcpyHostToDevice, st);
  if (e == hipSuccess && E > 0) e = hipMemcpyAsync(d_col, g->col, 4 * E, hipMemcpyHostToDevice, st);
  if (e == hipSuccess && E > 0) e = hipMemcpyAsync(d_cap, g->cap, 4 * E, hipMemcpyHostToDevice, st);
  if (e != hipSuccess) return hip_fail(e, "host to device copy");
  wbpr_csr dg{g->V, g->E, d_rp, d_col, d_cap};
  rc = solve_dev(c, &dg, s, t, st, d_val, arc_flow ? d_flow : nullptr, cut_side ? d_side : nullptr, stats);
  if (rc) return rc;
  e = hipMemcpyAsync(value, d_val, 8, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess && arc_flow && E > 0) e = hipMemcpyAsync(arc_flow, d_flow, 4 * E, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess && cut_side) e = hipMemcpyAsync(cut_side, d_side, (size_t)V, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return hip_fail(e, "device to host copy");
  return WBPR_OK;
}

}  // extern "C"
