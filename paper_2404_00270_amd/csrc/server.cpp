// Continuous-batching server (wbpr_server_* in include/wbpr.h).
//
// One worker thread per server owns an Engine with a fixed arena carved from
// the HBM budget.  Its loop: admit a group of waiting requests that fits the
// free ranges (host staging -> device staging -> residual build, preflow),
// then solve, and copy the outputs of the instances that finished back to
// host buffers and hand them out.  Two ways to solve:
//
// * persistent (batch_kernel = 2): admitted instances are published to the device
//   ring of a persistent kernel that keeps running while requests arrive:
//   its workgroups claim instances one at a time (largest first within an
//   admission) and solve each whole, so a request admitted while others are
//   on the GPU starts as soon as a workgroup is free, without waiting for a
//   round.  The worker polls the kernel's results ring, relaunches the
//   kernel when it has exited (idle) and work waits, and gives instances too
//   large for it, or stopped at one of its caps, to the rounds below, which
//   run only while the kernel is not running;
// * rounds (the default): one engine round over everything resident
//   (multi-root global relabel, per-instance phase steps, one batch of
//   sweeps) per loop; requests that arrive meanwhile join the next round.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <thread>
#include <vector>

#include "wb_ctx.h"

namespace wb {
namespace {

using Clock = std::chrono::steady_clock;

double ms_between(Clock::time_point a, Clock::time_point b) {
  return std::chrono::duration<double, std::milli>(b - a).count();
}

size_t al(size_t x) { return (x + 255) & ~(size_t)255; }

// Arena bytes one instance occupies while resident (header formula).
int64_t footprint(int64_t V, int64_t E) { return 69 * V + 44 * E + (E + 31) / 32; }

// Device output block of a group: values [n], flows [sum E], sides [sum V].
size_t out_bytes(int32_t n, int64_t E, int64_t V) { return al(8 * (size_t)n) + al(4 * (size_t)std::max<int64_t>(E, 1)) + al((size_t)V); }

// Device / pinned input staging of a group: row pointers, columns, capacities.
size_t in_bytes(int32_t n, int64_t E, int64_t V) {
  return al(8 * (size_t)(V + n)) + 2 * al(4 * (size_t)std::max<int64_t>(E, 1));
}

struct Req {
  uint64_t ticket = 0;
  int32_t V = 0, s = 0, t = 0;
  int64_t E = 0;
  std::vector<int64_t> row_ptr;
  std::vector<int32_t> col, cap;
  Clock::time_point t_submit, t_admit;
  int skipped = 0;
};

struct GroupRec {
  std::vector<Req> reqs;
  int64_t out_at = 0;   // byte offset of the output block in the output buffer
  size_t out_n = 0;
  int64_t Et = 0, Vt = 0;
  int remaining = 0;
  std::vector<int64_t> eoff, voff;
};

}  // namespace
}  // namespace wb

struct wbpr_server {
  int device = 0;
  hipStream_t stream = nullptr;
  hipStream_t pk_stream = nullptr;  // the persistent kernel's own stream
  bool pk = true;                   // persistent mode (see above)
  std::unique_ptr<wb::Engine> engine;
  bool want_flows = true, want_sides = true;
  int32_t max_admit = 0, max_slots = 256;
  // capacities
  int64_t Vcap = 0, Mcap = 0, Ecap = 0, gV = 0, gE = 0;
  int32_t gn = 0;
  size_t arena_b = 0, scratch_b = 0, staging_b = 0, output_b = 0;
  // device / pinned buffers
  void *d_in = nullptr, *d_out = nullptr;
  char *h_in = nullptr;
  wb::RangeAlloc out_alloc;  // in 256-byte units of d_out
  // shared state (mutex)
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  bool stop = false;
  uint64_t next_ticket = 1;
  std::deque<wb::Req> pending;
  std::map<uint64_t, wbpr_result> done;
  std::map<uint64_t, bool> known;  // tickets issued and not yet fetched
  // counters (mutex)
  int64_t submitted = 0, completed = 0, failed = 0, resident = 0, rounds = 0, admissions = 0, sweeps = 0;
  int32_t peak_resident = 0;
  double busy_ms = 0;
  std::vector<double> latencies;
  // worker-only state
  std::map<uint64_t, wb::GroupRec> groups;
  uint64_t next_group = 1;
  std::thread worker;
};

namespace wb {
namespace {

void finish_req(wbpr_server *S, const Req &r, int status, int64_t value, int32_t *flow, uint8_t *side,
                Clock::time_point now, bool admitted) {
  wbpr_result res;
  std::memset(&res, 0, sizeof(res));
  res.ticket = r.ticket;
  res.status = status;
  res.V = r.V;
  res.E = r.E;
  res.value = value;
  res.arc_flow = flow;
  res.cut_side = side;
  res.latency_ms = ms_between(r.t_submit, now);
  res.queue_ms = admitted ? ms_between(r.t_submit, r.t_admit) : res.latency_ms;
  std::lock_guard<std::mutex> lk(S->mu);
  if (!S->known.count(r.ticket)) {  // abandoned by destroy
    std::free(flow);
    std::free(side);
    return;
  }
  S->done[r.ticket] = res;
  if (status == WBPR_OK) {
    S->completed++;
    S->latencies.push_back(res.latency_ms);
  } else {
    S->failed++;
  }
  S->cv_done.notify_all();
}

// Picks waiting requests that fit the free ranges, slots and group limits.
// A request passed over 8 times blocks later ones (no starvation).
std::vector<Req> pick_group(wbpr_server *S) {
  std::vector<Req> g;
  Engine &E = *S->engine;
  int64_t fV = E.free_vertices(), fM = E.free_entries(), fA = E.free_arcs();
  int32_t fs = E.free_slots();
  const int64_t fO = S->out_alloc.largest_free() * 256;
  int64_t sV = 0, sE = 0;
  std::lock_guard<std::mutex> lk(S->mu);
  for (auto it = S->pending.begin(); it != S->pending.end();) {
    const Req &r = *it;
    const int32_t n = (int32_t)g.size() + 1;
    if (n > fs || n > S->gn || (S->max_admit > 0 && n > S->max_admit)) break;
    const bool fits = n <= fs && n <= S->gn && (S->max_admit <= 0 || n <= S->max_admit) && sV + r.V <= fV &&
                      2 * (sE + r.E) <= fM && sE + r.E <= fA && sV + r.V <= S->gV && sE + r.E <= S->gE &&
                      (int64_t)out_bytes(n, sE + r.E, sV + r.V) <= fO;
    if (fits) {
      sV += r.V;
      sE += r.E;
      g.push_back(std::move(*it));
      it = S->pending.erase(it);
    } else {
      if (++it->skipped > 8) break;  // it goes first once space frees up
      ++it;
    }
  }
  return g;
}

// Stages a group and admits it.  Returns 0, or the status of a failed
// admission (the group's requests are not resident then).
int admit_group(wbpr_server *S, std::vector<Req> &reqs, uint64_t *gid_out, std::string *err) {
  const int32_t n = (int32_t)reqs.size();
  GroupRec G;
  G.eoff.assign(n + 1, 0);
  G.voff.assign(n + 1, 0);
  for (int i = 0; i < n; i++) {
    G.eoff[i + 1] = G.eoff[i] + reqs[i].E;
    G.voff[i + 1] = G.voff[i] + reqs[i].V;
  }
  G.Et = G.eoff[n];
  G.Vt = G.voff[n];
  // pinned staging: row pointers (V_i + 1 each), columns, capacities
  const size_t rp_b = al(8 * (size_t)(G.Vt + n)), c_b = al(4 * (size_t)std::max<int64_t>(G.Et, 1));
  int64_t *h_rp = (int64_t *)S->h_in;
  int32_t *h_col = (int32_t *)(S->h_in + rp_b);
  int32_t *h_cap = (int32_t *)(S->h_in + rp_b + c_b);
  std::vector<int32_t> V(n), s(n), t(n);
  std::vector<int64_t> E(n);
  int64_t ro = 0;
  for (int i = 0; i < n; i++) {
    const Req &r = reqs[i];
    std::memcpy(h_rp + ro, r.row_ptr.data(), 8 * ((size_t)r.V + 1));
    if (r.E) {
      std::memcpy(h_col + G.eoff[i], r.col.data(), 4 * (size_t)r.E);
      std::memcpy(h_cap + G.eoff[i], r.cap.data(), 4 * (size_t)r.E);
    }
    ro += r.V + 1;
    V[i] = r.V;
    E[i] = r.E;
    s[i] = r.s;
    t[i] = r.t;
  }
  char *d = (char *)S->d_in;
  hipError_t e = hipMemcpyAsync(d, h_rp, 8 * (size_t)ro, hipMemcpyHostToDevice, S->stream);
  if (e == hipSuccess && G.Et)
    e = hipMemcpyAsync(d + rp_b, h_col, 4 * (size_t)G.Et, hipMemcpyHostToDevice, S->stream);
  if (e == hipSuccess && G.Et)
    e = hipMemcpyAsync(d + rp_b + c_b, h_cap, 4 * (size_t)G.Et, hipMemcpyHostToDevice, S->stream);
  if (e != hipSuccess) {
    *err = std::string("input staging: ") + hipGetErrorString(e);
    return WBPR_EDEVICE;
  }
  // output block
  G.out_n = out_bytes(n, G.Et, G.Vt);
  const int64_t units = (int64_t)(G.out_n / 256);
  G.out_at = S->out_alloc.alloc(units);
  if (G.out_at < 0) {
    *err = "output space";
    return WBPR_EAGAIN;
  }
  char *ob = (char *)S->d_out + G.out_at * 256;
  GroupInput in;
  in.n = n;
  in.V = V.data();
  in.E = E.data();
  in.s = s.data();
  in.t = t.data();
  in.row_ptr = (const int64_t *)d;
  in.col = (const int32_t *)(d + rp_b);
  in.cap = (const int32_t *)(d + rp_b + c_b);
  in.values = (int64_t *)ob;
  in.persistent = S->pk;
  in.flows = S->want_flows ? (int32_t *)(ob + al(8 * (size_t)n)) : nullptr;
  in.sides = S->want_sides ? (uint8_t *)(ob + al(8 * (size_t)n) + al(4 * (size_t)std::max<int64_t>(G.Et, 1))) : nullptr;
  const uint64_t gid = S->next_group++;
  in.tag = gid;
  const int rc = S->engine->admit(in, S->stream, err);  // synchronises the stream
  if (rc) {
    S->out_alloc.release(G.out_at, units);
    return rc;
  }
  const auto now = Clock::now();
  for (auto &r : reqs) r.t_admit = now;
  G.remaining = n;
  G.reqs = std::move(reqs);
  S->groups.emplace(gid, std::move(G));
  *gid_out = gid;
  return 0;
}

// Copies the outputs of finished instances back and publishes the results.
int publish(wbpr_server *S, const std::vector<Finished> &fin, std::string *err) {
  struct Out {
    GroupRec *G;
    int idx;
    int64_t value;
    int32_t *flow;
    uint8_t *side;
  };
  std::vector<Out> outs;
  outs.reserve(fin.size());  // copy destinations must not move
  hipError_t e = hipSuccess;
  for (const Finished &f : fin) {
    GroupRec &G = S->groups.at(f.tag);
    const Req &r = G.reqs[f.index];
    char *ob = (char *)S->d_out + G.out_at * 256;
    Out o{&G, f.index, 0, nullptr, nullptr};
    if (S->want_flows && r.E) o.flow = (int32_t *)std::malloc(4 * (size_t)r.E);
    if (S->want_sides) o.side = (uint8_t *)std::malloc((size_t)r.V);
    if ((S->want_flows && r.E && !o.flow) || (S->want_sides && !o.side)) {
      std::free(o.flow);
      std::free(o.side);
      *err = "host allocation for results";
      return WBPR_ENOMEM;
    }
    outs.push_back(o);
    if (e == hipSuccess) e = hipMemcpyAsync(&outs.back().value, ob + 8 * (size_t)f.index, 8, hipMemcpyDeviceToHost, S->stream);
    if (e == hipSuccess && o.flow)
      e = hipMemcpyAsync(o.flow, ob + al(8 * G.reqs.size()) + 4 * (size_t)G.eoff[f.index], 4 * (size_t)r.E,
                         hipMemcpyDeviceToHost, S->stream);
    if (e == hipSuccess && o.side)
      e = hipMemcpyAsync(o.side,
                         ob + al(8 * G.reqs.size()) + al(4 * (size_t)std::max<int64_t>(G.Et, 1)) + G.voff[f.index],
                         (size_t)r.V, hipMemcpyDeviceToHost, S->stream);
  }
  if (fin.empty()) return 0;
  if (e == hipSuccess) e = hipStreamSynchronize(S->stream);
  if (e != hipSuccess) {
    for (auto &o : outs) {
      std::free(o.flow);
      std::free(o.side);
    }
    *err = std::string("result copy: ") + hipGetErrorString(e);
    return WBPR_EDEVICE;
  }
  const auto now = Clock::now();
  for (size_t k = 0; k < outs.size(); k++) {
    const Out &o = outs[k];
    const int status = fin[k].status;
    finish_req(S, o.G->reqs[o.idx], status, o.value, o.flow, o.side, now, true);
  }
  // release output blocks of groups with nothing left
  for (const Finished &f : fin) {
    auto it = S->groups.find(f.tag);
    if (it == S->groups.end()) continue;
    if (--it->second.remaining == 0) {
      S->out_alloc.release(it->second.out_at, (int64_t)(it->second.out_n / 256));
      S->groups.erase(it);
    }
  }
  std::lock_guard<std::mutex> lk(S->mu);
  S->resident -= (int64_t)fin.size();
  return 0;
}

// Fails every resident request and empties the engine (after a device or
// internal error in a round).
void fail_resident(wbpr_server *S, int status) {
  S->engine->abandon(S->stream);
  const auto now = Clock::now();
  for (auto &kv : S->groups)
    for (const Req &r : kv.second.reqs) finish_req(S, r, status, 0, nullptr, nullptr, now, true);
  S->groups.clear();
  S->out_alloc.reset(S->out_alloc.capacity());
  std::lock_guard<std::mutex> lk(S->mu);
  S->resident = 0;
}

void admit_waiting(wbpr_server *S) {
  std::string err;
  std::vector<Req> g = pick_group(S);
  if (g.empty()) return;
  std::vector<std::vector<Req>> tries;
  tries.push_back(std::move(g));
  while (!tries.empty()) {
    std::vector<Req> grp = std::move(tries.back());
    tries.pop_back();
    uint64_t gid = 0;
    const int n = (int)grp.size();
    const int rc = admit_group(S, grp, &gid, &err);
    if (rc == 0) {
      std::lock_guard<std::mutex> lk(S->mu);
      S->resident += n;
      S->admissions++;
      S->peak_resident = std::max<int32_t>(S->peak_resident, (int32_t)S->resident);
    } else if (rc == WBPR_EAGAIN) {
      std::lock_guard<std::mutex> lk(S->mu);
      for (auto it = grp.rbegin(); it != grp.rend(); ++it) S->pending.push_front(std::move(*it));
    } else if (n > 1 && (rc == WBPR_EINVAL || rc == WBPR_EOVERFLOW)) {
      // isolate the offending request: admit the others one by one
      for (auto &r : grp) {
        std::vector<Req> one;
        one.push_back(std::move(r));
        tries.push_back(std::move(one));
      }
    } else {
      const auto now = Clock::now();
      for (const Req &r : grp) finish_req(S, r, rc, 0, nullptr, nullptr, now, false);
    }
  }
}

// One engine round over the instances in the rounds; publishes what finished.
int run_round(wbpr_server *S, std::string *err) {
  std::vector<Finished> fin;
  const int64_t sw0 = S->engine->sweeps_run();
  int rc = S->engine->round(S->stream, &fin, err);
  {
    std::lock_guard<std::mutex> lk(S->mu);
    S->rounds++;
    S->sweeps += S->engine->sweeps_run() - sw0;
  }
  if (rc == 0) rc = publish(S, fin, err);
  return rc;
}

void worker_main(wbpr_server *S) {
  hipSetDevice(S->device);
  Engine &E = *S->engine;
  auto tick = Clock::now();
  bool was_busy = false;
  for (;;) {
    {
      std::unique_lock<std::mutex> lk(S->mu);
      auto now = Clock::now();
      if (was_busy) S->busy_ms += ms_between(tick, now);
      tick = now;
      if (S->pk && S->resident > 0) {
        // instances on the device: look at them again after a short wait
        // (or at once when a request arrives)
        S->cv_work.wait_for(lk, std::chrono::microseconds(100), [&] { return S->stop || !S->pending.empty(); });
      } else {
        S->cv_work.wait(lk, [&] { return S->stop || !S->pending.empty() || S->resident > 0; });
        tick = Clock::now();  // idle until now
      }
      if (S->stop) break;
      was_busy = true;
    }
    std::string err;
    int rc = 0;
    if (!S->pk) {
      admit_waiting(S);
      if (!E.idle()) rc = run_round(S, &err);
    } else {
      // while instances wait for the rounds, admit nothing: the persistent
      // kernel drains and exits, then the rounds run
      if (E.rounds_resident() == 0) admit_waiting(S);
      std::vector<Finished> fin;
      rc = E.pk_collect(S->stream, &fin, &err);
      if (rc == 0) rc = publish(S, fin, &err);
      if (rc == 0 && E.rounds_resident() > 0) {
        if (!E.pk_alive()) rc = run_round(S, &err);
      } else if (rc == 0) {
        rc = E.pk_ensure_running(S->pk_stream, &err);
      }
    }
    if (rc) {
      hipStreamSynchronize(S->pk_stream);  // the kernel drains (idle exit) before the arena is cleared
      fail_resident(S, rc);
    }
    {
      std::lock_guard<std::mutex> lk(S->mu);
      was_busy = S->resident > 0 || !S->pending.empty();
    }
  }
}

}  // namespace
}  // namespace wb

using wb::fail;
using wb::hip_fail;

extern "C" {

int wbpr_server_footprint(int32_t V, int64_t E, int64_t *bytes) {
  if (!bytes) return fail(WBPR_EINVAL, "null output");
  if (V < 0 || E < 0) return fail(WBPR_EINVAL, "negative size");
  *bytes = wb::footprint(V, E);
  return WBPR_OK;
}

int wbpr_server_create(wbpr_ctx *ctx, const wbpr_server_options *opt, wbpr_server **out) {
  if (!ctx || !out) return fail(WBPR_EINVAL, "null argument");
  *out = nullptr;
  wbpr_server_options o;
  std::memset(&o, 0, sizeof(o));
  if (opt) o = *opt;
  if (o.hbm_budget_bytes < 0 || o.max_slots < 0 || o.arcs_per_vertex < 0 || o.max_admit < 0)
    return fail(WBPR_EINVAL, "negative server option");
  const int64_t budget = o.hbm_budget_bytes > 0 ? o.hbm_budget_bytes : (1ll << 30);
  const int32_t slots = o.max_slots > 0 ? o.max_slots : 256;
  const int64_t R = o.arcs_per_vertex > 0 ? o.arcs_per_vertex : 8;
  // largest arena (Vcap vertices, R*Vcap arcs) whose arena, builder scratch
  // and staging for a group of half the arena, and outputs fit the budget
  auto total = [&](int64_t Vc) -> int64_t {
    const int64_t Ec = R * Vc, gV = std::max<int64_t>(Vc / 2, 2), gE = std::max<int64_t>(Ec / 2, 1);
    return (int64_t)wb::Engine::arena_bytes(Vc, 2 * Ec, Ec, slots) +
           (int64_t)wb::Engine::scratch_bytes(gV, gE, slots) + (int64_t)wb::in_bytes(slots, gE, gV) +
           (int64_t)wb::out_bytes(slots, Ec, Vc) + 3 * 256 * (int64_t)slots;
  };
  int64_t lo = 0, hi = (1ll << 29) / std::max<int64_t>(R, 1);
  while (lo < hi) {
    const int64_t mid = (lo + hi + 1) / 2;
    if (total(mid) <= budget) lo = mid; else hi = mid - 1;
  }
  if (lo < 64) return fail(WBPR_ETOOBIG, "HBM budget too small for a server arena");
  wbpr_server *S = new (std::nothrow) wbpr_server();
  if (!S) return fail(WBPR_ENOMEM, "host allocation");
  S->device = ctx->device;
  S->want_flows = o.want_flows != 0;
  S->want_sides = o.want_sides != 0;
  S->max_admit = o.max_admit;
  S->max_slots = slots;
  S->Vcap = lo;
  S->Ecap = R * lo;
  S->Mcap = 2 * S->Ecap;
  S->gV = std::max<int64_t>(lo / 2, 2);
  S->gE = std::max<int64_t>(S->Ecap / 2, 1);
  S->gn = slots;
  auto cleanup = [&](int rc, const std::string &msg) {
    wbpr_server_destroy(S);
    return fail(rc, msg);
  };
  hipError_t e = hipSetDevice(S->device);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&S->stream, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&S->pk_stream, hipStreamNonBlocking);
  if (e != hipSuccess) return cleanup(hip_fail(e, "server stream"), wb::g_err);
  S->pk = ctx->cfg.batch_kernel == 2 && !ctx->cfg.debug_checks;
  S->engine.reset(new (std::nothrow) wb::Engine(S->device));
  if (!S->engine) return cleanup(WBPR_ENOMEM, "engine");
  wb::SolveConfig cfg = ctx->cfg;
  cfg.time_kernels = false;
  cfg.max_sweeps = 0;
  cfg.max_wall_ms = 0;
  S->engine->set_config(cfg);
  std::string err;
  int rc = S->engine->reserve(S->Vcap, S->Mcap, S->Ecap, slots, S->gV, S->gE, slots, &err);
  if (rc) return cleanup(rc, err);
  S->arena_b = wb::Engine::arena_bytes(S->Vcap, S->Mcap, S->Ecap, slots);
  S->scratch_b = wb::Engine::scratch_bytes(S->gV, S->gE, slots);
  S->staging_b = wb::in_bytes(slots, S->gE, S->gV);
  S->output_b = wb::out_bytes(slots, S->Ecap, S->Vcap) + 3 * 256 * (size_t)slots;
  e = hipMalloc(&S->d_in, S->staging_b);
  if (e == hipSuccess) e = hipMalloc(&S->d_out, S->output_b);
  if (e == hipSuccess) e = hipHostMalloc((void **)&S->h_in, S->staging_b, hipHostMallocDefault);
  if (e != hipSuccess) return cleanup(hip_fail(e, "server buffers"), wb::g_err);
  S->out_alloc.reset((int64_t)(S->output_b / 256));
  try {
    S->worker = std::thread(wb::worker_main, S);
  } catch (...) {
    return cleanup(WBPR_ENOMEM, "worker thread");
  }
  *out = S;
  return WBPR_OK;
}

int wbpr_server_submit(wbpr_server *S, const wbpr_csr *g, int32_t s, int32_t t, uint64_t *ticket) {
  if (!S || !g || !ticket) return fail(WBPR_EINVAL, "null argument");
  int rc = wb::check_shape(g->V, g->E, s, t);
  if (rc) return rc;
  if (!g->row_ptr || (g->E > 0 && (!g->col || !g->cap))) return fail(WBPR_EINVAL, "null CSR array");
  if (g->V > S->gV || g->E > S->gE)
    return fail(WBPR_ETOOBIG, "instance larger than the server admits under its HBM budget");
  const int64_t V = g->V, E = g->E;
  if (g->row_ptr[0] != 0 || g->row_ptr[V] != E) return fail(WBPR_EINVAL, "row_ptr must run from 0 to E");
  for (int64_t v = 0; v < V; v++)
    if (g->row_ptr[v + 1] < g->row_ptr[v]) return fail(WBPR_EINVAL, "row_ptr not monotone");
  for (int64_t i = 0; i < E; i++) {
    if (g->col[i] < 0 || g->col[i] >= V) return fail(WBPR_EINVAL, "col out of range");
    if (g->cap[i] < 0) return fail(WBPR_EINVAL, "negative capacity");
  }
  wb::Req r;
  r.V = g->V;
  r.E = E;
  r.s = s;
  r.t = t;
  try {
    r.row_ptr.assign(g->row_ptr, g->row_ptr + V + 1);
    r.col.assign(g->col, g->col + E);
    r.cap.assign(g->cap, g->cap + E);
  } catch (...) {
    return fail(WBPR_ENOMEM, "host copy of the request");
  }
  r.t_submit = wb::Clock::now();
  {
    std::lock_guard<std::mutex> lk(S->mu);
    if (S->stop) return fail(WBPR_ECANCELED, "server stopping");
    r.ticket = S->next_ticket++;
    *ticket = r.ticket;
    S->known[r.ticket] = true;
    S->submitted++;
    S->pending.push_back(std::move(r));
  }
  S->cv_work.notify_one();
  return WBPR_OK;
}

int wbpr_server_poll(wbpr_server *S, uint64_t ticket, wbpr_result *out) {
  return wbpr_server_wait(S, ticket, 0, out);
}

int wbpr_server_wait(wbpr_server *S, uint64_t ticket, int32_t timeout_ms, wbpr_result *out) {
  if (!S || !out) return fail(WBPR_EINVAL, "null argument");
  std::unique_lock<std::mutex> lk(S->mu);
  if (!S->known.count(ticket)) return fail(WBPR_EINVAL, "unknown ticket");
  auto ready = [&] { return S->done.count(ticket) > 0; };
  if (timeout_ms < 0) {
    S->cv_done.wait(lk, ready);
  } else if (timeout_ms > 0) {
    S->cv_done.wait_for(lk, std::chrono::milliseconds(timeout_ms), ready);
  }
  auto it = S->done.find(ticket);
  if (it == S->done.end()) return fail(WBPR_EAGAIN, "pending");
  *out = it->second;
  S->done.erase(it);
  S->known.erase(ticket);
  return WBPR_OK;
}

void wbpr_result_free(wbpr_result *r) {
  if (!r) return;
  std::free(r->arc_flow);
  std::free(r->cut_side);
  r->arc_flow = nullptr;
  r->cut_side = nullptr;
}

int wbpr_server_get_stats(wbpr_server *S, wbpr_server_stats *out) {
  if (!S || !out) return fail(WBPR_EINVAL, "null argument");
  std::memset(out, 0, sizeof(*out));
  std::vector<double> lat;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    out->submitted = S->submitted;
    out->completed = S->completed;
    out->failed = S->failed;
    out->pending = (int64_t)S->pending.size();
    out->resident = S->resident;
    out->rounds = S->rounds;
    out->admissions = S->admissions;
    out->sweeps = S->sweeps;
    out->busy_ms = S->busy_ms;
    out->peak_resident = S->peak_resident;
    lat = S->latencies;
  }
  out->solves_per_s = out->busy_ms > 0 ? out->completed / (out->busy_ms / 1e3) : 0;
  if (!lat.empty()) {
    std::sort(lat.begin(), lat.end());
    auto pct = [&](double q) {  // nearest rank
      size_t k = (size_t)std::ceil(q * (double)lat.size());
      if (k < 1) k = 1;
      return lat[std::min(k, lat.size()) - 1];
    };
    out->p50_ms = pct(0.50);
    out->p99_ms = pct(0.99);
    out->max_ms = lat.back();
  }
  out->arena_bytes = (int64_t)S->arena_b;
  out->scratch_bytes = (int64_t)S->scratch_b;
  out->staging_bytes = (int64_t)S->staging_b;
  out->output_bytes = (int64_t)S->output_b;
  out->Vcap = S->Vcap;
  out->Mcap = S->Mcap;
  out->Ecap = S->Ecap;
  out->max_slots = S->max_slots;
  return WBPR_OK;
}

void wbpr_server_destroy(wbpr_server *S) {
  if (!S) return;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    S->stop = true;
    S->known.clear();  // results of unfinished requests are dropped
    for (auto &kv : S->done) wbpr_result_free(&kv.second);
    S->done.clear();
    S->pending.clear();
  }
  S->cv_work.notify_all();
  S->cv_done.notify_all();
  if (S->worker.joinable()) S->worker.join();
  hipSetDevice(S->device);
  if (S->pk_stream) hipStreamSynchronize(S->pk_stream);  // the persistent kernel exits when idle
  if (S->stream) hipStreamSynchronize(S->stream);
  S->engine.reset();
  if (S->d_in) hipFree(S->d_in);
  if (S->d_out) hipFree(S->d_out);
  if (S->h_in) hipHostFree(S->h_in);
  if (S->stream) hipStreamDestroy(S->stream);
  if (S->pk_stream) hipStreamDestroy(S->pk_stream);
  delete S;
}

}  // extern "C"
