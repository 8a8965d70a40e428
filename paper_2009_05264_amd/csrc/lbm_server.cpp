// Serving loop: flow-boiling solves of different sizes and parameters are
// submitted as they arrive, admitted in arrival order when their device
// footprint fits under the memory cap and a slot is free, kept resident in
// HBM, and stepped together -- all running requests advance in the same
// launches (one batch over their tile tables) -- until each reaches its step
// budget.  Admission and retirement happen between quanta of steps, so a
// request that arrives while others are on the device joins them at the
// next quantum (continuous batching).  A request whose fields turn
// non-finite is failed at the end of the quantum in which that happens and
// its memory freed; the others go on unaffected (each domain keeps its own
// state and reductions).  lbm_server_pump waits for its quantum;
// lbm_server_pump_async launches it and returns, and a later call retires
// it once an event recorded after it has completed, so the host can take in
// arrivals while the device works.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <deque>
#include <map>
#include <vector>

#include "../../include/lbmflow.h"
#include "lbm_internal.h"
#include "lbm_runtime.h"

#define HIPCHECK(expr)                                                                     \
  do {                                                                                     \
    hipError_t e_ = (expr);                                                                \
    if (e_ != hipSuccess)                                                                  \
      return lbm_fail(LBM_E_DEVICE, "%s failed: %s", #expr, hipGetErrorString(e_));        \
  } while (0)

namespace {

double now_s() {
  using namespace std::chrono;
  return duration<double>(steady_clock::now().time_since_epoch()).count();
}

struct Request {
  uint64_t id = 0;
  lbm_params P{};
  bool walls = false;
  std::vector<double> Ts, rs, Tn, rn;
  std::vector<int32_t> heat;
  bool has_heat = false;
  double rho_init = 1.0, T_init = 1.0, noise = 0.0;
  uint64_t seed = 0;
  int64_t budget = 0, remaining = 0;
  size_t footprint = 0;
  int state = LBM_REQ_QUEUED;
  int error = LBM_OK;  // why a request failed (LBM_E_NAN: fields turned non-finite)
  double t_submit = 0, t_start = 0, t_done = 0;
  lbm_domain* dom = nullptr;
};

}  // namespace

struct lbm_server {
  size_t cap = 0;
  int max_slots = 0;
  int64_t quantum = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  std::map<uint64_t, Request> reqs;
  std::deque<uint64_t> queue;     // arrival order
  std::vector<uint64_t> active;   // admission order
  lbm_batch* batch = nullptr;
  size_t resident = 0, peak = 0;
  int64_t done = 0, failed = 0;
  double lups = 0.0, busy = 0.0;
  uint64_t next_id = 1;
  // the quantum on the device, if any: its steps and nodes, and events
  // recorded before and after it on the server's stream
  bool inflight = false;
  int64_t inflight_q = 0;
  double inflight_nodes = 0.0;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
};

extern "C" int lbm_admission_plan(const size_t* footprints, int n, size_t cap, size_t used,
                                  int free_slots, int* admit, int* n_admit) {
  if (n < 0 || (n > 0 && (!footprints || !admit)) || !n_admit)
    return lbm_fail(LBM_E_INVALID, "bad admission-plan arguments");
  int k = 0;
  for (int i = 0; i < n && k < free_slots; ++i) {
    if (used <= cap && footprints[i] <= cap - used) {
      used += footprints[i];
      admit[k++] = i;
    }
  }
  *n_admit = k;
  return LBM_OK;
}

// The requests' domains keep the batch's tile heights: most of them join the
// next batch, whose automatic height is then usually the same.
static int drop_batch(lbm_server* s) {
  if (s->batch) {
    int rc = lbm_batch_release(s->batch, true);
    s->batch = nullptr;
    if (rc) return rc;
  }
  return LBM_OK;
}

static int start_request(lbm_server* s, Request& r) {
  lbm_domain* d = nullptr;
  int rc = lbm_create(&r.P, s->stream, nullptr, 0, &d);
  if (rc) return rc;
  if (r.walls) {
    rc = lbm_set_wall_maps(d, LBM_SIDE_S, r.Ts.data(), r.rs.data(), r.has_heat ? r.heat.data() : nullptr);
    if (!rc) rc = lbm_set_wall_maps(d, LBM_SIDE_N, r.Tn.data(), r.rn.data(), nullptr);
  }
  if (!rc) rc = lbm_init_fields(d, nullptr, nullptr, r.rho_init, r.T_init, r.noise, r.seed);
  if (rc) {
    lbm_destroy(d);
    return rc;
  }
  r.dom = d;
  r.state = LBM_REQ_RUNNING;
  r.t_start = now_s();
  return LBM_OK;
}

static void free_request(lbm_server* s, Request& r) {
  if (r.dom) {
    lbm_destroy(r.dom);
    r.dom = nullptr;
    s->resident -= r.footprint;
  }
}

extern "C" int lbm_server_create(size_t hbm_cap_bytes, int max_slots, int64_t quantum_steps,
                                 void* hip_stream, lbm_server** out) {
  if (!out) return lbm_fail(LBM_E_INVALID, "out is NULL");
  *out = nullptr;
  if (hbm_cap_bytes == 0 || max_slots <= 0 || quantum_steps <= 0)
    return lbm_fail(LBM_E_INVALID, "cap, slots and quantum must be positive");
  lbm_server* s = new lbm_server();
  s->cap = hbm_cap_bytes;
  s->max_slots = max_slots;
  s->quantum = quantum_steps;
  if (hip_stream) {
    s->stream = (hipStream_t)hip_stream;
  } else {
    hipError_t e = hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking);
    if (e != hipSuccess) {
      delete s;
      return lbm_fail(LBM_E_DEVICE, "hipStreamCreate failed: %s", hipGetErrorString(e));
    }
    s->own_stream = true;
  }
  *out = s;
  return LBM_OK;
}

extern "C" int lbm_server_submit(lbm_server* s, const lbm_params* p, const lbm_request* rq,
                                 int64_t step_budget, uint64_t* req_id) {
  if (!s || !p || !rq || !req_id) return lbm_fail(LBM_E_INVALID, "NULL argument");
  if (step_budget <= 0) return lbm_fail(LBM_E_INVALID, "step budget must be positive");
  size_t fp = 0;
  int rc = lbm_required_bytes(p, &fp);
  if (rc) return rc;
  if (fp > s->cap)
    return lbm_fail(LBM_E_CAP, "request needs %zu bytes, above the server cap of %zu", fp, s->cap);
  Request r;
  r.P = *p;
  r.walls = p->bc_y == LBM_BCY_WALLS;
  const int nx = p->nx;
  if (r.walls) {
    if (!rq->T_wall_s || !rq->rho_w_s || !rq->T_wall_n || !rq->rho_w_n)
      return lbm_fail(LBM_E_INVALID, "a walled request needs both wall maps");
    r.Ts.assign(rq->T_wall_s, rq->T_wall_s + nx);
    r.rs.assign(rq->rho_w_s, rq->rho_w_s + nx);
    r.Tn.assign(rq->T_wall_n, rq->T_wall_n + nx);
    r.rn.assign(rq->rho_w_n, rq->rho_w_n + nx);
    if (rq->heater) {
      r.heat.assign(rq->heater, rq->heater + nx);
      r.has_heat = true;
    }
  }
  r.rho_init = rq->rho_init;
  r.T_init = rq->T_init;
  r.noise = rq->noise;
  r.seed = rq->seed;
  r.budget = r.remaining = step_budget;
  r.footprint = fp;
  r.id = s->next_id++;
  r.t_submit = now_s();
  *req_id = r.id;
  s->queue.push_back(r.id);
  s->reqs.emplace(r.id, std::move(r));
  return LBM_OK;
}

// Admission, in arrival order, by footprint and free slots; the batch is
// rebuilt when the running set changed.  Then one quantum of the running
// requests is launched (not waited for).  *launched: whether one was.
static int launch_quantum(lbm_server* s, bool* launched) {
  *launched = false;
  bool changed = false;
  if (!s->queue.empty() && (int)s->active.size() < s->max_slots) {
    std::vector<size_t> fps;
    for (uint64_t id : s->queue) fps.push_back(s->reqs[id].footprint);
    std::vector<int> adm(fps.size());
    int na = 0;
    int rc = lbm_admission_plan(fps.data(), (int)fps.size(), s->cap, s->resident,
                                s->max_slots - (int)s->active.size(), adm.data(), &na);
    if (rc) return rc;
    if (na > 0) {
      rc = drop_batch(s);
      if (rc) return rc;
      std::vector<uint64_t> ids;
      for (int k = 0; k < na; ++k) ids.push_back(s->queue[adm[k]]);
      for (uint64_t id : ids) {
        Request& r = s->reqs[id];
        s->queue.erase(std::find(s->queue.begin(), s->queue.end(), id));
        const int src = start_request(s, r);
        if (src != LBM_OK) {
          r.state = LBM_REQ_FAILED;  // e.g. the device allocation failed; lbm_last_error says why
          r.error = src;
          ++s->failed;
          continue;
        }
        s->resident += r.footprint;
        s->peak = std::max(s->peak, s->resident);
        s->active.push_back(id);
        changed = true;
      }
    }
  }
  if (s->active.empty()) return LBM_OK;
  if (changed || !s->batch) {
    int rc = drop_batch(s);
    if (rc) return rc;
    std::vector<lbm_domain*> doms;
    for (uint64_t id : s->active) doms.push_back(s->reqs[id].dom);
    rc = lbm_batch_create(doms.data(), (int)doms.size(), nullptr, &s->batch);
    if (rc) return rc;
    // single launches: a graph would be captured for every running set, and
    // whatever follows a graph starts late (saturated stream 32 590 ->
    // 32 750 MLUPS; at 4 requests/s p99 time to solution 1.235 -> 1.209 s)
    lbm_batch_plain_launches(s->batch);
  }
  int64_t q = s->quantum;
  double nodes = 0;
  for (uint64_t id : s->active) {
    const Request& r = s->reqs[id];
    q = std::min(q, r.remaining);
    nodes += (double)r.P.nx * r.P.ny;
  }
  if (!s->ev0) {
    HIPCHECK(hipEventCreate(&s->ev0));
    HIPCHECK(hipEventCreate(&s->ev1));
  }
  HIPCHECK(hipEventRecord(s->ev0, s->stream));
  int rc = lbm_batch_step(s->batch, q);
  if (rc) return rc;
  HIPCHECK(hipEventRecord(s->ev1, s->stream));
  s->inflight = true;
  s->inflight_q = q;
  s->inflight_nodes = nodes;
  *launched = true;
  return LBM_OK;
}

// Retirement of the quantum on the device, which has completed: budgets,
// the non-finite check, requests done or failed.
static int finish_quantum(lbm_server* s) {
  s->inflight = false;
  const double t1 = now_s();
  float ms = 0.f;
  HIPCHECK(hipEventElapsedTime(&ms, s->ev0, s->ev1));
  s->busy += 1e-3 * (double)ms;
  const int64_t q = s->inflight_q;
  s->lups += s->inflight_nodes * (double)q;
  std::vector<uint64_t> still;
  bool retired = false;
  for (uint64_t id : s->active) {
    Request& r = s->reqs[id];
    r.remaining -= q;
    int bad = 0;
    int rc = lbm_nonfinite_seen(r.dom, &bad);
    if (rc) return rc;
    if (bad) {
      r.state = LBM_REQ_FAILED;
      r.error = LBM_E_NAN;
      r.t_done = t1;
      ++s->failed;
      retired = true;  // its domain is freed once the batch is dropped
      continue;
    }
    if (r.remaining == 0) {
      r.state = LBM_REQ_DONE;
      r.t_done = t1;
      ++s->done;
      retired = true;
    } else {
      still.push_back(id);
    }
  }
  if (retired) {
    int rc = drop_batch(s);  // releases the finished domains for read-out
    if (rc) return rc;
    for (uint64_t id : s->active) {
      Request& r = s->reqs[id];
      if (r.state == LBM_REQ_FAILED) free_request(s, r);
    }
  }
  s->active.swap(still);
  return LBM_OK;
}

// Waits for the quantum on the device, if any, and retires it.
static int settle(lbm_server* s) {
  if (!s->inflight) return LBM_OK;
  HIPCHECK(hipEventSynchronize(s->ev1));
  return finish_quantum(s);
}

extern "C" int lbm_server_pump(lbm_server* s, int* running) {
  if (!s) return lbm_fail(LBM_E_INVALID, "server is NULL");
  int rc = settle(s);
  bool launched = false;
  if (!rc) rc = launch_quantum(s, &launched);
  if (!rc && launched) rc = settle(s);
  if (running) *running = (int)s->active.size();
  return rc;
}

extern "C" int lbm_server_pump_async(lbm_server* s, int* running, int* in_flight) {
  if (!s) return lbm_fail(LBM_E_INVALID, "server is NULL");
  int rc = LBM_OK;
  if (s->inflight) {
    const hipError_t e = hipEventQuery(s->ev1);
    if (e == hipErrorNotReady) {
      if (running) *running = (int)s->active.size();
      if (in_flight) *in_flight = 1;
      return LBM_OK;
    }
    if (e != hipSuccess) return lbm_fail(LBM_E_DEVICE, "hipEventQuery failed: %s", hipGetErrorString(e));
    rc = finish_quantum(s);
  }
  bool launched = false;
  if (!rc) rc = launch_quantum(s, &launched);
  if (running) *running = (int)s->active.size();
  if (in_flight) *in_flight = s->inflight ? 1 : 0;
  return rc;
}

extern "C" int lbm_server_poll(lbm_server* s, uint64_t id, int* state, double* time_to_solution_s) {
  if (!s || !state) return lbm_fail(LBM_E_INVALID, "NULL argument");
  auto it = s->reqs.find(id);
  if (it == s->reqs.end()) return lbm_fail(LBM_E_INVALID, "unknown request %llu", (unsigned long long)id);
  *state = it->second.state;
  if (it->second.state == LBM_REQ_FAILED)
    lbm_fail(it->second.error, "request %llu failed (%s)", (unsigned long long)id,
             it->second.error == LBM_E_NAN ? "its fields turned non-finite" : "it could not be started");
  if (time_to_solution_s)
    *time_to_solution_s = it->second.state == LBM_REQ_DONE ? it->second.t_done - it->second.t_submit : -1.0;
  return LBM_OK;
}

static int finished_domain(lbm_server* s, uint64_t id, lbm_domain** d) {
  auto it = s->reqs.find(id);
  if (it == s->reqs.end()) return lbm_fail(LBM_E_INVALID, "unknown request %llu", (unsigned long long)id);
  if (it->second.state != LBM_REQ_DONE || !it->second.dom)
    return lbm_fail(LBM_E_STATE, "request %llu has no finished state to read", (unsigned long long)id);
  *d = it->second.dom;
  return LBM_OK;
}

extern "C" int lbm_server_read_fields(lbm_server* s, uint64_t id, double* rho, double* ux, double* uy,
                                      double* T) {
  if (!s) return lbm_fail(LBM_E_INVALID, "server is NULL");
  lbm_domain* d = nullptr;
  int rc = finished_domain(s, id, &d);
  return rc ? rc : lbm_read_fields(d, rho, ux, uy, T);
}

extern "C" int lbm_server_read_diag(lbm_server* s, uint64_t id, lbm_diag* out) {
  if (!s) return lbm_fail(LBM_E_INVALID, "server is NULL");
  lbm_domain* d = nullptr;
  int rc = finished_domain(s, id, &d);
  return rc ? rc : lbm_read_diag(d, out);
}

extern "C" int lbm_server_release(lbm_server* s, uint64_t id) {
  if (!s) return lbm_fail(LBM_E_INVALID, "server is NULL");
  auto it = s->reqs.find(id);
  if (it == s->reqs.end()) return lbm_fail(LBM_E_INVALID, "unknown request %llu", (unsigned long long)id);
  if (it->second.state != LBM_REQ_DONE)
    return lbm_fail(LBM_E_STATE, "request %llu is not finished", (unsigned long long)id);
  free_request(s, it->second);
  return LBM_OK;
}

extern "C" int lbm_server_cancel(lbm_server* s, uint64_t id) {
  if (!s) return lbm_fail(LBM_E_INVALID, "server is NULL");
  auto it = s->reqs.find(id);
  if (it == s->reqs.end()) return lbm_fail(LBM_E_INVALID, "unknown request %llu", (unsigned long long)id);
  Request& r = it->second;
  if (r.state == LBM_REQ_RUNNING) {
    int rc = settle(s);  // the quantum on the device first (it may finish or fail the request)
    if (rc) return rc;
  }
  if (r.state == LBM_REQ_QUEUED) {
    s->queue.erase(std::find(s->queue.begin(), s->queue.end(), id));
  } else if (r.state == LBM_REQ_RUNNING) {
    int rc = drop_batch(s);
    if (rc) return rc;
    s->active.erase(std::find(s->active.begin(), s->active.end(), id));
    free_request(s, r);
  } else {
    return LBM_OK;  // finished or already cancelled
  }
  r.state = LBM_REQ_CANCELLED;
  return LBM_OK;
}

extern "C" int lbm_server_stats(lbm_server* s, lbm_server_info* out) {
  if (!s || !out) return lbm_fail(LBM_E_INVALID, "NULL argument");
  out->queued = (int64_t)s->queue.size();
  out->running = (int64_t)s->active.size();
  out->done = s->done;
  out->failed = s->failed;
  out->resident_bytes = s->resident;
  out->peak_resident_bytes = s->peak;
  out->lups = s->lups;
  out->busy_seconds = s->busy;
  return LBM_OK;
}

extern "C" int lbm_server_destroy(lbm_server* s) {
  if (!s) return LBM_OK;
  if (s->inflight) (void)hipEventSynchronize(s->ev1);
  (void)drop_batch(s);
  for (auto& kv : s->reqs) free_request(s, kv.second);
  if (s->ev0) (void)hipEventDestroy(s->ev0);
  if (s->ev1) (void)hipEventDestroy(s->ev1);
  if (s->own_stream && s->stream) (void)hipStreamDestroy(s->stream);
  delete s;
  return LBM_OK;
}
