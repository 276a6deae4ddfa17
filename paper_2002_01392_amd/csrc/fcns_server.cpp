// Serving engine: a request loop over independent solves of different grid
// sizes.  Requests are admitted in arrival order as soon as a slot and device
// memory allow (first fit: a request that does not fit yet does not block the
// ones behind it), run on solver contexts that stay resident and are reused by
// later requests of the same shape, and overlap on the device through one
// non-blocking HIP stream per context.  A running request keeps up to
// kLookahead steps enqueued; each poll collects the completed ones (their
// non-finite flag included) and tops the queue up, so a cancelled or
// blown-up request stops within a few steps and frees its slot.  Every step
// of every request is bracketed by HIP events, so step latency under load is
// measured on the device; request latency is measured on the host clock from
// submission to the detection of the finished result.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <string>
#include <vector>

#include "../../include/fcns.h"

namespace {

using Clock = std::chrono::steady_clock;

struct PoolCtx {
  fcns_ctx* ctx = nullptr;
  hipStream_t stream = nullptr;
  std::string key;
  int64_t bytes = 0;        // device bytes held (solver + staging)
  double* dphys = nullptr;  // device staging: 3 velocity fields then theta
  double* hphys = nullptr;  // pinned host staging of the same size
  int64_t npts = 0;         // points of one physical field
  int nphys = 3;            // physical fields staged (3, or 4 with theta)
  bool busy = false;
  uint64_t last_used = 0;
};

enum { Q_QUEUED = 0, Q_RUNNING, Q_FINISHING, Q_DONE };

// steps of one request on its stream ahead of the host
constexpr int kLookahead = 3;

struct Request {
  int64_t id = 0;
  fcns_problem prob{};
  std::vector<double> table;
  const double* v0 = nullptr;  // caller's host arrays (read at admission)
  const double* th0 = nullptr;
  double* v_out = nullptr;     // caller's host arrays (written when done)
  double* th_out = nullptr;
  double dt = 0.0;
  int nsteps = 0;
  int enq = 0;               // steps enqueued
  int done_steps = 0;        // steps known complete
  bool cancel = false;       // stop enqueuing; finish as ECANCELED
  bool nonfinite = false;    // a completed step left a non-finite state
  double t_submit = 0.0, t_admit = -1.0, t_done = -1.0;
  int state = Q_QUEUED;
  PoolCtx* pc = nullptr;
  std::vector<hipEvent_t> ev;
  hipEvent_t fin = nullptr;
  std::vector<float> step_ms;
  fcns_status status = FCNS_OK;
  std::string err;
};

std::string shape_key(const fcns_problem& p, const std::vector<double>& table) {
  char buf[512];
  snprintf(buf, sizeof(buf), "%d %d %d %.17g %.17g %.17g %d %d %d %d %d %.17g %.17g", p.nx, p.ny,
           p.nz, p.lx, p.ly, p.lz, p.fc_d, p.fc_C, p.boussinesq, p.rk_order, p.precision,
           p.filter_beta, p.filter_2p);
  // the continuation table is part of the shape (contexts copy it at create)
  uint64_t h = 1469598103934665603ULL;
  for (double x : table) {
    uint64_t b;
    memcpy(&b, &x, 8);
    h = (h ^ b) * 1099511628211ULL;
  }
  return std::string(buf) + " " + std::to_string(h);
}

}  // namespace

struct fcns_server {
  int max_active = 1;
  int64_t max_bytes = 0;
  int64_t used_bytes = 0;
  Clock::time_point t0;
  std::vector<std::unique_ptr<PoolCtx>> pool;
  std::map<int64_t, std::unique_ptr<Request>> reqs;
  std::deque<int64_t> queue;
  std::vector<int64_t> active;
  int64_t next_id = 1;
  int64_t n_done = 0;
  uint64_t tick = 0;
  std::string err;
  std::map<std::string, std::string> choices;   // shape key -> tuned launch choices
  int max_large = 0;          // > 0: at most this many running requests of
  int64_t large_points = 0;   // at least large_points grid points

  double now() const { return std::chrono::duration<double>(Clock::now() - t0).count(); }
};

static fcns_status srv_fail(fcns_server* s, fcns_status st, const std::string& m) {
  if (s) s->err = m;
  return st;
}

static void destroy_pool_ctx(fcns_server* s, PoolCtx* pc) {
  if (pc->ctx) fcns_destroy(pc->ctx);
  if (pc->dphys) (void)hipFree(pc->dphys);
  if (pc->hphys) (void)hipHostFree(pc->hphys);
  if (pc->stream) (void)hipStreamDestroy(pc->stream);
  s->used_bytes -= pc->bytes;
}

extern "C" fcns_status fcns_server_create(int32_t max_active, int64_t max_bytes,
                                          fcns_server** out) {
  if (!out) return FCNS_EINVAL;
  *out = nullptr;
  if (max_active < 1 || max_bytes <= 0) return FCNS_EINVAL;
  fcns_server* s = new fcns_server();
  s->max_active = max_active;
  s->max_bytes = max_bytes;
  s->t0 = Clock::now();
  *out = s;
  return FCNS_OK;
}

extern "C" double fcns_server_now(const fcns_server* s) { return s ? s->now() : 0.0; }

extern "C" fcns_status fcns_server_set_mix(fcns_server* s, int32_t max_large,
                                           int64_t large_points) {
  if (!s) return FCNS_EINVAL;
  if (max_large < 0 || (max_large > 0 && large_points < 1))
    return srv_fail(s, FCNS_EINVAL, "need max_large >= 0 and large_points >= 1");
  s->max_large = max_large;
  s->large_points = large_points;
  return FCNS_OK;
}

extern "C" fcns_status fcns_server_set_choices(fcns_server* s, const fcns_problem* prob,
                                               const char* choices) {
  if (!s) return FCNS_EINVAL;
  if (!prob || !prob->fc_table || !choices) return srv_fail(s, FCNS_EINVAL, "NULL argument");
  int64_t need = 0;
  if (fcns_footprint(prob, &need) != FCNS_OK) return srv_fail(s, FCNS_EINVAL, "bad problem");
  const int d = prob->fc_d, C = prob->fc_C;
  std::vector<double> table(prob->fc_table, prob->fc_table + (size_t)d * d + (size_t)C * d);
  fcns_problem p = *prob;
  p.fc_table = nullptr;
  s->choices[shape_key(p, table)] = choices;
  return FCNS_OK;
}

extern "C" fcns_status fcns_server_submit(fcns_server* s, const fcns_problem* prob,
                                          const double* v0, const double* theta0, double dt,
                                          int32_t nsteps, double* v_out, double* theta_out,
                                          int64_t* id) {
  if (!s) return FCNS_EINVAL;
  if (!prob || !v0 || !v_out || !id || !prob->fc_table)
    return srv_fail(s, FCNS_EINVAL, "NULL argument");
  if (prob->boussinesq && (!theta0 || !theta_out))
    return srv_fail(s, FCNS_EINVAL, "theta0 and theta_out required");
  if (!(dt > 0.0) || nsteps < 1) return srv_fail(s, FCNS_EINVAL, "need dt > 0 and nsteps >= 1");
  int64_t need = 0;
  if (fcns_footprint(prob, &need) != FCNS_OK) return srv_fail(s, FCNS_EINVAL, "bad problem");
  auto r = std::make_unique<Request>();
  r->id = s->next_id++;
  r->prob = *prob;
  const int d = prob->fc_d, C = prob->fc_C;
  r->table.assign(prob->fc_table, prob->fc_table + (size_t)d * d + (size_t)C * d);
  r->prob.fc_table = nullptr;
  r->v0 = v0;
  r->th0 = prob->boussinesq ? theta0 : nullptr;
  r->v_out = v_out;
  r->th_out = prob->boussinesq ? theta_out : nullptr;
  r->dt = dt;
  r->nsteps = nsteps;
  r->t_submit = s->now();
  *id = r->id;
  s->queue.push_back(r->id);
  s->reqs[r->id] = std::move(r);
  return FCNS_OK;
}

// a free resident context of this shape, or a new one if memory allows
// (evicting idle contexts of other shapes, least recently used first)
static PoolCtx* acquire(fcns_server* s, Request& r, const std::string& key, fcns_status& st) {
  st = FCNS_OK;
  PoolCtx* best = nullptr;
  for (auto& pc : s->pool)
    if (!pc->busy && pc->key == key) {
      best = pc.get();
      break;
    }
  if (best) return best;
  int64_t need = 0;
  fcns_footprint(&r.prob, &need);
  const int nphys = r.prob.boussinesq ? 4 : 3;
  const int64_t npts = (int64_t)r.prob.nx * r.prob.ny * r.prob.nz;
  need += (int64_t)nphys * npts * 8;
  if (need > s->max_bytes) {
    st = FCNS_ENOMEM;
    return nullptr;
  }
  while (s->used_bytes + need > s->max_bytes) {
    PoolCtx* victim = nullptr;
    for (auto& pc : s->pool)
      if (!pc->busy && (!victim || pc->last_used < victim->last_used)) victim = pc.get();
    if (!victim) return nullptr;  // wait for a running request to finish
    destroy_pool_ctx(s, victim);
    s->pool.erase(std::find_if(s->pool.begin(), s->pool.end(),
                               [&](const std::unique_ptr<PoolCtx>& p) { return p.get() == victim; }));
  }
  auto pc = std::make_unique<PoolCtx>();
  pc->key = key;
  pc->npts = npts;
  pc->nphys = nphys;
  if (hipStreamCreateWithFlags(&pc->stream, hipStreamNonBlocking) != hipSuccess) {
    st = FCNS_EDEVICE;
    return nullptr;
  }
  fcns_problem p = r.prob;
  p.fc_table = r.table.data();
  if ((st = fcns_create(&p, pc->stream, &pc->ctx)) != FCNS_OK) {
    s->err = std::string("context: ") + fcns_last_error(nullptr);
    (void)hipStreamDestroy(pc->stream);
    return nullptr;
  }
  // rk_step stays asynchronous; the flag is read as each step completes
  (void)fcns_set_finite_check(pc->ctx, FCNS_CHECK_DEFERRED);
  // launch choices tuned for this shape beforehand (fcns_server_set_choices)
  const auto ch = s->choices.find(key);
  if (ch != s->choices.end() && (st = fcns_set_choices(pc->ctx, ch->second.c_str())) != FCNS_OK) {
    s->err = std::string("choices: ") + fcns_last_error(pc->ctx);
    fcns_destroy(pc->ctx);
    (void)hipStreamDestroy(pc->stream);
    return nullptr;
  }
  const size_t sb = (size_t)nphys * npts * sizeof(double);
  if (hipMalloc((void**)&pc->dphys, sb) != hipSuccess ||
      hipHostMalloc((void**)&pc->hphys, sb, hipHostMallocDefault) != hipSuccess) {
    pc->bytes = 0;
    destroy_pool_ctx(s, pc.get());
    st = FCNS_ENOMEM;
    return nullptr;
  }
  pc->bytes = need;
  s->used_bytes += need;
  s->pool.push_back(std::move(pc));
  return s->pool.back().get();
}

static void finish_with_error(fcns_server* s, Request& r, fcns_status st, const std::string& m) {
  r.status = st;
  r.err = m;
  r.state = Q_DONE;
  r.t_done = s->now();
  s->n_done++;
}

static fcns_status launch_request(fcns_server* s, Request& r) {
  PoolCtx* pc = r.pc;
  fcns_ctx* c = pc->ctx;
  const size_t n = (size_t)pc->npts;
  fcns_status st = fcns_set_params(c, r.prob.nu, r.prob.kappa, r.prob.gamma, r.prob.forcing_x);
  if (st != FCNS_OK) return st;
  // straight from the caller's (pageable) arrays: the runtime stages the copy
  if (hipMemcpyAsync(pc->dphys, r.v0, 3 * n * sizeof(double), hipMemcpyHostToDevice,
                     pc->stream) != hipSuccess)
    return FCNS_EDEVICE;
  if (pc->nphys == 4 && hipMemcpyAsync(pc->dphys + 3 * n, r.th0, n * sizeof(double),
                                       hipMemcpyHostToDevice, pc->stream) != hipSuccess)
    return FCNS_EDEVICE;
  if ((st = fcns_set_state(c, pc->dphys, pc->nphys == 4 ? pc->dphys + 3 * n : nullptr)) != FCNS_OK)
    return st;
  r.ev.assign(r.nsteps + 1, nullptr);
  for (auto& e : r.ev)
    if (hipEventCreate(&e) != hipSuccess) return FCNS_EDEVICE;
  if (hipEventCreateWithFlags(&r.fin, hipEventDisableTiming) != hipSuccess) return FCNS_EDEVICE;
  (void)hipEventRecord(r.ev[0], pc->stream);
  r.enq = r.done_steps = 0;
  return FCNS_OK;
}

// Keep up to kLookahead steps of a running request on its stream.
static fcns_status top_up(Request& r) {
  while (!r.cancel && !r.nonfinite && r.enq < r.nsteps && r.enq - r.done_steps < kLookahead) {
    fcns_status st = fcns_rk_step(r.pc->ctx, r.dt, 1);
    if (st != FCNS_OK) return st;
    if (hipEventRecord(r.ev[r.enq + 1], r.pc->stream) != hipSuccess) return FCNS_EDEVICE;
    r.enq++;
  }
  return FCNS_OK;
}

static void release_events(Request& r) {
  for (auto e : r.ev)
    if (e) (void)hipEventDestroy(e);
  r.ev.clear();
  if (r.fin) (void)hipEventDestroy(r.fin);
  r.fin = nullptr;
}

extern "C" fcns_status fcns_server_poll(fcns_server* s, int32_t* n_queued, int32_t* n_active,
                                        int64_t* n_done) {
  if (!s) return FCNS_EINVAL;
  // 1. progress of the admitted requests
  for (size_t i = 0; i < s->active.size();) {
    Request& r = *s->reqs[s->active[i]];
    bool remove = false;
    if (r.state == Q_RUNNING) {
      hipError_t q = hipSuccess;
      while (r.done_steps < r.enq && (q = hipEventQuery(r.ev[r.done_steps + 1])) == hipSuccess)
        r.done_steps++;
      // the flag is sticky until set_state, so its latest host copy covers
      // every step completed so far
      if (r.done_steps > 0 && fcns_nonfinite_flag(r.pc->ctx)) r.nonfinite = true;
      fcns_status st = FCNS_OK;
      if (q != hipSuccess && q != hipErrorNotReady) {
        finish_with_error(s, r, FCNS_EDEVICE, hipGetErrorString(q));
        remove = true;
      } else if ((st = top_up(r)) != FCNS_OK) {
        finish_with_error(s, r, st, fcns_last_error(r.pc->ctx));
        remove = true;
      } else if (r.done_steps == r.enq) {
        // nothing of this request is left on the device
        r.step_ms.resize(r.done_steps);
        for (int k = 0; k < r.done_steps; ++k) {
          float ms = 0.f;
          (void)hipEventElapsedTime(&ms, r.ev[k], r.ev[k + 1]);
          r.step_ms[k] = ms;
        }
        if (r.cancel) {
          finish_with_error(s, r, FCNS_ECANCELED, "cancelled");
          remove = true;
        } else if (r.nonfinite) {
          finish_with_error(s, r, FCNS_ENONFINITE, "non-finite state");
          remove = true;
        } else {
          PoolCtx* pc = r.pc;
          const size_t n = (size_t)pc->npts;
          st = fcns_get_state(pc->ctx, pc->dphys, pc->nphys == 4 ? pc->dphys + 3 * n : nullptr,
                              nullptr);
          if (st == FCNS_OK &&
              hipMemcpyAsync(pc->hphys, pc->dphys, pc->nphys * n * sizeof(double),
                             hipMemcpyDeviceToHost, pc->stream) == hipSuccess &&
              hipEventRecord(r.fin, pc->stream) == hipSuccess) {
            r.state = Q_FINISHING;
          } else {
            finish_with_error(s, r, st == FCNS_OK ? FCNS_EDEVICE : st, "result copy failed");
            remove = true;
          }
        }
      }
    }
    if (r.state == Q_FINISHING) {
      const hipError_t q = hipEventQuery(r.fin);
      if (q == hipSuccess) {
        PoolCtx* pc = r.pc;
        const size_t n = (size_t)pc->npts;
        memcpy(r.v_out, pc->hphys, 3 * n * sizeof(double));
        if (pc->nphys == 4) memcpy(r.th_out, pc->hphys + 3 * n, n * sizeof(double));
        // every step's state passed the device check (all fields)
        r.status = FCNS_OK;
        r.state = Q_DONE;
        r.t_done = s->now();
        s->n_done++;
        remove = true;
      } else if (q != hipErrorNotReady) {
        finish_with_error(s, r, FCNS_EDEVICE, hipGetErrorString(q));
        remove = true;
      }
    }
    if (remove) {
      release_events(r);
      if (r.pc) {
        r.pc->busy = false;
        r.pc->last_used = ++s->tick;
        r.pc = nullptr;
      }
      s->active.erase(s->active.begin() + i);
    } else {
      ++i;
    }
  }
  // 2. admission, first fit in arrival order; with a mix limit, a large
  // request waits (keeping its place) while max_large of them run, and
  // smaller ones behind it go ahead
  auto is_large = [&](const Request& q) {
    return s->max_large > 0 && (int64_t)q.prob.nx * q.prob.ny * q.prob.nz >= s->large_points;
  };
  int n_large = 0;
  for (int64_t id : s->active) n_large += is_large(*s->reqs[id]) ? 1 : 0;
  for (auto it = s->queue.begin(); it != s->queue.end() && (int)s->active.size() < s->max_active;) {
    Request& r = *s->reqs[*it];
    if (is_large(r) && n_large >= s->max_large) {
      ++it;
      continue;
    }
    fcns_status st;
    PoolCtx* pc = acquire(s, r, shape_key(r.prob, r.table), st);
    if (!pc) {
      if (st != FCNS_OK) {  // can never run: report it
        finish_with_error(s, r, st, s->err.empty() ? "does not fit" : s->err);
        it = s->queue.erase(it);
      } else {
        ++it;
      }
      continue;
    }
    pc->busy = true;
    pc->last_used = ++s->tick;
    r.pc = pc;
    r.t_admit = s->now();
    if ((st = launch_request(s, r)) != FCNS_OK) {
      finish_with_error(s, r, st, fcns_last_error(pc->ctx));
      release_events(r);
      pc->busy = false;
      r.pc = nullptr;
    } else if ((st = top_up(r)) != FCNS_OK) {
      finish_with_error(s, r, st, fcns_last_error(pc->ctx));
      (void)hipStreamSynchronize(pc->stream);
      release_events(r);
      pc->busy = false;
      r.pc = nullptr;
    } else {
      r.state = Q_RUNNING;
      s->active.push_back(r.id);
      n_large += is_large(r) ? 1 : 0;
    }
    it = s->queue.erase(it);
  }
  if (n_queued) *n_queued = (int32_t)s->queue.size();
  if (n_active) *n_active = (int32_t)s->active.size();
  if (n_done) *n_done = s->n_done;
  return FCNS_OK;
}

extern "C" fcns_status fcns_server_result(fcns_server* s, int64_t id, double* stats) {
  if (!s) return FCNS_EINVAL;
  auto f = s->reqs.find(id);
  if (f == s->reqs.end()) return srv_fail(s, FCNS_EINVAL, "unknown request");
  Request& r = *f->second;
  if (r.state != Q_DONE) return srv_fail(s, FCNS_ESTATE, "request not finished");
  if (r.status != FCNS_OK && r.status != FCNS_ENONFINITE && r.status != FCNS_ECANCELED)
    return srv_fail(s, r.status, r.err);
  if (stats) {
    std::vector<float> sm = r.step_ms;
    std::sort(sm.begin(), sm.end());
    double sum = 0.0;
    for (float x : sm) sum += x;
    const auto pct = [&](double q) {
      if (sm.empty()) return 0.0;
      const size_t k = (size_t)std::min<double>(sm.size() - 1, std::ceil(q * sm.size()) - 1);
      return (double)sm[k];
    };
    stats[0] = r.t_submit;
    stats[1] = r.t_admit;
    stats[2] = r.t_done;
    stats[3] = sm.empty() ? 0.0 : sum / sm.size();
    stats[4] = pct(0.5);
    stats[5] = sm.empty() ? 0.0 : (double)sm.back();
  }
  return r.status;
}

extern "C" fcns_status fcns_server_step_times(fcns_server* s, int64_t id, int32_t max, float* ms,
                                              int32_t* n) {
  if (!s || !n) return FCNS_EINVAL;
  auto f = s->reqs.find(id);
  if (f == s->reqs.end()) return srv_fail(s, FCNS_EINVAL, "unknown request");
  const Request& r = *f->second;
  if (r.state != Q_DONE) return srv_fail(s, FCNS_ESTATE, "request not finished");
  const int k = std::min<int>(max, (int)r.step_ms.size());
  if (ms) memcpy(ms, r.step_ms.data(), k * sizeof(float));
  *n = k;
  return FCNS_OK;
}

extern "C" fcns_status fcns_server_cancel(fcns_server* s, int64_t id) {
  if (!s) return FCNS_EINVAL;
  auto f = s->reqs.find(id);
  if (f == s->reqs.end()) return srv_fail(s, FCNS_EINVAL, "unknown request");
  Request& r = *f->second;
  if (r.state == Q_QUEUED) {
    s->queue.erase(std::find(s->queue.begin(), s->queue.end(), id));
    finish_with_error(s, r, FCNS_ECANCELED, "cancelled");
  } else if (r.state == Q_RUNNING) {
    r.cancel = true;   // the next poll finishes it once its steps are done
  }
  return FCNS_OK;
}

extern "C" fcns_status fcns_server_release(fcns_server* s, int64_t id) {
  if (!s) return FCNS_EINVAL;
  auto f = s->reqs.find(id);
  if (f == s->reqs.end()) return FCNS_EINVAL;
  if (f->second->state != Q_DONE) return srv_fail(s, FCNS_ESTATE, "request not finished");
  s->reqs.erase(f);
  return FCNS_OK;
}

extern "C" fcns_status fcns_server_destroy(fcns_server* s) {
  if (!s) return FCNS_OK;
  for (auto& pc : s->pool)
    if (pc->stream) (void)hipStreamSynchronize(pc->stream);
  for (auto& kv : s->reqs) release_events(*kv.second);
  for (auto& pc : s->pool) destroy_pool_ctx(s, pc.get());
  delete s;
  return FCNS_OK;
}

extern "C" const char* fcns_server_last_error(const fcns_server* s) {
  return s ? s->err.c_str() : "";
}
