// lbm_ehd_serve.cpp -- continuous-batching request server for droplet
// simulations (declarations and documentation in include/lbm_ehd.h).
//
// Built only on the library's public C ABI: every admitted request is a
// simulation whose state the library allocates and keeps resident in HBM;
// all running requests are members of one batch, advanced by one sweep
// launch per step (graph-captured blocks).  Between blocks the scheduler
// retires finished requests (their results are read, their memory is freed
// on release) and admits queued ones, first fit in arrival order, while the
// sum of the footprints stays within the HBM budget.
#include <algorithm>
#include <chrono>
#include <cstring>
#include <deque>
#include <map>
#include <new>
#include <string>
#include <vector>

#include "lbm_ehd.h"

namespace {

struct Request {
  int64_t id = 0;
  lbm_ehd_params P;
  double xc = 0, yc = 0, radius = 0, noise = 0;
  uint64_t seed = 0;
  int64_t steps_total = 0, steps_done = 0;
  int32_t state = LBM_REQ_QUEUED;
  size_t footprint = 0;
  double t_submit = 0, t_start = -1, t_done = -1;
  lbm_ehd* sim = nullptr;
  lbm_ehd_diag diag;
  std::string error;
};

}  // namespace

struct lbm_ehd_server {
  size_t budget = 0;
  size_t used = 0;               // footprints of running and finished, unreleased requests
  int32_t block_steps = 256;
  lbm_ehd_batch* batch = nullptr;
  std::map<int64_t, Request> req;
  std::deque<int64_t> queue;     // arrival order
  std::vector<int64_t> running;
  int64_t next_id = 1;
  std::chrono::steady_clock::time_point t0;
  double now() const {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }
};

namespace {

thread_local std::string g_serr;

lbm_status serr(lbm_status code, const std::string& msg) {
  g_serr = msg;
  return code;
}

// Launch shape for the current members: strips of 256 columns when most of
// the cells are in grids at least that wide, else 128, else 64; bands of 8.
lbm_status pick_launch(lbm_ehd_server* s) {
  double wide = 0, mid = 0, all = 0;
  for (int64_t id : s->running) {
    const lbm_ehd_params& P = s->req[id].P;
    const double c = (double)P.nx * P.ny;
    all += c;
    if (P.nx >= 256) wide += c;
    if (P.nx >= 128) mid += c;
  }
  const int waves = wide >= 0.5 * all ? 4 : (mid >= 0.5 * all ? 2 : 1);
  return lbm_ehd_batch_set_launch(s->batch, waves, 8);
}

// Retire running requests with no steps left: leave the batch (which waits
// for the batch's work), read the diagnostics.
lbm_status retire(lbm_ehd_server* s, bool* changed) {
  for (size_t k = 0; k < s->running.size();) {
    Request& r = s->req[s->running[k]];
    if (r.steps_done < r.steps_total) {
      ++k;
      continue;
    }
    lbm_status st = lbm_ehd_batch_remove(s->batch, r.sim);
    if (st) return serr(st, std::string("retire: ") + lbm_ehd_last_error());
    st = lbm_ehd_diagnostics(r.sim, &r.diag);
    r.state = st == LBM_OK ? LBM_REQ_DONE : LBM_REQ_FAILED;
    if (st) r.error = lbm_ehd_last_error();
    r.t_done = s->now();
    s->running.erase(s->running.begin() + k);
    *changed = true;
  }
  return LBM_OK;
}

// Admit queued requests that fit, first fit in arrival order.
lbm_status admit(lbm_ehd_server* s, bool* changed) {
  for (auto it = s->queue.begin(); it != s->queue.end();) {
    Request& r = s->req[*it];
    if (s->used + r.footprint > s->budget) {
      ++it;
      continue;
    }
    lbm_status st = lbm_ehd_create(&r.P, nullptr, &r.sim);
    if (!st) st = lbm_ehd_init_droplet(r.sim, r.xc, r.yc, r.radius, r.noise, r.seed);
    if (!st) st = lbm_ehd_batch_add(s->batch, r.sim);
    if (st) {
      r.state = LBM_REQ_FAILED;
      r.error = lbm_ehd_last_error();
      r.t_done = s->now();
      lbm_ehd_destroy(r.sim);
      r.sim = nullptr;
      if (st == LBM_EDEVICE) return serr(st, "admit: " + r.error);
      it = s->queue.erase(it);
      continue;
    }
    s->used += r.footprint;
    r.state = LBM_REQ_RUNNING;
    r.t_start = s->now();
    s->running.push_back(r.id);
    it = s->queue.erase(it);
    *changed = true;
  }
  return LBM_OK;
}

}  // namespace

extern "C" {

lbm_status lbm_ehd_server_create(size_t hbm_budget_bytes, int32_t block_steps,
                                 lbm_ehd_server** out) {
  if (!out) return serr(LBM_EINVAL, "out is NULL");
  *out = nullptr;
  if (hbm_budget_bytes == 0) return serr(LBM_EINVAL, "budget must be > 0");
  if (block_steps < 2 || (block_steps & 1)) return serr(LBM_EINVAL, "block_steps: even, >= 2");
  lbm_ehd_server* s = new (std::nothrow) lbm_ehd_server;
  if (!s) return serr(LBM_ENOMEM, "host allocation failed");
  s->budget = hbm_budget_bytes;
  s->block_steps = block_steps;
  s->t0 = std::chrono::steady_clock::now();
  lbm_status st = lbm_ehd_batch_create(nullptr, 0, nullptr, &s->batch);
  if (!st) st = lbm_ehd_batch_set_graph_steps(s->batch, std::min<int32_t>(block_steps, 32));
  if (st) {
    const std::string msg = lbm_ehd_last_error();
    lbm_ehd_batch_destroy(s->batch);
    delete s;
    return serr(st, msg);
  }
  *out = s;
  return LBM_OK;
}

lbm_status lbm_ehd_server_submit(lbm_ehd_server* s, const lbm_ehd_params* p, double xc,
                                 double yc, double radius, double noise, uint64_t seed,
                                 int64_t nsteps, int64_t* id) {
  if (!s || !p || !id) return serr(LBM_EINVAL, "NULL argument");
  if (nsteps < 0) return serr(LBM_EINVAL, "nsteps < 0");
  if (p->poisson_iters != 0 || p->poisson_tol > 0)
    return serr(LBM_EINVAL, "served requests need poisson_iters = 0 and poisson_tol = 0");
  Request r;
  r.P = *p;
  lbm_status st = lbm_ehd_footprint_bytes(p, &r.footprint);
  if (st) return serr(st, lbm_ehd_last_error());
  if (r.footprint > s->budget) return serr(LBM_ERANGE, "request larger than the HBM budget");
  for (const auto& kv : s->req)
    if (kv.second.P.precision != p->precision)
      return serr(LBM_EINVAL, "all requests of a server share one storage precision");
  r.id = s->next_id++;
  r.xc = xc;
  r.yc = yc;
  r.radius = radius;
  r.noise = noise;
  r.seed = seed;
  r.steps_total = nsteps;
  r.t_submit = s->now();
  std::memset(&r.diag, 0, sizeof r.diag);
  s->req[r.id] = r;
  s->queue.push_back(r.id);
  *id = r.id;
  return LBM_OK;
}

lbm_status lbm_ehd_server_advance(lbm_ehd_server* s, int32_t* running, int32_t* queued) {
  if (!s) return serr(LBM_EINVAL, "server is NULL");
  bool changed = false;
  lbm_status st = retire(s, &changed);
  if (!st) st = admit(s, &changed);
  if (!st && changed && !s->running.empty()) st = pick_launch(s);
  if (!st && !s->running.empty()) {
    int64_t block = s->block_steps;
    for (int64_t id : s->running) {
      const Request& r = s->req[id];
      block = std::min(block, r.steps_total - r.steps_done);
    }
    if (block > 0) {
      st = lbm_ehd_batch_run(s->batch, block);
      if (st)
        st = serr(st, std::string("run: ") + lbm_ehd_last_error());
      else
        for (int64_t id : s->running) s->req[id].steps_done += block;
    }
  }
  if (running) *running = (int32_t)s->running.size();
  if (queued) *queued = (int32_t)s->queue.size();
  return st;
}

lbm_status lbm_ehd_server_info(lbm_ehd_server* s, int64_t id, lbm_ehd_request_info* out) {
  if (!s || !out) return serr(LBM_EINVAL, "NULL argument");
  auto it = s->req.find(id);
  if (it == s->req.end()) return serr(LBM_EINVAL, "unknown request id");
  const Request& r = it->second;
  std::memset(out, 0, sizeof *out);
  out->id = r.id;
  out->state = r.state;
  out->steps_done = r.steps_done;
  out->steps_total = r.steps_total;
  out->t_submit = r.t_submit;
  out->t_start = r.t_start;
  out->t_done = r.t_done;
  out->footprint = r.footprint;
  out->diag = r.diag;
  return LBM_OK;
}

lbm_status lbm_ehd_server_fields(lbm_ehd_server* s, int64_t id, uint32_t mask, double* out,
                                 size_t n_doubles) {
  if (!s) return serr(LBM_EINVAL, "server is NULL");
  auto it = s->req.find(id);
  if (it == s->req.end()) return serr(LBM_EINVAL, "unknown request id");
  const Request& r = it->second;
  if (r.state != LBM_REQ_DONE || !r.sim) return serr(LBM_ESTATE, "request not finished");
  lbm_status st = lbm_ehd_get_fields(r.sim, mask, out, n_doubles);
  if (st) return serr(st, lbm_ehd_last_error());
  return LBM_OK;
}

lbm_status lbm_ehd_server_release(lbm_ehd_server* s, int64_t id) {
  if (!s) return serr(LBM_EINVAL, "server is NULL");
  auto it = s->req.find(id);
  if (it == s->req.end()) return serr(LBM_EINVAL, "unknown request id");
  Request& r = it->second;
  if (r.state == LBM_REQ_QUEUED || r.state == LBM_REQ_RUNNING)
    return serr(LBM_ESTATE, "request still queued or running");
  if (r.sim) {
    lbm_ehd_destroy(r.sim);
    r.sim = nullptr;
    s->used -= r.footprint;
  }
  s->req.erase(it);
  return LBM_OK;
}

size_t lbm_ehd_server_used_bytes(const lbm_ehd_server* s) { return s ? s->used : 0; }

const char* lbm_ehd_server_last_error(void) { return g_serr.c_str(); }

lbm_status lbm_ehd_server_destroy(lbm_ehd_server* s) {
  if (!s) return LBM_OK;
  lbm_ehd_batch_synchronize(s->batch);
  lbm_ehd_batch_destroy(s->batch);
  for (auto& kv : s->req)
    if (kv.second.sim) lbm_ehd_destroy(kv.second.sim);
  delete s;
  return LBM_OK;
}

}  // extern "C"
