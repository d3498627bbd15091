// Continuous-batching request loop over independent solves (lindblad_serve.h).
//
// n_slots host threads share one queue of requests ordered by arrival time
// (ties: larger footprint first).
// A thread takes the head of the queue once it has arrived and its device
// footprint fits in the budget left by the running solves, then drives that
// solve on the solver's own HIP stream: upload of the initial state, the
// steps, the observables, release of its device memory.  Completion frees
// budget and wakes the threads waiting for it.  Only the public C ABI of the
// solver is used here.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "../../include/lindblad.h"
#include "../../include/lindblad_serve.h"

namespace {

using Clock = std::chrono::steady_clock;

struct Request {
  lb_solver* solver = nullptr;
  std::vector<std::vector<double>> init;   // per mode, interleaved complex
  int n_steps = 0;
  std::vector<const lb_op*> obs;
  double arrival = 0.0;
  int64_t bytes = 0;
  bool finished = false;
  lb_result res{};
  std::vector<double> obs_out;
};

}  // namespace

struct lb_server {
  lb_server_config cfg{};
  std::vector<Request> reqs;
  std::vector<int> queue;        // indices of requests of the current run, by arrival
  size_t head = 0;
  int64_t used = 0;
  int running = 0;
  bool in_run = false;
  bool have_run = false;
  Clock::time_point t0;
  lb_server_stats stats{};
  std::mutex mu;
  std::condition_variable cv;
};

namespace {

double since(const lb_server* sv) {
  return std::chrono::duration<double>(Clock::now() - sv->t0).count();
}

void run_one(Request& r) {
  lb_result& out = r.res;
  std::vector<const double*> ptrs(r.init.size());
  for (size_t m = 0; m < r.init.size(); ++m) ptrs[m] = r.init[m].data();
  lb_status st = lindblad_set_state_product(r.solver, ptrs.data());
  if (st == LB_OK) st = lindblad_step(r.solver, r.n_steps);
  r.obs_out.assign(2 * r.obs.size(), 0.0);
  for (size_t o = 0; o < r.obs.size() && st == LB_OK; ++o) st = lindblad_observe(r.solver, r.obs[o], &r.obs_out[2 * o]);
  if (st == LB_OK) {
    lb_diag d;
    st = lindblad_diagnostics(r.solver, &d);
    if (st == LB_OK) {
      out.max_tau_defect = d.max_tau_defect;
      out.chi_mu = d.chi_mu;
      int mb = 1;
      for (int i = 0; i + 1 < d.n_sites; ++i) mb = std::max(mb, (int)d.bonds[i]);
      out.max_bond = mb;
    }
  }
  const lb_status rel = lindblad_release(r.solver);
  out.status = (st != LB_OK) ? st : rel;
}

void worker(lb_server* sv) {
  std::unique_lock<std::mutex> lk(sv->mu);
  for (;;) {
    if (sv->head >= sv->queue.size()) return;
    Request& r = sv->reqs[sv->queue[sv->head]];
    const auto due = sv->t0 + std::chrono::duration_cast<Clock::duration>(std::chrono::duration<double>(r.arrival));
    if (Clock::now() < due) {
      sv->cv.wait_until(lk, due);
      continue;
    }
    const int64_t budget = sv->cfg.hbm_budget;
    if (budget > 0 && sv->running > 0 && sv->used + r.bytes > budget) {
      sv->cv.wait(lk);
      continue;
    }
    sv->head++;
    sv->used += r.bytes;
    sv->running++;
    sv->stats.peak_bytes = std::max(sv->stats.peak_bytes, sv->used);
    sv->stats.peak_running = std::max(sv->stats.peak_running, sv->running);
    r.res.admitted = since(sv);
    sv->cv.notify_all();
    lk.unlock();
    run_one(r);
    lk.lock();
    r.res.done = since(sv);
    r.finished = true;
    sv->used -= r.bytes;
    sv->running--;
    sv->stats.completed++;
    sv->stats.makespan = std::max(sv->stats.makespan, r.res.done);
    sv->cv.notify_all();
  }
}

}  // namespace

extern "C" {

lb_status lindblad_server_create(const lb_server_config* cfg, lb_server** out) {
  if (!cfg || !out) return LB_ERR_ARG;
  *out = nullptr;
  if (cfg->n_slots < 1 || cfg->n_slots > 256) return LB_ERR_ARG;
  lb_server* sv = new (std::nothrow) lb_server;
  if (!sv) return LB_ERR_OOM;
  sv->cfg = *cfg;
  *out = sv;
  return LB_OK;
}

lb_status lindblad_server_submit(lb_server* sv, const lb_request* req, int32_t* ticket) {
  if (!sv || !req || !req->solver || !req->init || req->n_steps < 0 || req->n_obs < 0 || req->n_obs > 64)
    return LB_ERR_ARG;
  if (req->n_obs > 0 && !req->obs) return LB_ERR_ARG;
  std::lock_guard<std::mutex> g(sv->mu);
  if (sv->in_run) return LB_ERR_STATE;
  lb_config cfg;
  if (lindblad_get_config(req->solver, &cfg) != LB_OK) return LB_ERR_ARG;
  Request r;
  r.solver = req->solver;
  for (int m = 0; m < cfg.n_modes; ++m) {
    if (!req->init[m]) return LB_ERR_ARG;
    const size_t n = (size_t)2 << cfg.bits[m];
    r.init.emplace_back(req->init[m], req->init[m] + n);
  }
  for (int o = 0; o < req->n_obs; ++o) {
    if (!req->obs[o]) return LB_ERR_ARG;
    r.obs.push_back(req->obs[o]);
  }
  r.n_steps = req->n_steps;
  r.arrival = std::max(0.0, req->arrival);
  const lb_status st = lindblad_footprint(req->solver, &r.bytes);
  if (st != LB_OK) return st;
  r.res.arrival = r.arrival;
  r.res.bytes = r.bytes;
  r.res.admitted = r.res.done = -1.0;
  sv->reqs.push_back(std::move(r));
  if (ticket) *ticket = (int32_t)sv->reqs.size() - 1;
  return LB_OK;
}

lb_status lindblad_server_run(lb_server* sv) {
  if (!sv) return LB_ERR_ARG;
  {
    std::lock_guard<std::mutex> g(sv->mu);
    if (sv->in_run) return LB_ERR_STATE;
    sv->queue.clear();
    for (int i = 0; i < (int)sv->reqs.size(); ++i)
      if (!sv->reqs[i].finished) sv->queue.push_back(i);
    // arrival order; among requests that arrive together the larger footprint
    // (a proxy for the longer solve) goes first, so a burst does not end on a
    // long solve admitted last
    std::stable_sort(sv->queue.begin(), sv->queue.end(), [&](int a, int b) {
      const Request& x = sv->reqs[a];
      const Request& y = sv->reqs[b];
      if (x.arrival != y.arrival) return x.arrival < y.arrival;
      return x.bytes > y.bytes;
    });
    sv->head = 0;
    sv->used = 0;
    sv->running = 0;
    sv->stats = lb_server_stats{};
    sv->in_run = true;
    sv->t0 = Clock::now();
  }
  const int n = std::min<int>(sv->cfg.n_slots, std::max<int>(1, (int)sv->queue.size()));
  std::vector<std::thread> th;
  th.reserve(n);
  for (int k = 0; k < n; ++k) th.emplace_back(worker, sv);
  for (auto& t : th) t.join();
  std::lock_guard<std::mutex> g(sv->mu);
  sv->in_run = false;
  sv->have_run = true;
  return LB_OK;
}

lb_status lindblad_server_result(const lb_server* sv, int32_t ticket, lb_result* res, double* obs_out) {
  if (!sv || !res || ticket < 0 || ticket >= (int32_t)sv->reqs.size()) return LB_ERR_ARG;
  const Request& r = sv->reqs[ticket];
  if (!r.finished) return LB_ERR_STATE;
  *res = r.res;
  if (obs_out) std::memcpy(obs_out, r.obs_out.data(), r.obs_out.size() * sizeof(double));
  return LB_OK;
}

lb_status lindblad_server_stats(const lb_server* sv, lb_server_stats* out) {
  if (!sv || !out) return LB_ERR_ARG;
  lb_server* m = const_cast<lb_server*>(sv);   // the lock only
  std::lock_guard<std::mutex> g(m->mu);
  *out = sv->stats;
  return LB_OK;
}

void lindblad_server_destroy(lb_server* sv) { delete sv; }

}  // extern "C"
