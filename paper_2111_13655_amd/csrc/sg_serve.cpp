// Continuous-batching server of Chebyshev propagation requests.
//
// Threads: compile workers turn submitted descriptions into host term sets
// (compile_problem); one scheduler thread owns the device.  Each scheduler
// tick admits compiled requests while the device-memory budget and the slots
// allow (FIFO by ticket), rebuilds the launch plan when the resident set
// changed, and advances every resident request by one Chebyshev step with one
// term-sweep launch and one reduce launch per series term for all of them.
// A request whose step count is reached (or whose norm drifts beyond the
// tolerance, or that was cancelled) is copied to host and evicted.
#include <algorithm>
#include <chrono>
#include <climits>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <thread>
#include <unordered_map>
#include <vector>

#include "sg_internal.h"

namespace {

enum class JobState { Queued, Compiled, Resident, Done };

struct Job {
  uint64_t ticket = 0;
  int D = 0, L = 0, nbA = 1, nbB = 2, nqA = 2, nqB = 2;
  std::vector<double> omega, c, k, shift;
  double dt = 0.0;
  int nsteps = 0;
  JobState state = JobState::Queued;
  sg_problem *prob = nullptr;       // compiled, then uploaded
  double2 *d_psi = nullptr;
  int64_t bytes = 0;                // device bytes held while resident
  double t_submit = 0, t_admit = 0, t_done = 0;
  int steps_done = 0;
  int checks = 0;
  int status = SG_OK;
  bool cancel = false;
  sg_prop_stats stats{};
  std::vector<double2> result;
};

}  // namespace

struct sg_server {
  sg_serve_config cfg{};
  int device = 0;
  hipStream_t stream = nullptr;
  std::chrono::steady_clock::time_point t0;
  std::mutex mu;
  std::condition_variable cv_sched, cv_compile;
  std::deque<Job *> queued;                 // waiting for a compile worker
  std::map<uint64_t, Job *> compiled;       // compiled, waiting for admission
  std::vector<Job *> resident;
  std::unordered_map<uint64_t, Job *> jobs; // every live ticket
  uint64_t next_ticket = 1;
  int64_t budget = 0, used = 0;
  int64_t finished = 0, ticks = 0;
  bool stop = false;
  std::vector<std::thread> workers;
  std::thread scheduler;
  sg::Plan plan;
  double *d_results = nullptr, *h_results = nullptr;
  int results_cap = 0;

  double now() const {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }
};

namespace sg {
namespace {

// A lower bound of the device bytes a request holds (its vectors and index
// maps), known before compiling: a request above the budget can never fit.
int64_t request_bytes_lower_bound(int D, int L, int nbA, int nbB) {
  int64_t sz[3];
  if (count_sizes(D, L, nbA, nbB, sz) != SG_OK) return INT64_MAX;
  const int64_t ns = sz[1], ncs = sz[2];
  return ns * (int64_t)(sizeof(int32_t) + sizeof(double2)) +
         ncs * (int64_t)(5 * sizeof(double2));
}

void compile_worker(sg_server *s) {
  for (;;) {
    Job *j = nullptr;
    {
      std::unique_lock<std::mutex> lk(s->mu);
      s->cv_compile.wait(lk, [&] { return s->stop || !s->queued.empty(); });
      if (s->stop) return;
      j = s->queued.front();
      s->queued.pop_front();
    }
    sg_problem *p = new (std::nothrow) sg_problem();
    sg_status st = p ? SG_OK : SG_ENOMEM;
    std::string err;
    if (p) {
      sg_problem_desc d{j->D, j->L, j->nbA, j->nbB, j->nqA, j->nqB,
                        j->omega.data(), j->c.data(), j->k.data()};
      try {
        st = compile_problem(&d, &p->h, &err);
      } catch (const std::bad_alloc &) {
        st = SG_ENOMEM;
      }
      if (st == SG_OK && s->cfg.prec == SG_MIXED && s->cfg.mixed_threshold >= 0)
        p->h.mixed_max_fp32_coeff = s->cfg.mixed_threshold;
    }
    std::lock_guard<std::mutex> lk(s->mu);
    if (st != SG_OK || j->cancel) {
      delete p;
      j->status = j->cancel ? SG_ECANCELED : st;
      j->state = JobState::Done;
      j->t_done = s->now();
      s->finished++;
    } else if (estimate_device_bytes(p->h) > s->budget) {
      delete p;
      j->status = SG_ENOMEM;
      j->state = JobState::Done;
      j->t_done = s->now();
      s->finished++;
    } else {
      j->prob = p;
      j->bytes = estimate_device_bytes(p->h);
      j->state = JobState::Compiled;
      s->compiled[j->ticket] = j;
    }
    s->cv_sched.notify_all();
  }
}

// Device side of admission: upload, initial state, spectral bounds, series.
sg_status admit(sg_server *s, Job *j) {
  sg_problem *up = nullptr;
  sg_status st = upload_problem(j->prob, &up);
  j->prob = up;  // upload_problem frees on failure
  if (st != SG_OK) return st;
  const int64_t n = up->h.ncs;
  hipError_t e = hipMalloc((void **)&j->d_psi, n * sizeof(double2));
  if (e != hipSuccess) return fail(SG_ENOMEM, "device allocation of a request state failed");
  j->bytes = up->device_bytes + n * (int64_t)sizeof(double2);
  if ((st = sg_init_gaussian(up, j->shift.data(), j->d_psi, nullptr, s->stream)) != SG_OK) return st;
  double lo, hi;
  if ((st = sg_spectral_bounds(up, 40, &lo, &hi, s->stream)) != SG_OK) return st;
  const double half = 0.5 * (hi - lo), ebar = 0.5 * (hi + lo);
  std::vector<double> a;
  const int K = chebyshev_series(half * j->dt, &a);
  if (K < 2 || K > kMaxChebTerms) return fail(SG_EINVAL, "Chebyshev series length out of range");
  e = hipMemcpyAsync(up->d_cheb_a, a.data(), K * sizeof(double), hipMemcpyHostToDevice, s->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
  if (e != hipSuccess) return hip_fail(e, "upload series");
  j->stats.cheb_terms = K;
  j->stats.emin = lo;
  j->stats.emax = hi;
  return SG_OK;
}

void finish(sg_server *s, Job *j, int status) {
  if (j->d_psi && j->prob && status != SG_ECANCELED) {
    j->result.resize(j->prob->h.ncs);
    hipMemcpyAsync(j->result.data(), j->d_psi, j->result.size() * sizeof(double2),
                   hipMemcpyDeviceToHost, s->stream);
    hipStreamSynchronize(s->stream);
  }
  hipFree(j->d_psi);
  j->d_psi = nullptr;
  if (j->prob) release_problem(j->prob);
  j->prob = nullptr;
  std::lock_guard<std::mutex> lk(s->mu);
  s->used -= j->bytes;
  j->status = status;
  j->state = JobState::Done;
  j->t_done = s->now();
  s->finished++;
}

sg_status rebuild_plan(sg_server *s) {
  std::vector<sg_problem *> probs;
  for (Job *j : s->resident) probs.push_back(j->prob);
  std::string err;
  sg_status st = plan_build(&s->plan, probs, &err);
  if (st != SG_OK) return fail(st, err);
  if ((int)probs.size() > s->results_cap) {
    hipFree(s->d_results);
    if (s->h_results) hipHostFree(s->h_results);
    s->results_cap = std::max<int>((int)probs.size(), 2 * s->results_cap);
    if (hipMalloc((void **)&s->d_results, 2 * s->results_cap * sizeof(double)) != hipSuccess ||
        hipHostMalloc((void **)&s->h_results, 2 * s->results_cap * sizeof(double),
                      hipHostMallocDefault) != hipSuccess)
      return fail(SG_ENOMEM, "server result buffers");
  }
  for (size_t i = 0; i < s->resident.size(); ++i) {
    Job *j = s->resident[i];
    InstDev &I = s->plan.inst[i];
    const double lo = j->stats.emin, hi = j->stats.emax;
    const double half = 0.5 * (hi - lo), ebar = 0.5 * (hi + lo);
    I.x0 = j->d_psi;
    I.result = s->d_results + 2 * i;
    I.K = j->stats.cheb_terms;
    I.ebar = ebar;
    I.inv_half = 1.0 / half;
    I.phase_re = std::cos(-ebar * j->dt);
    I.phase_im = std::sin(-ebar * j->dt);
    I.active = 1;
  }
  return plan_upload(&s->plan, s->stream);
}

void scheduler_loop(sg_server *s) {
  hipSetDevice(s->device);
  bool dirty = true;
  for (;;) {
    std::vector<Job *> to_admit;
    {
      std::unique_lock<std::mutex> lk(s->mu);
      s->cv_sched.wait(lk, [&] {
        return s->stop || !s->resident.empty() || !s->compiled.empty();
      });
      if (s->stop) break;
      for (auto it = s->compiled.begin(); it != s->compiled.end();) {
        Job *j = it->second;
        if (!j->cancel) {
          ++it;
          continue;
        }
        delete j->prob;
        j->prob = nullptr;
        j->status = SG_ECANCELED;
        j->state = JobState::Done;
        j->t_done = s->now();
        s->finished++;
        it = s->compiled.erase(it);
      }
      // admission, FIFO by ticket; a request alone always fits (the compile
      // workers reject requests above the budget)
      while (!s->compiled.empty() &&
             (int)(s->resident.size() + to_admit.size()) < s->cfg.max_slots) {
        Job *j = s->compiled.begin()->second;
        if (s->used + j->bytes > s->budget && !(s->resident.empty() && to_admit.empty())) break;
        s->compiled.erase(s->compiled.begin());
        s->used += j->bytes;
        to_admit.push_back(j);
      }
    }
    for (Job *j : to_admit) {
      const int64_t est = j->bytes;
      sg_status st = admit(s, j);
      {
        std::lock_guard<std::mutex> lk(s->mu);
        s->used += j->bytes - est;
      }
      if (st != SG_OK) {
        finish(s, j, st);
        continue;
      }
      j->t_admit = s->now();
      j->state = JobState::Resident;
      std::lock_guard<std::mutex> lk(s->mu);
      s->resident.push_back(j);
      dirty = true;
    }
    // evict cancelled residents
    {
      std::vector<Job *> gone;
      {
        std::lock_guard<std::mutex> lk(s->mu);
        for (auto it = s->resident.begin(); it != s->resident.end();) {
          if ((*it)->cancel) {
            gone.push_back(*it);
            it = s->resident.erase(it);
          } else {
            ++it;
          }
        }
      }
      for (Job *j : gone) finish(s, j, SG_ECANCELED);
      if (!gone.empty()) dirty = true;
    }
    if (s->resident.empty()) continue;
    if (dirty) {
      if (rebuild_plan(s) != SG_OK) {
        std::vector<Job *> all;
        {
          std::lock_guard<std::mutex> lk(s->mu);
          all.swap(s->resident);
        }
        for (Job *j : all) finish(s, j, SG_EDEVICE);
        continue;
      }
      dirty = false;
    }
    // one Chebyshev step for every resident request
    bool check = false;
    int kmax = 0;
    for (Job *j : s->resident) {
      kmax = std::max(kmax, j->stats.cheb_terms);
      if (j->steps_done == 0 || (s->cfg.check_every > 0 && j->steps_done % s->cfg.check_every == 0))
        check = true;
    }
    LaunchCtl c;
    c.mode = Mode::Cheb;
    // with no FP32 term resident, the mixed path is the FP64 split path term
    // by term: launch that pack set (laid out for FP64 tables only)
    c.prec = (s->cfg.prec == SG_MIXED && !s->plan.any32 && s->plan.fp64_split) ? SG_FP64
                                                                                 : s->cfg.prec;
    hipError_t e = hipSuccess;
    for (int k = 1; k < kmax && e == hipSuccess; ++k) {
      c.k = k;
      c.want_partials = (k == 1 && check) ? 1 : 0;
      e = launch_sweep(&s->plan, c, s->stream);
      if (e == hipSuccess) e = launch_reduce(&s->plan, c, s->stream);
      if (e == hipSuccess && k == 1 && check) e = launch_finalize(&s->plan, s->stream);
    }
    if (e == hipSuccess && check)
      e = hipMemcpyAsync(s->h_results, s->d_results, 2 * s->resident.size() * sizeof(double),
                         hipMemcpyDeviceToHost, s->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    s->ticks++;
    std::vector<Job *> done;
    std::vector<int> done_status;
    for (size_t i = 0; i < s->resident.size(); ++i) {
      Job *j = s->resident[i];
      if (e != hipSuccess) {
        done.push_back(j);
        done_status.push_back(SG_EDEVICE);
        continue;
      }
      if (check) {
        const double nrm2 = s->h_results[2 * i], ene = s->h_results[2 * i + 1];
        const double nrm = std::sqrt(nrm2), E = ene / nrm2;
        sg_prop_stats &st = j->stats;
        if (j->checks == 0) {
          st.norm0 = nrm;
          st.energy0 = E;
        }
        st.norm_last = nrm;
        st.energy_last = E;
        st.max_norm_drift = std::max(st.max_norm_drift, std::fabs(nrm - st.norm0));
        st.max_energy_drift = std::max(st.max_energy_drift, std::fabs(E - st.energy0));
        j->checks++;
      }
      j->steps_done++;
      j->stats.steps_done = j->steps_done;
      j->stats.applies += j->stats.cheb_terms - 1;
      const bool drift = s->cfg.tol > 0.0 && j->stats.max_norm_drift > s->cfg.tol;
      if (drift || j->steps_done >= j->nsteps) {
        done.push_back(j);
        done_status.push_back(drift ? SG_ETOL : SG_OK);
      }
    }
    if (!done.empty()) {
      {
        std::lock_guard<std::mutex> lk(s->mu);
        for (Job *j : done) s->resident.erase(std::find(s->resident.begin(), s->resident.end(), j));
      }
      for (size_t q = 0; q < done.size(); ++q) finish(s, done[q], done_status[q]);
      dirty = true;
    }
  }
}

}  // namespace
}  // namespace sg

using namespace sg;

extern "C" {

sg_status sg_serve_create(const sg_serve_config *cfg, sg_server **out) {
  if (!cfg || !out) return fail(SG_EINVAL, "NULL argument");
  if (cfg->max_slots < 1) return fail(SG_EINVAL, "max_slots must be >= 1");
  if (cfg->prec != SG_FP64 && cfg->prec != SG_MIXED) return fail(SG_EINVAL, "unknown precision");
  *out = nullptr;
  sg_server *s = new (std::nothrow) sg_server();
  if (!s) return fail(SG_ENOMEM, "host allocation failed");
  s->cfg = *cfg;
  s->t0 = std::chrono::steady_clock::now();
  hipGetDevice(&s->device);
  if (hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking) != hipSuccess) {
    delete s;
    return fail(SG_EDEVICE, "stream creation failed");
  }
  s->budget = cfg->hbm_budget_bytes;
  if (s->budget <= 0) {
    size_t fr = 0, tot = 0;
    hipMemGetInfo(&fr, &tot);
    s->budget = (int64_t)(0.8 * (double)fr);
  }
  const int nw = cfg->compile_threads > 0 ? cfg->compile_threads : 4;
  for (int i = 0; i < nw; ++i) s->workers.emplace_back(compile_worker, s);
  s->scheduler = std::thread(scheduler_loop, s);
  *out = s;
  return SG_OK;
}

sg_status sg_serve_submit(sg_server *s, const sg_problem_desc *desc, const double *shift,
                          double dt, int32_t nsteps, uint64_t *ticket) {
  if (!s || !desc || !shift || !ticket) return fail(SG_EINVAL, "NULL argument");
  if (!(dt > 0.0) || !std::isfinite(dt) || nsteps < 1) return fail(SG_EINVAL, "dt > 0, nsteps >= 1");
  if (desc->D < 1 || desc->D > 64 || !desc->omega || !desc->c) return fail(SG_EINVAL, "invalid description");
  const int64_t need = request_bytes_lower_bound(desc->D, desc->L, desc->nb_A, desc->nb_B);
  if (need > s->budget) return fail(SG_ENOMEM, "request can never fit the device-memory budget");
  Job *j = new (std::nothrow) Job();
  if (!j) return fail(SG_ENOMEM, "host allocation failed");
  const int D = desc->D;
  j->D = D;
  j->L = desc->L;
  j->nbA = desc->nb_A;
  j->nbB = desc->nb_B;
  j->nqA = desc->nq_A;
  j->nqB = desc->nq_B;
  j->omega.assign(desc->omega, desc->omega + D);
  j->c.assign(desc->c, desc->c + (size_t)D * D);
  j->k.assign((size_t)D * D, 0.0);
  if (desc->k) j->k.assign(desc->k, desc->k + (size_t)D * D);
  j->shift.assign(shift, shift + D);
  j->dt = dt;
  j->nsteps = nsteps;
  std::lock_guard<std::mutex> lk(s->mu);
  j->ticket = s->next_ticket++;
  j->t_submit = s->now();
  s->jobs[j->ticket] = j;
  s->queued.push_back(j);
  *ticket = j->ticket;
  s->cv_compile.notify_one();
  return SG_OK;
}

sg_status sg_serve_poll(sg_server *s, uint64_t ticket, sg_result *out) {
  if (!s || !out) return fail(SG_EINVAL, "NULL argument");
  Job *j = nullptr;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->jobs.find(ticket);
    if (it == s->jobs.end()) return fail(SG_ENOTFOUND, "unknown ticket");
    if (it->second->state != JobState::Done) return SG_EAGAIN;
    j = it->second;
    s->jobs.erase(it);
  }
  out->status = j->status;
  out->D = j->D;
  out->L = j->L;
  out->n_cs = (int64_t)j->result.size();
  if (out->psi_host && out->psi_capacity >= out->n_cs && !j->result.empty())
    std::memcpy(out->psi_host, j->result.data(), j->result.size() * sizeof(double2));
  out->stats = j->stats;
  out->t_submit = j->t_submit;
  out->t_admit = j->t_admit;
  out->t_done = j->t_done;
  delete j;
  return SG_OK;
}

sg_status sg_serve_cancel(sg_server *s, uint64_t ticket) {
  if (!s) return fail(SG_EINVAL, "NULL argument");
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->jobs.find(ticket);
  if (it == s->jobs.end()) return fail(SG_ENOTFOUND, "unknown ticket");
  Job *j = it->second;
  if (j->state == JobState::Done) return SG_OK;
  j->cancel = true;
  auto q = std::find(s->queued.begin(), s->queued.end(), j);
  if (q != s->queued.end()) {
    s->queued.erase(q);
    j->status = SG_ECANCELED;
    j->state = JobState::Done;
    j->t_done = s->now();
    s->finished++;
  }
  s->cv_sched.notify_all();
  return SG_OK;
}

sg_status sg_serve_counters(sg_server *s, int64_t out[4]) {
  if (!s || !out) return fail(SG_EINVAL, "NULL argument");
  std::lock_guard<std::mutex> lk(s->mu);
  out[0] = (int64_t)(s->queued.size() + s->compiled.size());
  out[1] = (int64_t)s->resident.size();
  out[2] = s->finished;
  out[3] = s->ticks;
  return SG_OK;
}

sg_status sg_serve_destroy(sg_server *s) {
  if (!s) return SG_OK;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
  }
  s->cv_compile.notify_all();
  s->cv_sched.notify_all();
  for (auto &t : s->workers) t.join();
  if (s->scheduler.joinable()) s->scheduler.join();
  hipSetDevice(s->device);
  for (Job *j : s->resident) {
    hipFree(j->d_psi);
    if (j->prob) release_problem(j->prob);
  }
  for (auto &kv : s->compiled) delete kv.second->prob;
  for (auto &kv : s->jobs) delete kv.second;
  plan_free(&s->plan);
  hipFree(s->d_results);
  if (s->h_results) hipHostFree(s->h_results);
  hipStreamDestroy(s->stream);
  delete s;
  return SG_OK;
}

}  // extern "C"
