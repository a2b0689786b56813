// Batched Chebyshev propagation: many problem instances advance together,
// one term-sweep launch and one reduce launch per Chebyshev term for all of
// them (see sg_plan.cpp for the term -> workgroup schedule).  The step's
// launches can be captured once into a hipGraph and replayed.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "sg_internal.h"

struct sg_batch {
  sg::Plan plan;
  std::vector<sg_problem *> probs;
  double *d_results = nullptr;     // [2 * n]
  double *h_results = nullptr;     // pinned mirror
  hipStream_t own = nullptr;       // stream of graph replays
  int device = 0;
};

namespace sg {
namespace {

// The precision a batch launch runs in: with no FP32 term in the plan, the
// mixed path is the FP64 split path term by term (same tables, same
// contractions, same fixed-order reduce), so it launches that pack set, which
// the cached multi-problem packs lay out for FP64 tables only.
sg_precision launch_precision(const Plan &pl, sg_precision prec) {
  return (prec == SG_MIXED && !pl.any32 && pl.fp64_split) ? SG_FP64 : prec;
}

// The batch's instance records still name every problem's current potential
// tables (a potential set, changed or cleared after the batch was created
// would leave them naming other, possibly freed, tables).
bool potentials_current(const sg_batch *b) {
  for (size_t i = 0; i < b->probs.size(); ++i)
    if (b->plan.inst[i].veff != b->probs[i]->d_veff || b->plan.inst[i].voff != b->probs[i]->d_voff)
      return false;
  return true;
}

// A tabulated potential runs in FP64: a mixed batch holding one runs only
// when no term of the batch is in FP32 (then it is the FP64 split path).
bool precision_ok(const Plan &pl, sg_precision prec) {
  return !(pl.any_tab && launch_precision(pl, prec) == SG_MIXED);
}

sg_status batch_step_launches(sg_batch *b, sg_precision prec, int kmax, hipStream_t s) {
  LaunchCtl c;
  c.mode = Mode::Cheb;
  c.prec = launch_precision(b->plan, prec);
  for (int k = 1; k < kmax; ++k) {
    c.k = k;
    c.want_partials = 0;
    hipError_t e = launch_sweep(&b->plan, c, s);
    if (e == hipSuccess) e = launch_reduce(&b->plan, c, s);
    if (e != hipSuccess) return hip_fail(e, "batched step");
  }
  return SG_OK;
}

}  // namespace
}  // namespace sg

using namespace sg;

extern "C" {

sg_status sg_batch_create(sg_problem *const *problems, int32_t n, sg_batch **out) {
  if (!out || !problems || n < 1) return fail(SG_EINVAL, "need at least one problem");
  *out = nullptr;
  int dev = 0;
  hipGetDevice(&dev);
  for (int i = 0; i < n; ++i) {
    if (!problems[i] || problems[i]->host_only) return fail(SG_EINVAL, "invalid problem handle");
    if (problems[i]->device != dev) return fail(SG_EINVAL, "problems must be on the current device");
    for (int j = 0; j < i; ++j)
      if (problems[j] == problems[i]) return fail(SG_EINVAL, "a problem appears twice");
  }
  sg_batch *b = new (std::nothrow) sg_batch();
  if (!b) return fail(SG_ENOMEM, "host allocation failed");
  b->device = dev;
  b->probs.assign(problems, problems + n);
  std::string err;
  sg_status st = plan_build(&b->plan, b->probs, &err);
  if (st != SG_OK) {
    delete b;
    return fail(st, err);
  }
  hipError_t e = hipMalloc((void **)&b->d_results, 2 * (size_t)n * sizeof(double));
  if (e == hipSuccess) e = hipHostMalloc((void **)&b->h_results, 2 * (size_t)n * sizeof(double),
                                         hipHostMallocDefault);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&b->own, hipStreamNonBlocking);
  if (e != hipSuccess) {
    sg_batch_free(b);
    return fail(SG_ENOMEM, "batch allocation failed");
  }
  for (int i = 0; i < n; ++i) b->plan.inst[i].result = b->d_results + 2 * i;
  st = plan_upload(&b->plan, nullptr);
  if (st != SG_OK) {
    sg_batch_free(b);
    return st;
  }
  *out = b;
  return SG_OK;
}

sg_status sg_batch_tune_schedule(sg_batch *b, void *const *psi, int32_t n_psi, int32_t prec,
                                 int32_t reps, int32_t *chosen_block_min_grid, double *best_ms,
                                 void *stream) {
  if (!b || !psi) return fail(SG_EINVAL, "NULL argument");
  if (n_psi != (int32_t)b->probs.size())
    return fail(SG_EINVAL, "the number of states must equal the batch's number of instances");
  if (reps < 1) return fail(SG_EINVAL, "reps must be >= 1");
  if (prec != SG_FP64 && prec != SG_MIXED) return fail(SG_EINVAL, "unknown precision");
  if (!precision_ok(b->plan, (sg_precision)prec))
    return fail(SG_EINVAL, "a tabulated potential runs in FP64 (the batch has FP32 terms)");
  if (!potentials_current(b))
    return fail(SG_EINVAL, "a problem's potential changed after the batch was created");
  for (int i = 0; i < n_psi; ++i)
    if (!psi[i]) return fail(SG_EINVAL, "NULL state");
  hipStream_t s = (hipStream_t)stream;
  const int n = (int)b->probs.size();
  int64_t max_grid = 0, total = 0;
  for (sg_problem *p : b->probs) {
    max_grid = std::max<int64_t>(max_grid, p->h.max_grid);
    total += p->h.ncs;
  }
  // candidates: terms of at least g grid points run on a whole workgroup
  std::vector<int32_t> cand = {0};
  for (int32_t g = 256; g <= max_grid; g *= 2) cand.push_back(g);
  const std::vector<int32_t> saved = [&] {
    std::vector<int32_t> v;
    for (sg_problem *p : b->probs) v.push_back(p->block_grid);
    return v;
  }();
  // one batched apply: every instance's state in x0, its own work buffer out
  auto rebuild = [&](int32_t g) -> sg_status {
    hipError_t e = hipDeviceSynchronize();
    if (e != hipSuccess) return hip_fail(e, "synchronise before the plan upload");
    for (sg_problem *p : b->probs) p->block_grid = g;
    std::string err;
    sg_status st = plan_build(&b->plan, b->probs, &err);
    if (st != SG_OK) return fail(st, err);
    for (int i = 0; i < n; ++i) {
      b->plan.inst[i].result = b->d_results + 2 * i;
      b->plan.inst[i].x0 = (double2 *)psi[i];
    }
    return plan_upload(&b->plan, s);
  };
  LaunchCtl c;
  c.mode = Mode::Apply;
  c.prec = launch_precision(b->plan, (sg_precision)prec);
  auto apply_all = [&]() -> hipError_t {
    hipError_t e = launch_sweep(&b->plan, c, s);
    if (e == hipSuccess) e = launch_reduce(&b->plan, c, s);
    return e;
  };
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
    return fail(SG_EDEVICE, "hipEventCreate");
  std::vector<double2> h_ref((size_t)total), h_out((size_t)total);
  sg_status st = SG_OK;
  int32_t best = cand[0];
  double best_t = 1e300;
  for (size_t ci = 0; ci < cand.size() && st == SG_OK; ++ci) {
    if ((st = rebuild(cand[ci])) != SG_OK) break;
    if (apply_all() != hipSuccess) {
      st = fail(SG_EDEVICE, "batched apply");
      break;
    }
    // every schedule computes each term with the same arithmetic: the
    // outputs must agree bitwise
    double2 *dst = ci == 0 ? h_ref.data() : h_out.data();
    size_t at = 0;
    for (int i = 0; i < n && st == SG_OK; ++i) {
      const int64_t m = b->probs[i]->h.ncs;
      if (hipMemcpyAsync(dst + at, b->plan.inst[i].x1, (size_t)m * sizeof(double2),
                         hipMemcpyDeviceToHost, s) != hipSuccess)
        st = fail(SG_EDEVICE, "copy of the tuning result");
      at += (size_t)m;
    }
    if (st != SG_OK || hipStreamSynchronize(s) != hipSuccess) {
      if (st == SG_OK) st = fail(SG_EDEVICE, "tuning synchronisation");
      break;
    }
    if (ci > 0 && std::memcmp(h_ref.data(), h_out.data(), (size_t)total * sizeof(double2)) != 0) {
      st = fail(SG_EDEVICE, "schedules disagree bitwise");
      break;
    }
    double t = 1e300;
    for (int round = 0; round < 3; ++round) {
      hipEventRecord(e0, s);
      for (int r = 0; r < reps; ++r) apply_all();
      hipEventRecord(e1, s);
      hipEventSynchronize(e1);
      float ms = 0.f;
      hipEventElapsedTime(&ms, e0, e1);
      t = std::min(t, (double)ms / reps);
    }
    // the default (first) stays unless another schedule is faster by more
    // than the timing noise
    if (ci == 0 || t < 0.99 * best_t) {
      best_t = t;
      best = cand[ci];
    }
  }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  if (st != SG_OK) {
    for (int i = 0; i < n; ++i) b->probs[i]->block_grid = saved[i];
    rebuild(saved.empty() ? 0 : saved[0]);
    for (int i = 0; i < n; ++i) b->probs[i]->block_grid = saved[i];
    return st;
  }
  if ((st = rebuild(best)) != SG_OK) return st;
  if (chosen_block_min_grid) *chosen_block_min_grid = best;
  if (best_ms) *best_ms = best_t;
  return SG_OK;
}

sg_status sg_batch_free(sg_batch *b) {
  if (!b) return SG_OK;
  plan_free(&b->plan);
  hipFree(b->d_results);
  if (b->h_results) hipHostFree(b->h_results);
  if (b->own) hipStreamDestroy(b->own);
  delete b;
  return SG_OK;
}

sg_status sg_batch_size(const sg_batch *b, int32_t *n, int64_t *n_cs) {
  if (!b || !n) return fail(SG_EINVAL, "NULL argument");
  *n = (int32_t)b->probs.size();
  if (n_cs)
    for (size_t i = 0; i < b->probs.size(); ++i) n_cs[i] = b->probs[i]->h.ncs;
  return SG_OK;
}

sg_status sg_batch_propagate(sg_batch *b, void *const *psi, int32_t n_psi, const double *dt,
                             int32_t nsteps, const double *emin, const double *emax, double tol,
                             sg_precision prec, int32_t check_every, int32_t use_graph,
                             sg_prop_stats *stats, void *stream) {
  if (!b || !psi || !dt) return fail(SG_EINVAL, "NULL argument");
  if (n_psi != (int32_t)b->probs.size())
    return fail(SG_EINVAL, "the number of states must equal the batch's number of instances");
  if (nsteps < 0 || check_every < 0) return fail(SG_EINVAL, "nsteps, check_every must be >= 0");
  if (prec != SG_FP64 && prec != SG_MIXED) return fail(SG_EINVAL, "unknown precision");
  if (!precision_ok(b->plan, prec))
    return fail(SG_EINVAL, "a tabulated potential runs in FP64 (the batch has FP32 terms)");
  if (!potentials_current(b))
    return fail(SG_EINVAL, "a problem's potential changed after the batch was created");
  hipStream_t s = (hipStream_t)stream;
  const int n = (int)b->probs.size();
  Plan &pl = b->plan;
  std::vector<sg_prop_stats> st(n);
  std::vector<int> ntrace(n, 0);
  int kmax = 0;
  for (int i = 0; i < n; ++i) {
    sg_problem *p = b->probs[i];
    if (!psi[i] || !(dt[i] > 0.0) || !std::isfinite(dt[i])) return fail(SG_EINVAL, "bad psi or dt");
    double lo = emin ? emin[i] : NAN, hi = emax ? emax[i] : NAN;
    if (std::isnan(lo) || std::isnan(hi)) {
      sg_status r = sg_spectral_bounds(p, 40, &lo, &hi, stream);
      if (r != SG_OK) return r;
    }
    if (!(hi > lo)) return fail(SG_EINVAL, "emax must exceed emin");
    const double half = 0.5 * (hi - lo), ebar = 0.5 * (hi + lo);
    std::vector<double> a;
    const int K = chebyshev_series(half * dt[i], &a);
    if (K < 2 || K > kMaxChebTerms) return fail(SG_EINVAL, "Chebyshev series length out of range");
    hipError_t e = hipMemcpyAsync(p->d_cheb_a, a.data(), K * sizeof(double), hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return hip_fail(e, "upload series");
    InstDev &I = pl.inst[i];
    I.x0 = (double2 *)psi[i];
    I.K = K;
    I.ebar = ebar;
    I.inv_half = 1.0 / half;
    I.phase_re = std::cos(-ebar * dt[i]);
    I.phase_im = std::sin(-ebar * dt[i]);
    I.active = 1;
    kmax = std::max(kmax, K);
    st[i].cheb_terms = K;
    st[i].emin = lo;
    st[i].emax = hi;
  }
  sg_status r = plan_upload_inst(&pl, s);
  if (r != SG_OK) return r;

  // optional graph of one step, replayed on the library's own stream
  hipGraphExec_t exec = nullptr;
  hipEvent_t ev_in = nullptr, ev_out = nullptr;
  auto cleanup = [&]() {
    if (exec) hipGraphExecDestroy(exec);
    if (ev_in) hipEventDestroy(ev_in);
    if (ev_out) hipEventDestroy(ev_out);
  };
  if (use_graph) {
    hipGraph_t g = nullptr;
    hipError_t e = hipEventCreateWithFlags(&ev_in, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&ev_out, hipEventDisableTiming);
    if (e == hipSuccess) e = hipStreamBeginCapture(b->own, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) {
      cleanup();
      return hip_fail(e, "graph capture");
    }
    sg_status cs = batch_step_launches(b, prec, kmax, b->own);
    e = hipStreamEndCapture(b->own, &g);
    if (cs != SG_OK) {
      if (g) hipGraphDestroy(g);
      cleanup();
      return cs;
    }
    if (e == hipSuccess) e = hipGraphInstantiate(&exec, g, nullptr, nullptr, 0);
    if (g) hipGraphDestroy(g);
    if (e != hipSuccess) {
      cleanup();
      return hip_fail(e, "graph instantiate");
    }
  }

  sg_status ret = SG_OK;
  LaunchCtl c;
  c.mode = Mode::Cheb;
  c.prec = launch_precision(pl, prec);
  for (int step = 0; step < nsteps && ret == SG_OK; ++step) {
    const bool check = step == 0 || (check_every > 0 && step % check_every == 0);
    if (check || !exec) {
      for (int k = 1; k < kmax; ++k) {
        c.k = k;
        c.want_partials = (k == 1 && check) ? 1 : 0;
        hipError_t e = launch_sweep(&pl, c, s);
        if (e == hipSuccess) e = launch_reduce(&pl, c, s);
        if (e == hipSuccess && k == 1 && check) e = launch_finalize(&pl, s);
        if (e == hipSuccess && k == 1 && check)
          e = hipMemcpyAsync(b->h_results, b->d_results, 2 * n * sizeof(double),
                             hipMemcpyDeviceToHost, s);
        if (e != hipSuccess) {
          cleanup();
          return hip_fail(e, "batched step");
        }
      }
      if (check) {
        hipError_t e = hipStreamSynchronize(s);
        if (e != hipSuccess) {
          cleanup();
          return hip_fail(e, "batched check");
        }
        for (int i = 0; i < n; ++i) {
          const double nrm2 = b->h_results[2 * i], ene = b->h_results[2 * i + 1];
          const double nrm = std::sqrt(nrm2), E = ene / nrm2;
          if (ntrace[i] == 0) {
            st[i].norm0 = nrm;
            st[i].energy0 = E;
          }
          st[i].norm_last = nrm;
          st[i].energy_last = E;
          st[i].max_norm_drift = std::max(st[i].max_norm_drift, std::fabs(nrm - st[i].norm0));
          st[i].max_energy_drift = std::max(st[i].max_energy_drift, std::fabs(E - st[i].energy0));
          ntrace[i]++;
          if (tol > 0.0 && std::fabs(nrm - st[i].norm0) > tol) ret = SG_ETOL;
        }
      }
    } else {
      hipError_t e = hipEventRecord(ev_in, s);
      if (e == hipSuccess) e = hipStreamWaitEvent(b->own, ev_in, 0);
      if (e == hipSuccess) e = hipGraphLaunch(exec, b->own);
      if (e == hipSuccess) e = hipEventRecord(ev_out, b->own);
      if (e == hipSuccess) e = hipStreamWaitEvent(s, ev_out, 0);
      if (e != hipSuccess) {
        cleanup();
        return hip_fail(e, "graph launch");
      }
    }
    for (int i = 0; i < n; ++i) {
      st[i].applies += st[i].cheb_terms - 1;
      st[i].steps_done = step + 1;
    }
  }
  hipError_t e = hipStreamSynchronize(s);
  cleanup();
  if (e != hipSuccess) return hip_fail(e, "batched propagation");
  if (stats)
    for (int i = 0; i < n; ++i) stats[i] = st[i];
  if (ret == SG_ETOL) return fail(SG_ETOL, "norm drift beyond tolerance in a batch instance");
  return ret;
}

}  // extern "C"
