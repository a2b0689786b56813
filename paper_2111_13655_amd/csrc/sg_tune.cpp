// Precision autotuner of the mixed path.
//
// Candidate policies put the terms with |D_l| <= t in FP32 for t running
// from "all terms" down to "none" (the exact FP64 split).  Each candidate is
// applied to the caller's state and compared with the plain FP64 operator;
// among those whose relative error stays below half the tolerance, the one
// with the shortest measured apply time is kept.  Rounding errors of one
// apply amplify with the spread of the D_l (they enter the Smolyak sum with
// weight |D_l|), so the tolerance is checked by measurement, not by a model.
#include <algorithm>
#include <climits>
#include <cmath>
#include <cstring>
#include <vector>

#include "sg_internal.h"

namespace sg {
namespace {

sg_status rel_error(sg_problem *p, const double2 *x, const double2 *ref, double2 *diff,
                    hipStream_t s, double *rel) {
  const int64_t n = p->h.ncs;
  hipError_t e = hipMemcpyAsync(diff, x, n * sizeof(double2), hipMemcpyDeviceToDevice, s);
  if (e == hipSuccess) e = launch_axpby(n, diff, ref, -1.0, 0.0, 1.0, s);
  if (e == hipSuccess) e = launch_dot(p, diff, diff, s);
  if (e != hipSuccess) return hip_fail(e, "tuning error norm");
  double d2, di, r2, ri;
  e = hipMemcpyAsync(p->h_result, p->d_result, 2 * sizeof(double), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(e, "tuning readback");
  d2 = p->h_result[0];
  di = p->h_result[1];
  e = launch_dot(p, ref, ref, s);
  if (e == hipSuccess)
    e = hipMemcpyAsync(p->h_result, p->d_result, 2 * sizeof(double), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(e, "tuning readback");
  r2 = p->h_result[0];
  ri = p->h_result[1];
  (void)di;
  (void)ri;
  *rel = r2 > 0.0 ? std::sqrt(std::max(d2, 0.0) / r2) : 0.0;
  return SG_OK;
}

}  // namespace
}  // namespace sg

using namespace sg;

extern "C" {

sg_status sg_tune_mixed(sg_problem *p, const void *psi, double tol, int32_t reps,
                        int32_t *chosen, double *chosen_error, void *stream) {
  if (!p || !psi) return fail(SG_EINVAL, "NULL argument");
  if (p->host_only) return fail(SG_EINVAL, "handle was built without device tables");
  if (!(tol > 0.0) || reps < 1) return fail(SG_EINVAL, "tol must be > 0 and reps >= 1");
  hipStream_t s = (hipStream_t)stream;
  const int64_t n = p->h.ncs;
  double2 *ref = p->d_work + 2 * n, *out = p->d_work + 3 * n, *diff = p->d_work + 0 * n;
  if (psi == ref || psi == out || psi == diff) return fail(SG_EINVAL, "psi aliases work buffers");
  sg_status st = sg_apply_H(p, psi, ref, SG_FP64, stream);
  if (st != SG_OK) return st;
  std::vector<int32_t> cand = {INT_MAX};
  {
    std::vector<int32_t> mags;
    for (int32_t c : p->h.coeff) mags.push_back(std::abs(c));
    std::sort(mags.begin(), mags.end());
    mags.erase(std::unique(mags.begin(), mags.end()), mags.end());
    for (auto it = mags.rbegin(); it != mags.rend(); ++it) cand.push_back(*it);
    cand.push_back(0);
  }
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
    return fail(SG_EDEVICE, "hipEventCreate");
  int32_t best = 0;
  double best_t = 1e300, best_err = 0.0;
  const int32_t saved = p->h.mixed_max_fp32_coeff;
  for (int32_t t : cand) {
    if ((st = sg_set_mixed_threshold(p, t)) != SG_OK) break;
    if ((st = sg_apply_H(p, psi, out, SG_MIXED, stream)) != SG_OK) break;
    double err = 0.0;
    if ((st = rel_error(p, out, ref, diff, s, &err)) != SG_OK) break;
    if (err > 0.5 * tol) continue;
    hipEventRecord(e0, s);
    for (int r = 0; r < reps; ++r)
      if ((st = sg_apply_H(p, psi, out, SG_MIXED, stream)) != SG_OK) break;
    if (st != SG_OK) break;
    hipEventRecord(e1, s);
    hipEventSynchronize(e1);
    float ms = 0.f;
    hipEventElapsedTime(&ms, e0, e1);
    if (ms < best_t) {
      best_t = ms;
      best = t;
      best_err = err;
    }
  }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  if (st != SG_OK) {
    sg_set_mixed_threshold(p, saved);
    return st;
  }
  if ((st = sg_set_mixed_threshold(p, best)) != SG_OK) return st;
  if (chosen) *chosen = best;
  if (chosen_error) *chosen_error = best_err;
  return SG_OK;
}


sg_status sg_tune_schedule(sg_problem *p, const void *psi, int32_t prec, int32_t reps,
                           int32_t *chosen_block_min_grid, int32_t *chosen_packs_per_cu,
                           void *stream) {
  if (!p || !psi) return fail(SG_EINVAL, "NULL argument");
  if (p->host_only) return fail(SG_EINVAL, "handle was built without device tables");
  if (reps < 1) return fail(SG_EINVAL, "reps must be >= 1");
  if (prec != SG_FP64 && prec != SG_MIXED) return fail(SG_EINVAL, "unknown precision");
  hipStream_t s = (hipStream_t)stream;
  const int64_t n = p->h.ncs;
  double2 *ref = p->d_work + 2 * n, *out = p->d_work + 3 * n;
  if (psi == ref || psi == out) return fail(SG_EINVAL, "psi aliases work buffers");
  std::vector<std::pair<int32_t, int32_t>> cand;
  for (int32_t spread = 1; spread <= 2; ++spread) {
    cand.push_back({0, spread});
    for (int32_t g = 64; g <= p->h.max_grid; g *= 2) cand.push_back({g, spread});
  }
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
    return fail(SG_EDEVICE, "hipEventCreate");
  const std::pair<int32_t, int32_t> saved = {p->block_grid, p->packs_per_cu};
  std::vector<double2> h_ref((size_t)n), h_out((size_t)n);
  sg_status st = SG_OK;
  std::pair<int32_t, int32_t> best = saved;
  double best_t = 1e300;
  for (size_t i = 0; i < cand.size() && st == SG_OK; ++i) {
    if ((st = sg_set_schedule(p, cand[i].first, cand[i].second)) != SG_OK) break;
    if ((st = sg_apply_H(p, psi, out, (sg_precision)prec, stream)) != SG_OK) break;
    // every schedule computes each term with the same arithmetic
    double2 *dst = i == 0 ? h_ref.data() : h_out.data();
    if (hipMemcpyAsync(dst, out, (size_t)n * sizeof(double2), hipMemcpyDeviceToHost, s) !=
            hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess) {
      st = fail(SG_EDEVICE, "copy of the tuning result");
      break;
    }
    if (i > 0 && std::memcmp(h_ref.data(), h_out.data(), (size_t)n * sizeof(double2)) != 0) {
      st = fail(SG_EDEVICE, "schedules disagree bitwise");
      break;
    }
    // best of three timed rounds
    double t = 1e300;
    for (int round = 0; round < 3 && st == SG_OK; ++round) {
      hipEventRecord(e0, s);
      for (int r = 0; r < reps && st == SG_OK; ++r)
        st = sg_apply_H(p, psi, out, (sg_precision)prec, stream);
      hipEventRecord(e1, s);
      hipEventSynchronize(e1);
      float ms = 0.f;
      hipEventElapsedTime(&ms, e0, e1);
      t = std::min(t, (double)ms);
    }
    if (st != SG_OK) break;
    // the default schedule (the first candidate) stays unless another one is
    // faster by more than the timing noise
    if (i == 0 || t < 0.99 * best_t) {
      best_t = t;
      best = cand[i];
    }
  }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  if (st != SG_OK) {
    sg_set_schedule(p, saved.first, saved.second);
    return st;
  }
  if ((st = sg_set_schedule(p, best.first, best.second)) != SG_OK) return st;
  if (chosen_block_min_grid) *chosen_block_min_grid = best.first;
  if (chosen_packs_per_cu) *chosen_packs_per_cu = best.second;
  return SG_OK;
}

}  // extern "C"
