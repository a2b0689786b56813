// C ABI entry points: problem lifetime, ordering exports, initial state and
// the operator action.  See include/sg.h for the contract of each call.
#include <cmath>
#include <cstring>
#include <new>
#include <string>

#include "sg_internal.h"

namespace sg {
thread_local std::string g_last_error;

sg_status fail(sg_status st, const std::string &msg) {
  g_last_error = msg;
  return st;
}

sg_status hip_fail(hipError_t e, const char *what) {
  return fail(SG_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

namespace {

template <typename T>
hipError_t upload(T **dst, const T *src, size_t n, int64_t *bytes) {
  size_t sz = n * sizeof(T);
  if (sz == 0) sz = sizeof(T);
  hipError_t e = hipMalloc((void **)dst, sz);
  if (e != hipSuccess) return e;
  *bytes += (int64_t)sz;
  if (n) e = hipMemcpy(*dst, src, n * sizeof(T), hipMemcpyHostToDevice);
  return e;
}

constexpr int kTimingPairs = 2048;

// Reads back every recorded (start, stop) pair and accumulates durations.
hipError_t flush_timing(sg_problem *p) {
  auto &T = p->timing;
  if (T.used == 0) return hipSuccess;
  hipError_t e = hipEventSynchronize(T.ev[2 * (T.used - 1) + 1]);
  if (e != hipSuccess) return e;
  for (int i = 0; i < T.used; ++i) {
    float ms = 0.f;
    e = hipEventElapsedTime(&ms, T.ev[2 * i], T.ev[2 * i + 1]);
    if (e != hipSuccess) return e;
    T.ms[T.kind[i]] += ms;
    T.n[T.kind[i]] += 1;
  }
  T.used = 0;
  return hipSuccess;
}

// The events are attached to the kernel dispatches (start of the first,
// end of the last), so a pair measures the kernels and no event packets.
template <typename F>
hipError_t timed(sg_problem *p, int kind, hipStream_t s, const LaunchCtl &c, F launch) {
  auto &T = p->timing;
  if (!T.on) return launch(c);
  if (T.used == kTimingPairs) {
    hipError_t e = flush_timing(p);
    if (e != hipSuccess) return e;
  }
  LaunchCtl ct = c;
  ct.ev0 = T.ev[2 * T.used];
  ct.ev1 = T.ev[2 * T.used + 1];
  hipError_t e = launch(ct);
  if (e != hipSuccess) return e;
  T.kind[T.used] = kind;
  T.used += 1;
  T.stream = s;
  return hipSuccess;
}

void release(sg_problem *p) {
  if (!p) return;
  if (p->host_only) {
    delete p;
    return;
  }
  for (hipEvent_t ev : p->timing.ev) hipEventDestroy(ev);
  hipFree(p->d_veff);
  hipFree(p->d_voff);
  if (p->plan) {
    plan_free(p->plan);
    delete p->plan;
  }
  hipFree(p->d_terms);
  hipFree(p->d_tables32);
  hipFree(p->d_tables32r);
  hipFree(p->d_mb);
  hipFree(p->d_inv_ptr);
  hipFree(p->d_inv_col);
  hipFree(p->d_rows);
  hipFree(p->d_tables);
  hipFree(p->d_pairs);
  hipFree(p->d_potc);
  hipFree(p->d_h0);
  hipFree(p->d_tm);
  hipFree(p->d_work);
  hipFree(p->d_partials);
  hipFree(p->d_abc);
  hipFree(p->d_cheb_a);
  hipFree(p->d_result);
  if (p->h_result) hipHostFree(p->h_result);
  delete p;
}

}  // namespace

hipError_t run_sweep(sg_problem *owner, const Plan *pl, const LaunchCtl &c, hipStream_t s) {
  if (!owner) return launch_sweep(pl, c, s);
  return timed(owner, 0, s, c, [&](const LaunchCtl &ct) { return launch_sweep(pl, ct, s); });
}

hipError_t run_reduce(sg_problem *owner, const Plan *pl, const LaunchCtl &c, hipStream_t s) {
  if (!owner) return launch_reduce(pl, c, s);
  return timed(owner, 1, s, c, [&](const LaunchCtl &ct) { return launch_reduce(pl, ct, s); });
}

hipError_t run_vib_sweep(sg_problem *owner, const VibLaunch &v, const double2 *vin, double2 *tm,
                         hipStream_t s) {
  if (!owner) return launch_vib_sweep(v, vin, tm, s, nullptr, nullptr);
  return timed(owner, 0, s, LaunchCtl{}, [&](const LaunchCtl &ct) {
    return launch_vib_sweep(v, vin, tm, s, ct.ev0, ct.ev1);
  });
}

}  // namespace sg

using namespace sg;

extern "C" {

const char *sg_last_error(void) { return g_last_error.c_str(); }

sg_status sg_count_sizes(int32_t D, int32_t L, int32_t nb_A, int32_t nb_B, int64_t out[3]) {
  if (!out) return fail(SG_EINVAL, "out is NULL");
  sg_status st = count_sizes(D, L, nb_A, nb_B, out);
  if (st != SG_OK) return fail(st, "invalid or overflowing size parameters");
  return SG_OK;
}

sg_status sg_build_terms(const sg_problem_desc *desc, sg_problem **out) {
  if (!out) return fail(SG_EINVAL, "out is NULL");
  *out = nullptr;
  sg_problem *p = new (std::nothrow) sg_problem();
  if (!p) return fail(SG_ENOMEM, "host allocation failed");
  std::string err;
  sg_status st;
  try {
    st = compile_problem(desc, &p->h, &err);
  } catch (const std::bad_alloc &) {
    delete p;
    return fail(SG_ENOMEM, "host allocation failed while compiling terms");
  }
  if (st != SG_OK) {
    delete p;
    return fail(st, err);
  }
  return upload_problem(p, out);
}

}  // extern "C"

namespace sg {

int64_t estimate_device_bytes(const Compiled &h) {
  const int64_t ns = (int64_t)h.MB.size();
  return (int64_t)h.terms.size() * (int64_t)sizeof(TermDev) + (int64_t)h.pairs.size() * 8 + (int64_t)h.potc.size() * 8 +
         ns * 4 * 2 + (h.ncs + 1) * 4 + h.ncs * 4 + h.ncs * 8 + ns * 16 + 4 * h.ncs * 16 +
         4 * std::max<int64_t>(h.n_items, 256) * 8 +
         6 * std::max<int64_t>(h.nfib, 1) * 8 +
         (int64_t)h.tables.size() * 20 +
         (int64_t)sizeof(double) * (kMaxChebTerms + 8);
}

// Uploads a compiled problem to the current device (takes ownership of p;
// frees it on failure).
sg_status upload_problem(sg_problem *p, sg_problem **out) {
  std::string err;
  sg_status st;
  const Compiled &h = p->h;
  hipError_t e = hipGetDevice(&p->device);
  if (e != hipSuccess) { delete p; return hip_fail(e, "hipGetDevice"); }
  int64_t &bytes = p->device_bytes;
  const int64_t ns = (int64_t)h.MB.size();
#define SG_UP(dst, vec)                                                  \
  e = upload(&p->dst, (vec).data(), (vec).size(), &bytes);               \
  if (e != hipSuccess) { release(p); return hip_fail(e, "upload " #dst); }
  SG_UP(d_terms, h.terms)
  SG_UP(d_tables32, h.tables32)
  SG_UP(d_tables32r, h.tables32r)
  SG_UP(d_mb, h.mbd)
  SG_UP(d_inv_ptr, h.red_ptr)
  SG_UP(d_inv_col, h.red_col)
  SG_UP(d_rows, h.rows)
  SG_UP(d_tables, h.tables)
  SG_UP(d_pairs, h.pairs)
  SG_UP(d_potc, h.potc)
  SG_UP(d_h0, h.h0)
#undef SG_UP
  {
    // per-fiber coefficients of the split coupling potential, both variants
    const size_t abc_bytes = 6 * (size_t)std::max<int64_t>(h.nfib, 1) * sizeof(double);
    e = hipMalloc((void **)&p->d_abc, abc_bytes);
    if (e != hipSuccess) { release(p); return fail(SG_ENOMEM, "device allocation failed"); }
    bytes += (int64_t)abc_bytes;
    e = launch_fiber_coeffs(p->d_terms, h.nterms, p->d_potc, p->d_tables, p->d_tables32r,
                            p->d_abc, h.nfib, nullptr);
    if (e == hipSuccess) e = hipStreamSynchronize(nullptr);
    if (e != hipSuccess) { release(p); return hip_fail(e, "per-fiber potential coefficients"); }
  }
  size_t tm_bytes = (size_t)ns * sizeof(double2);
  e = hipMalloc((void **)&p->d_tm, tm_bytes);
  if (e != hipSuccess) { release(p); return fail(SG_ENOMEM, "device allocation of the term-major buffer failed"); }
  bytes += (int64_t)tm_bytes;
  size_t work_bytes = 4 * (size_t)h.ncs * sizeof(double2);
  e = hipMalloc((void **)&p->d_work, work_bytes);
  if (e != hipSuccess) { release(p); return fail(SG_ENOMEM, "device allocation of work vectors failed"); }
  bytes += (int64_t)work_bytes;
  const int64_t npart = std::max<int64_t>(h.n_items, 256);
  e = hipMalloc((void **)&p->d_partials, 2 * (size_t)npart * sizeof(double));
  if (e != hipSuccess) { release(p); return fail(SG_ENOMEM, "device allocation failed"); }
  bytes += 2 * npart * (int64_t)sizeof(double);
  e = hipMalloc((void **)&p->d_cheb_a, kMaxChebTerms * sizeof(double));
  if (e != hipSuccess) { release(p); return fail(SG_ENOMEM, "device allocation failed"); }
  e = hipMalloc((void **)&p->d_result, 8 * sizeof(double));
  if (e != hipSuccess) { release(p); return fail(SG_ENOMEM, "device allocation failed"); }
  e = hipHostMalloc((void **)&p->h_result, 8 * sizeof(double), hipHostMallocDefault);
  if (e != hipSuccess) { release(p); return fail(SG_ENOMEM, "pinned host allocation failed"); }
  p->plan = new (std::nothrow) Plan();
  if (!p->plan) { release(p); return fail(SG_ENOMEM, "host allocation failed"); }
  st = plan_build(p->plan, {p}, &err);
  if (st == SG_OK) st = plan_upload(p->plan, nullptr);
  if (st != SG_OK) {
    std::string msg = sg_last_error();
    release(p);
    return fail(st, msg.empty() ? err : msg);
  }
  bytes += p->plan->scratch_bytes;
  *out = p;
  return SG_OK;
}

void release_problem(sg_problem *p) { release(p); }

}  // namespace sg

extern "C" {

sg_status sg_build_terms_host(const sg_problem_desc *desc, sg_problem **out) {
  if (!out) return fail(SG_EINVAL, "out is NULL");
  *out = nullptr;
  sg_problem *p = new (std::nothrow) sg_problem();
  if (!p) return fail(SG_ENOMEM, "host allocation failed");
  p->host_only = true;
  std::string err;
  sg_status st;
  try {
    st = compile_problem(desc, &p->h, &err);
  } catch (const std::bad_alloc &) {
    delete p;
    return fail(SG_ENOMEM, "host allocation failed while compiling terms");
  }
  if (st != SG_OK) {
    delete p;
    return fail(st, err);
  }
  *out = p;
  return SG_OK;
}

sg_status sg_free(sg_problem *p) {
  if (!p) return SG_OK;
  if (p->host_only) {
    release(p);
    return SG_OK;
  }
  int cur = 0;
  hipGetDevice(&cur);
  hipSetDevice(p->device);
  release(p);
  hipSetDevice(cur);
  return SG_OK;
}

sg_status sg_problem_info(const sg_problem *p, sg_info *out) {
  if (!p || !out) return fail(SG_EINVAL, "NULL argument");
  const Compiled &h = p->h;
  out->D = h.D;
  out->L = h.L;
  out->n_terms = h.nterms;
  out->n_cs = h.ncs;
  out->n_s = (int64_t)h.MB.size();
  out->grid_literal = h.grid_literal;
  out->grid_active = h.grid_active;
  out->max_term_basis = h.max_basis;
  out->max_term_grid = h.max_grid;
  const bool split = p->host_only ? (h.split_exact && !p->grid_kinetic)
                                   : (p->plan && p->plan->fp64_split);
  const double red_grid = 2.0 * (double)h.MB.size();
  const double red_split = 2.0 * (double)h.MB.size() + 4.0 * (double)h.ncs;
  out->flops_fp64 = split ? h.flops_mixed : h.flops_fp64;
  out->flops_mixed = h.flops_mixed;
  out->sweep_flops_fp64 = split ? h.flops_mixed - red_split : h.flops_fp64 - red_grid;
  out->sweep_flops_mixed = h.flops_mixed - red_split;
  out->bytes_fp64 = h.bytes_apply;
  out->device_bytes = p->device_bytes;
  out->fp64_split = split ? 1 : 0;
  out->pad = 0;
  const double ns = (double)h.MB.size(), ncs = (double)h.ncs;
  out->sweep_bytes = 16.0 * ncs + 4.0 * ns + 16.0 * ns + 4.0 * kTermHdrDwords * (double)h.nterms +
                     (p->d_veff ? 8.0 * (double)h.grid_active : split ? 24.0 * (double)h.nfib : 0.0);
  out->reduce_bytes = 16.0 * ns + 4.0 * ns + 8.0 * ncs + 16.0 * ncs + (split ? 8.0 * ncs : 0.0) +
                      16.0 * ncs;
  return SG_OK;
}

sg_status sg_basis_indices(const sg_problem *p, int32_t *n_out) {
  if (!p || !n_out) return fail(SG_EINVAL, "NULL argument");
  for (size_t i = 0; i < p->h.compact.size(); ++i) n_out[i] = p->h.compact[i];
  return SG_OK;
}

sg_status sg_term_levels(const sg_problem *p, int32_t *levels, int32_t *coeffs) {
  if (!p) return fail(SG_EINVAL, "NULL problem");
  if (levels)
    for (size_t i = 0; i < p->h.lev.size(); ++i) levels[i] = p->h.lev[i];
  if (coeffs)
    for (size_t i = 0; i < p->h.coeff.size(); ++i) coeffs[i] = p->h.coeff[i];
  return SG_OK;
}

sg_status sg_mapping_table(const sg_problem *p, int32_t *mb) {
  if (!p || !mb) return fail(SG_EINVAL, "NULL argument");
  std::memcpy(mb, p->h.MB.data(), p->h.MB.size() * sizeof(int32_t));
  return SG_OK;
}

sg_status sg_init_gaussian(const sg_problem *p, const double *shift, void *psi_dev,
                           double *captured_norm, void *stream) {
  if (!p || !shift || !psi_dev) return fail(SG_EINVAL, "NULL argument");
  if (p->host_only) return fail(SG_EINVAL, "handle was built without device tables");
  const Compiled &h = p->h;
  // coherent-state coefficients e^{-a^2/2} a^n / sqrt(n!), a = s/sqrt(2)
  std::vector<double> tab((size_t)h.D * (h.nmax + 1));
  for (int i = 0; i < h.D; ++i) {
    if (!std::isfinite(shift[i])) return fail(SG_EINVAL, "shift must be finite");
    const double a = shift[i] / std::sqrt(2.0);
    double v = std::exp(-0.5 * a * a);
    for (int n = 0; n <= h.nmax; ++n) {
      if (n > 0) v *= a / std::sqrt((double)n);
      tab[(size_t)i * (h.nmax + 1) + n] = v;
    }
  }
  std::vector<double2> c(h.ncs);
  double nrm2 = 0.0;
  for (int64_t r = 0; r < h.ncs; ++r) {
    double v = 1.0;
    for (int i = 0; i < h.D; ++i) v *= tab[(size_t)i * (h.nmax + 1) + h.compact[(size_t)r * h.D + i]];
    c[r] = make_double2(v, 0.0);
    nrm2 += v * v;
  }
  const double nrm = std::sqrt(nrm2);
  if (!(nrm > 0.0)) return fail(SG_EINVAL, "initial state has zero projection");
  for (auto &x : c) x.x /= nrm;
  if (captured_norm) *captured_norm = nrm;
  hipError_t e = hipMemcpyAsync(psi_dev, c.data(), c.size() * sizeof(double2),
                                hipMemcpyHostToDevice, (hipStream_t)stream);
  if (e == hipSuccess) e = hipStreamSynchronize((hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "upload initial state");
  return SG_OK;
}

sg_status sg_apply_H(sg_problem *p, const void *psi_in, void *psi_out, sg_precision prec,
                     void *stream) {
  if (!p || !psi_in || !psi_out) return fail(SG_EINVAL, "NULL argument");
  if (psi_in == psi_out) return fail(SG_EINVAL, "psi_in and psi_out must differ");
  if (p->host_only) return fail(SG_EINVAL, "handle was built without device tables");
  if (prec != SG_FP64 && prec != SG_MIXED) return fail(SG_EINVAL, "unknown precision");
  if (p->d_veff && prec != SG_FP64) return fail(SG_EINVAL, "a tabulated potential runs in FP64");
  hipStream_t s = (hipStream_t)stream;
  LaunchCtl c;
  c.mode = Mode::Apply;
  c.prec = prec;
  c.x0o = (double2 *)psi_in;
  c.x1o = (double2 *)psi_out;
  hipError_t e = run_sweep(p, p->plan, c, s);
  if (e != hipSuccess) return hip_fail(e, "term sweep launch");
  e = run_reduce(p, p->plan, c, s);
  if (e != hipSuccess) return hip_fail(e, "reduce launch");
  return SG_OK;
}

}  // extern "C"

namespace {
// Rebuilds and re-uploads a problem's launch plan after a setting changed.
// The device is synchronised first: launches still in flight on any stream
// read the plan's packs and items, which the upload overwrites in place.
sg_status rebuild_plan(sg_problem *p) {
  if (p->host_only) return SG_OK;
  hipError_t e = hipDeviceSynchronize();
  if (e != hipSuccess) return hip_fail(e, "synchronise before the plan upload");
  std::string err;
  sg_status st = plan_build(p->plan, {p}, &err);
  if (st != SG_OK) return fail(st, err);
  st = plan_upload(p->plan, nullptr);
  if (st != SG_OK) return st;
  e = hipStreamSynchronize(nullptr);
  return e == hipSuccess ? SG_OK : hip_fail(e, "plan upload");
}
}  // namespace

namespace sg {
sg_status problem_replan(sg_problem *p) { return rebuild_plan(p); }
}  // namespace sg

extern "C" {

sg_status sg_set_mixed_threshold(sg_problem *p, int32_t max_fp32_coeff) {
  if (!p) return fail(SG_EINVAL, "NULL problem");
  if (max_fp32_coeff < 0) return fail(SG_EINVAL, "threshold must be >= 0");
  p->h.mixed_max_fp32_coeff = max_fp32_coeff;
  return rebuild_plan(p);
}

sg_status sg_set_schedule(sg_problem *p, int32_t block_min_grid, int32_t packs_per_cu) {
  if (!p) return fail(SG_EINVAL, "NULL problem");
  if (block_min_grid < 0) return fail(SG_EINVAL, "block_min_grid must be >= 0");
  if (packs_per_cu < 1 || packs_per_cu > 4) return fail(SG_EINVAL, "packs_per_cu must be 1..4");
  p->block_grid = block_min_grid;
  p->packs_per_cu = packs_per_cu;
  return rebuild_plan(p);
}
sg_status sg_set_operator_form(sg_problem *p, int32_t grid_kinetic) {
  if (!p) return fail(SG_EINVAL, "NULL problem");
  if (grid_kinetic != 0 && grid_kinetic != 1) return fail(SG_EINVAL, "grid_kinetic must be 0 or 1");
  if (p->d_veff && grid_kinetic)
    return fail(SG_EINVAL, "a tabulated potential needs the split operator form");
  p->grid_kinetic = grid_kinetic;
  return rebuild_plan(p);
}

sg_status sg_set_timing(sg_problem *p, int32_t enable) {
  if (!p) return fail(SG_EINVAL, "NULL problem");
  if (p->host_only) return fail(SG_EINVAL, "handle was built without device tables");
  auto &T = p->timing;
  if (T.on) {
    hipError_t e = flush_timing(p);
    if (e != hipSuccess) return hip_fail(e, "timing flush");
  }
  if (enable && T.ev.empty()) {
    T.ev.resize(2 * kTimingPairs);
    T.kind.resize(kTimingPairs);
    for (auto &ev : T.ev) {
      hipError_t e = hipEventCreate(&ev);
      if (e != hipSuccess) return hip_fail(e, "hipEventCreate");
    }
  }
  T.on = enable != 0;
  T.used = 0;
  T.ms[0] = T.ms[1] = 0.0;
  T.n[0] = T.n[1] = 0;
  return SG_OK;
}

sg_status sg_get_timing(sg_problem *p, sg_timing *out) {
  if (!p || !out) return fail(SG_EINVAL, "NULL argument");
  hipError_t e = flush_timing(p);
  if (e != hipSuccess) return hip_fail(e, "timing flush");
  out->sweep_ms = p->timing.ms[0];
  out->sweep_launches = p->timing.n[0];
  out->reduce_ms = p->timing.ms[1];
  out->reduce_launches = p->timing.n[1];
  return SG_OK;
}

}  // extern "C"
