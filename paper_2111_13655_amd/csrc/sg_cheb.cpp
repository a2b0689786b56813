// Chebyshev propagator and spectral bounds.
//
// The paper propagates wave packets with "the Chebyshev method" (Sec. 3,
// Sec. 5) without formulas; the library uses the Tal-Ezer--Kosloff series
// (hbar = 1):
//   Hs = (H - Ebar)/(dE/2),  R = dE dt / 2,
//   exp(-i H dt) psi = exp(-i Ebar dt) sum_k (2 - delta_k0) J_k(R) phi_k,
//   phi_0 = psi, phi_1 = -i Hs psi, phi_{k+1} = -2i Hs phi_k + phi_{k-1}.
// Every apply of H is one term sweep plus one reduce whose epilogue runs the
// recurrence, accumulates the series and, on the last term, writes the new
// state back; the vectors stay on the device for the whole call.
// Bessel values: backward (Miller) recurrence normalised by
// J_0 + 2 sum_k J_{2k} = 1.
#include <algorithm>
#include <cmath>
#include <limits>
#include <vector>

#include "sg_internal.h"

namespace sg {

void bessel_j_sequence(double x, int n, double *out) {
  if (n <= 0) return;
  if (x == 0.0) {
    out[0] = 1.0;
    for (int k = 1; k < n; ++k) out[k] = 0.0;
    return;
  }
  // start well above both n and x
  int start = std::max(n, (int)std::ceil(std::fabs(x))) + 40 + (int)std::sqrt(40.0 * std::fabs(x));
  if (start % 2) ++start;
  std::vector<double> j(start + 2, 0.0);
  j[start + 1] = 0.0;
  j[start] = 1e-300;
  for (int k = start; k >= 1; --k) {
    j[k - 1] = (2.0 * k / x) * j[k] - j[k + 1];
    if (std::fabs(j[k - 1]) > 1e250) {  // rescale to avoid overflow
      for (int m = k - 1; m <= start + 1; ++m) j[m] *= 1e-250;
    }
  }
  double norm = j[0];
  for (int k = 2; k <= start; k += 2) norm += 2.0 * j[k];
  for (int k = 0; k < n; ++k) out[k] = j[k] / norm;
}

int chebyshev_series(double R, std::vector<double> *a) {
  const int K = chebyshev_terms(R, 1e-16);
  a->assign(K, 0.0);
  bessel_j_sequence(R, K, a->data());
  for (int k = 1; k < K; ++k) (*a)[k] *= 2.0;
  return K;
}

int chebyshev_terms(double R, double tol) {
  int k = (int)std::floor(R) + 1;
  std::vector<double> j;
  while (true) {
    j.resize(k + 2);
    bessel_j_sequence(R, k + 2, j.data());
    if (std::fabs(j[k]) < tol && std::fabs(j[k + 1]) < tol) return std::max(k, 2);
    ++k;
    if (k > 100000) return k;
  }
}

namespace {

sg_status read_result(sg_problem *p, hipStream_t s, double *a, double *b) {
  hipError_t e = hipMemcpyAsync(p->h_result, p->d_result, 2 * sizeof(double),
                                hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(e, "read reduction result");
  *a = p->h_result[0];
  *b = p->h_result[1];
  return SG_OK;
}

}  // namespace
}  // namespace sg

using namespace sg;

extern "C" {

sg_status sg_spectral_bounds(sg_problem *p, int32_t iters, double *emin, double *emax,
                             void *stream) {
  if (!p || !emin || !emax) return fail(SG_EINVAL, "NULL argument");
  if (iters < 2) return fail(SG_EINVAL, "iters must be >= 2");
  if (p->host_only) return fail(SG_EINVAL, "handle was built without device tables");
  hipStream_t s = (hipStream_t)stream;
  const int64_t n = p->h.ncs;
  const int m = (int)std::min<int64_t>(iters, n);
  double2 *v_prev = p->d_work + 0 * n, *v = p->d_work + 1 * n, *w = p->d_work + 2 * n;
  // deterministic start vector with every component non-zero
  std::vector<double2> v0(n);
  double nn = 0.0;
  for (int64_t i = 0; i < n; ++i) {
    double x = 1.0 + 0.5 * std::sin(0.7 * (double)i + 0.3);
    v0[i] = make_double2(x, 0.0);
    nn += x * x;
  }
  nn = std::sqrt(nn);
  for (auto &x : v0) x.x /= nn;
  hipError_t e = hipMemcpyAsync(v, v0.data(), n * sizeof(double2), hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipMemsetAsync(v_prev, 0, n * sizeof(double2), s);
  if (e != hipSuccess) return hip_fail(e, "Lanczos setup");
  std::vector<double> alpha, beta;
  double b_prev = 0.0;
  for (int j = 0; j < m; ++j) {
    sg_status st = sg_apply_H(p, v, w, SG_FP64, stream);
    if (st != SG_OK) return st;
    if ((e = launch_dot(p, v, w, s)) != hipSuccess) return hip_fail(e, "dot");
    double are, aim;
    if ((st = read_result(p, s, &are, &aim)) != SG_OK) return st;
    alpha.push_back(are);
    // w = w - alpha v - b_prev v_prev
    if ((e = launch_axpby(n, w, v, -are, 0.0, 1.0, s)) != hipSuccess) return hip_fail(e, "axpby");
    if (j > 0 && (e = launch_axpby(n, w, v_prev, -b_prev, 0.0, 1.0, s)) != hipSuccess)
      return hip_fail(e, "axpby");
    if ((e = launch_dot(p, w, w, s)) != hipSuccess) return hip_fail(e, "dot");
    double bb, bi;
    if ((st = read_result(p, s, &bb, &bi)) != SG_OK) return st;
    double b = std::sqrt(std::max(bb, 0.0));
    beta.push_back(b);
    if (b < 1e-12 || j == m - 1) break;
    // v_prev <- v ; v <- w / b   (rotate by copies through axpby)
    if ((e = launch_axpby(n, v_prev, v, 1.0, 0.0, 0.0, s)) != hipSuccess) return hip_fail(e, "axpby");
    if ((e = launch_axpby(n, v, w, 1.0 / b, 0.0, 0.0, s)) != hipSuccess) return hip_fail(e, "axpby");
    b_prev = b;
  }
  const int k = (int)alpha.size();
  std::vector<double> T((size_t)k * k, 0.0), ev, V;
  for (int i = 0; i < k; ++i) {
    T[(size_t)i * k + i] = alpha[i];
    if (i + 1 < k) T[(size_t)i * k + i + 1] = T[(size_t)(i + 1) * k + i] = beta[i];
  }
  jacobi_eigen(T, k, &ev, &V);
  const double blast = beta.empty() ? 0.0 : beta.back();
  const double res_lo = std::fabs(blast * V[(size_t)(k - 1) * k + 0]);
  const double res_hi = std::fabs(blast * V[(size_t)(k - 1) * k + (k - 1)]);
  const double lo = ev.front(), hi = ev.back();
  const double pad = 0.05 * (hi - lo);
  *emin = lo - std::max(pad, res_lo) - pad;
  *emax = hi + std::max(pad, res_hi) + pad;
  return SG_OK;
}

sg_status sg_propagate_chebyshev(sg_problem *p, void *psi, double dt, int32_t nsteps,
                                 double emin, double emax, double tol, sg_precision prec,
                                 int32_t check_every, sg_prop_stats *stats,
                                 double *norm_trace, double *energy_trace, void *stream) {
  if (!p || !psi) return fail(SG_EINVAL, "NULL argument");
  if (!(dt > 0.0) || !std::isfinite(dt) || nsteps < 0 || check_every < 0)
    return fail(SG_EINVAL, "dt must be > 0, nsteps and check_every >= 0");
  if (prec != SG_FP64 && prec != SG_MIXED) return fail(SG_EINVAL, "unknown precision");
  if (p->d_veff && prec != SG_FP64) return fail(SG_EINVAL, "a tabulated potential runs in FP64");
  if (p->host_only) return fail(SG_EINVAL, "handle was built without device tables");
  hipStream_t s = (hipStream_t)stream;
  if (std::isnan(emin) || std::isnan(emax)) {
    sg_status st = sg_spectral_bounds(p, 40, &emin, &emax, stream);
    if (st != SG_OK) return st;
  }
  if (!(emax > emin)) return fail(SG_EINVAL, "emax must exceed emin");
  const int64_t n = p->h.ncs;
  const double half = 0.5 * (emax - emin), ebar = 0.5 * (emax + emin);
  std::vector<double> a;
  const int K = chebyshev_series(half * dt, &a);
  if (K < 2 || K > kMaxChebTerms) return fail(SG_EINVAL, "Chebyshev series length out of range");
  hipError_t e = hipMemcpyAsync(p->d_cheb_a, a.data(), K * sizeof(double), hipMemcpyHostToDevice, s);
  if (e != hipSuccess) return hip_fail(e, "upload series");
  Plan *pl = p->plan;
  InstDev &I = pl->inst[0];
  I.K = K;
  I.ebar = ebar;
  I.inv_half = 1.0 / half;
  I.phase_re = std::cos(-ebar * dt);
  I.phase_im = std::sin(-ebar * dt);
  I.active = 1;
  sg_status st0 = plan_upload_inst(pl, s);
  if (st0 != SG_OK) return st0;

  sg_prop_stats st{};
  st.cheb_terms = K;
  st.emin = emin;
  st.emax = emax;
  int ntrace = 0;
  bool have0 = false;
  sg_status ret = SG_OK;
  auto record = [&](double nrm2, double ene) {
    const double nrm = std::sqrt(nrm2), E = ene / nrm2;
    if (!have0) {
      st.norm0 = nrm;
      st.energy0 = E;
      have0 = true;
    }
    st.norm_last = nrm;
    st.energy_last = E;
    st.max_norm_drift = std::max(st.max_norm_drift, std::fabs(nrm - st.norm0));
    st.max_energy_drift = std::max(st.max_energy_drift, std::fabs(E - st.energy0));
    if (norm_trace) norm_trace[ntrace] = nrm;
    if (energy_trace) energy_trace[ntrace] = E;
    ++ntrace;
  };
  LaunchCtl c;
  c.mode = Mode::Cheb;
  c.prec = prec;
  c.x0o = (double2 *)psi;
  for (int step = 0; step < nsteps; ++step) {
    const bool check = step == 0 || (check_every > 0 && step % check_every == 0);
    for (int k = 1; k < K; ++k) {
      c.k = k;
      c.want_partials = (k == 1 && check) ? 1 : 0;
      if ((e = run_sweep(p, pl, c, s)) != hipSuccess) return hip_fail(e, "sweep");
      if ((e = run_reduce(p, pl, c, s)) != hipSuccess) return hip_fail(e, "reduce");
      if (k == 1 && check) {
        if ((e = launch_finalize(pl, s)) != hipSuccess) return hip_fail(e, "finalize");
        double nrm2, ene;
        sg_status rs = read_result(p, s, &nrm2, &ene);
        if (rs != SG_OK) return rs;
        record(nrm2, ene);
        if (tol > 0.0 && std::fabs(std::sqrt(nrm2) - st.norm0) > tol) ret = SG_ETOL;
      }
    }
    st.applies += K - 1;
    st.steps_done = step + 1;
    if (ret != SG_OK) break;
  }
  if (ret == SG_OK) {
    // final norm and energy
    double2 *w = p->d_work + 3 * n;
    sg_status as = sg_apply_H(p, psi, w, prec, stream);
    if (as != SG_OK) return as;
    double nr, ni, er, ei;
    if ((e = launch_dot(p, (const double2 *)psi, (const double2 *)psi, s)) != hipSuccess)
      return hip_fail(e, "dot");
    if ((as = read_result(p, s, &nr, &ni)) != SG_OK) return as;
    if ((e = launch_dot(p, (const double2 *)psi, w, s)) != hipSuccess) return hip_fail(e, "dot");
    if ((as = read_result(p, s, &er, &ei)) != SG_OK) return as;
    record(nr, er);
    st.applies += 1;
    if (tol > 0.0 && std::fabs(std::sqrt(nr) - st.norm0) > tol) ret = SG_ETOL;
  }
  if (stats) *stats = st;
  if (ret == SG_ETOL) return fail(SG_ETOL, "norm drift beyond tolerance: spectral bounds too tight?");
  return ret;
}

}  // extern "C"
