// Taylor, Runge-Kutta, Bulirsch-Stoer and short-iterative-Lanczos propagation
// on the operator
// action (the other propagators the paper lists beside the Chebyshev method,
// Sec. 3 overview of the program flow; it gives no formulas).  With hbar = 1
// and d psi/dt = -i H psi:
//
//   Taylor, order n:  psi <- sum_{k<=n} (-i H dt)^k / k! psi, built term by
//     term (term_k = (-i dt / k) H term_{k-1}).
//   Runge-Kutta, order n = 1..4: explicit tableaux (Euler; explicit
//     midpoint; Heun's third-order method; the classical fourth-order
//     method).  Stage i applies H to psi + dt sum_j A_ij k_j with
//     k_j = -i H y_j; the -i is folded into the complex coefficients.
//   Bulirsch-Stoer, k columns (1..8): the modified midpoint rule over
//     n_i = 2i substeps of the step (i = 1..k; H psi is shared by all of
//     them), extrapolated to zero substep size.  The extrapolated value is
//     the interpolating polynomial in h^2 at 0, formed here in Lagrange form,
//     sum_i c_i T_i with c_i = prod_{j != i} i^2 / (i^2 - j^2), in one
//     vector combination.
//   Short iterative Lanczos, Krylov dimension m (Park and Light, 1986):
//     Lanczos from psi/|psi|, every new vector orthogonalised against all
//     earlier ones twice; T = tridiag(alpha, beta); psi <- |psi| V
//     exp(-i T dt) e_1, with exp(-i T dt) from the eigenpairs of T (host).
//     T is cut at the first new vector whose norm is below 1e-13 |psi| (an
//     invariant space).
//
// Every H application is one term sweep plus one reduce; vector updates run
// in the library's vector kernels; the state never leaves the device.  Only
// Lanczos coefficients and checked norms and energies are read back.
#include <algorithm>
#include <cmath>
#include <complex>
#include <utility>
#include <vector>

#include "sg_internal.h"

using namespace sg;

namespace {

constexpr int kMaxTaylorOrder = 40;
constexpr int kMaxKrylov = 64;
constexpr int kMaxColumns = 8;

using Buffers = PropBuffers;

// explicit tableaux: strictly lower A (row-major, 4 x 4) and weights b
struct Tableau {
  int s;
  double A[4][4];
  double b[4];
};
const Tableau kRK[4] = {
    {1, {{0}}, {1.0}},
    {2, {{0, 0}, {0.5, 0}}, {0.0, 1.0}},
    {3, {{0, 0, 0}, {1.0 / 3.0, 0, 0}, {0, 2.0 / 3.0, 0}}, {0.25, 0.0, 0.75}},
    {4, {{0, 0, 0, 0}, {0.5, 0, 0, 0}, {0, 0.5, 0, 0}, {0, 0, 1.0, 0}},
     {1.0 / 6.0, 2.0 / 6.0, 2.0 / 6.0, 1.0 / 6.0}},
};

sg_status read2(sg_problem *p, hipStream_t s, double *a, double *b) {
  hipError_t e = hipMemcpyAsync(p->h_result, p->d_result, 2 * sizeof(double),
                                hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(e, "read reduction result");
  *a = p->h_result[0];
  *b = p->h_result[1];
  return SG_OK;
}

// x = beta x + sum_j c_j V_j (synchronises: the coefficient buffer is reused)
sg_status combine(const Buffers &B, double2 *x, double beta, const double2 *V, int64_t n,
                  const std::vector<std::complex<double>> &c, hipStream_t s) {
  std::vector<double> h(2 * c.size());
  for (size_t j = 0; j < c.size(); ++j) {
    h[2 * j] = c[j].real();
    h[2 * j + 1] = c[j].imag();
  }
  hipError_t e = hipMemcpyAsync(B.coef, h.data(), h.size() * sizeof(double),
                                hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = launch_multi_axpy(x, beta, V, n, (int)c.size(), B.coef, n, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(e, "Lanczos combination");
  return SG_OK;
}

sg_status taylor_step(sg_problem *p, double2 *psi, double dt, int order, sg_precision prec,
                      double2 *term, double2 *hv, hipStream_t s, void *stream) {
  const int64_t n = p->h.ncs;
  hipError_t e = hipMemcpyAsync(term, psi, n * sizeof(double2), hipMemcpyDeviceToDevice, s);
  if (e != hipSuccess) return hip_fail(e, "copy");
  for (int k = 1; k <= order; ++k) {
    sg_status st = sg_apply_H(p, term, hv, prec, stream);
    if (st != SG_OK) return st;
    // term = (-i dt / k) H term ; psi += term
    if ((e = launch_scale_accumulate(n, term, hv, make_double2(0.0, -dt / k), psi, s)) !=
        hipSuccess)
      return hip_fail(e, "Taylor update");
  }
  return SG_OK;
}

// hk: the stage vectors H y_i, contiguous; wcoef (device): -i dt b_i
sg_status rk_step(sg_problem *p, double2 *psi, double dt, const Tableau &T, sg_precision prec,
                  double2 *y, double2 *const hk[4], const double *wcoef, hipStream_t s,
                  void *stream) {
  const int64_t n = p->h.ncs;
  hipError_t e;
  for (int i = 0; i < T.s; ++i) {
    const double2 *in = psi;
    int nz = 0, jz = -1;
    for (int j = 0; j < i; ++j)
      if (T.A[i][j] != 0.0) ++nz, jz = j;
    if (nz == 1) {
      // y = psi + dt A_ij k_j,  k_j = -i H y_j  (the tableaux here have one)
      if ((e = launch_comb3(n, y, psi, make_double2(1.0, 0.0), hk[jz],
                            make_double2(0.0, -dt * T.A[i][jz]), nullptr, make_double2(0.0, 0.0),
                            s)) != hipSuccess)
        return hip_fail(e, "stage input");
      in = y;
    } else if (nz > 1) {
      if ((e = hipMemcpyAsync(y, psi, n * sizeof(double2), hipMemcpyDeviceToDevice, s)) !=
          hipSuccess)
        return hip_fail(e, "copy");
      // y += dt A_ij k_j,  k_j = -i H y_j
      for (int j = 0; j < i; ++j)
        if (T.A[i][j] != 0.0 &&
            (e = launch_axpby(n, y, hk[j], 0.0, -dt * T.A[i][j], 1.0, s)) != hipSuccess)
          return hip_fail(e, "axpby");
      in = y;
    }
    sg_status st = sg_apply_H(p, in, hk[i], prec, stream);
    if (st != SG_OK) return st;
  }
  // psi += sum_i (-i dt b_i) H y_i
  if ((e = launch_multi_axpy(psi, 1.0, hk[0], n, T.s, wcoef, n, s)) != hipSuccess)
    return hip_fail(e, "Runge-Kutta update");
  return SG_OK;
}

// w: H psi, the two midpoint iterates, H z, then the k midpoint results;
// coef (device) holds the k extrapolation weights
sg_status bs_step(sg_problem *p, double2 *psi, double dt, int k, sg_precision prec, double2 *w,
                  const double *coef, hipStream_t s, void *stream) {
  const int64_t n = p->h.ncs;
  double2 *hy = w, *zp = w + n, *z = w + 2 * n, *f = w + 3 * n, *T = w + 4 * n;
  sg_status st = sg_apply_H(p, psi, hy, prec, stream);
  if (st != SG_OK) return st;
  hipError_t e = hipSuccess;
  for (int i = 1; i <= k; ++i) {
    const int nsub = 2 * i;
    const double h = dt / nsub;
    double2 *a = zp, *b = z;   // z_{m-1}, z_m
    e = hipMemcpyAsync(a, psi, n * sizeof(double2), hipMemcpyDeviceToDevice, s);
    // z_1 = z_0 - i h H z_0
    if (e == hipSuccess)
      e = launch_comb3(n, b, psi, make_double2(1.0, 0.0), hy, make_double2(0.0, -h), nullptr,
                       make_double2(0.0, 0.0), s);
    if (e != hipSuccess) return hip_fail(e, "midpoint start");
    for (int m = 1; m < nsub; ++m) {
      if ((st = sg_apply_H(p, b, f, prec, stream)) != SG_OK) return st;
      // z_{m+1} = z_{m-1} - 2 i h H z_m, written over z_{m-1}
      if ((e = launch_axpby(n, a, f, 0.0, -2.0 * h, 1.0, s)) != hipSuccess)
        return hip_fail(e, "midpoint");
      std::swap(a, b);
    }
    if ((st = sg_apply_H(p, b, f, prec, stream)) != SG_OK) return st;
    // T_i = (z_n + z_{n-1} - i h H z_n) / 2
    double2 *Ti = T + (size_t)(i - 1) * n;
    if ((e = launch_comb3(n, Ti, b, make_double2(0.5, 0.0), a, make_double2(0.5, 0.0), f,
                          make_double2(0.0, -0.5 * h), s)) != hipSuccess)
      return hip_fail(e, "midpoint end");
  }
  if ((e = launch_multi_axpy(psi, 0.0, T, n, k, coef, n, s)) != hipSuccess)
    return hip_fail(e, "extrapolation");
  return SG_OK;
}

// V holds m + 1 vectors of n (zero-filled once); lz holds 2m + 1 doubles:
// beta0, alpha[m], beta[m - 1], a scale slot.  The Krylov vectors, their
// projections and norms stay on the device; the step reads alpha and beta
// back once.  A vector whose norm falls below 1e-13 |psi| is dropped with
// beta = 0 (it and every later vector are zero), and the host cuts T there.
// Returns the Krylov size used.
sg_status sil_step(sg_problem *p, double2 *psi, double dt, int m, sg_precision prec,
                   const Buffers &B, double *lz, hipStream_t s, void *stream, int *used) {
  const int64_t n = p->h.ncs;
  double2 *V = B.v;
  double *beta0 = lz, *alpha = lz + 1, *beta = lz + 1 + m, *scale = lz + 2 * m;
  hipError_t e = launch_dot(p, psi, psi, s);
  if (e == hipSuccess) e = launch_lanczos_norm(p->d_result, beta0, nullptr, 0.0, scale, s);
  if (e == hipSuccess) e = launch_scale_copy(V, psi, scale, n, s);
  if (e != hipSuccess) return hip_fail(e, "Lanczos start");
  sg_status st;
  for (int j = 0; j < m; ++j) {
    double2 *w = V + (size_t)(j + 1) * n;
    if ((st = sg_apply_H(p, V + (size_t)j * n, w, prec, stream)) != SG_OK) return st;
    // two projection passes; the second also sums |w|^2 for beta
    for (int pass = 0; pass < 2 && e == hipSuccess; ++pass) {
      e = launch_lanczos_project(V, n, j + 1, w, n, B.partials, B.coef, alpha + j, pass > 0, s);
      if (e != hipSuccess) break;
      if (pass == 0 || j == m - 1)
        e = launch_multi_axpy(w, 1.0, V, n, j + 1, B.coef, n, s);
      else
        e = launch_multi_axpy_norm(w, V, n, j + 1, B.coef, n, B.npart, s);
    }
    if (e == hipSuccess && j < m - 1) {
      e = launch_lanczos_norm_partials(B.npart, n, beta + j, beta0, 1e-13, scale, s);
      if (e == hipSuccess) e = launch_scale_copy(w, w, scale, n, s);
    }
    if (e != hipSuccess) return hip_fail(e, "Lanczos step");
  }
  std::vector<double> h(2 * (size_t)m);
  e = hipMemcpyAsync(h.data(), lz, (2 * (size_t)m) * sizeof(double), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(e, "read Lanczos coefficients");
  const double b0 = h[0];
  *used = 0;
  if (!(b0 > 0.0)) return SG_OK;  // the zero state stays zero
  int k = m;
  for (int j = 0; j + 1 < m; ++j)
    if (h[1 + m + j] == 0.0) {
      k = j + 1;
      break;
    }
  std::vector<double> T((size_t)k * k, 0.0), ev, U;
  for (int i = 0; i < k; ++i) {
    T[(size_t)i * k + i] = h[1 + i];
    if (i + 1 < k) T[(size_t)i * k + i + 1] = T[(size_t)(i + 1) * k + i] = h[1 + m + i];
  }
  jacobi_eigen(T, k, &ev, &U);
  // coefficients of psi(t + dt) in V: beta0 U exp(-i ev dt) U^T e_1
  // (U row-major, eigenvectors in columns)
  std::vector<std::complex<double>> coef(k, 0.0);
  for (int q = 0; q < k; ++q) {
    const std::complex<double> ph = std::polar(1.0, -ev[q] * dt) * (b0 * U[(size_t)0 * k + q]);
    for (int i = 0; i < k; ++i) coef[i] += U[(size_t)i * k + q] * ph;
  }
  if ((st = combine(B, psi, 0.0, V, n, coef, s)) != SG_OK) return st;
  *used = k;
  return SG_OK;
}

}  // namespace

namespace sg {

PropBuffers::~PropBuffers() {
  if (!owned) return;
  hipFree(v);
  hipFree(npart);
  hipFree(lz);
  hipFree(partials);
  hipFree(coef);
}

// Checks the arguments of a propagation and sizes its work buffers: m (the
// Krylov dimension used) and nvec (work vectors besides the check vector).
sg_status propagate_check(sg_problem *p, void *psi_v, double dt, int32_t nsteps, int32_t method,
                          int32_t order, sg_precision prec, int32_t check_every, int *m_out,
                          int *nvec_out) {
  if (!p || !psi_v) return fail(SG_EINVAL, "NULL argument");
  if (!(dt > 0.0) || !std::isfinite(dt) || nsteps < 0 || check_every < 0)
    return fail(SG_EINVAL, "dt must be > 0, nsteps and check_every >= 0");
  if (prec != SG_FP64 && prec != SG_MIXED) return fail(SG_EINVAL, "unknown precision");
  if (method == SG_PROP_TAYLOR) {
    if (order < 1 || order > kMaxTaylorOrder) return fail(SG_EINVAL, "Taylor order must be 1..40");
  } else if (method == SG_PROP_RK) {
    if (order < 1 || order > 4) return fail(SG_EINVAL, "Runge-Kutta order must be 1..4");
  } else if (method == SG_PROP_SIL) {
    if (order < 1 || order > kMaxKrylov) return fail(SG_EINVAL, "Krylov dimension must be 1..64");
  } else if (method == SG_PROP_BS) {
    if (order < 1 || order > kMaxColumns) return fail(SG_EINVAL, "Bulirsch-Stoer columns must be 1..8");
  } else {
    return fail(SG_EINVAL, "unknown propagator");
  }
  if (p->host_only) return fail(SG_EINVAL, "handle was built without device tables");
  const int64_t n = p->h.ncs;
  const int m = method == SG_PROP_SIL ? (int)std::min<int64_t>(order, n) : 0;
  // work vectors: Taylor 2, Runge-Kutta 1 + stages, Lanczos m + 1,
  // Bulirsch-Stoer 4 + columns; one more for the checks
  *m_out = m;
  *nvec_out = method == SG_PROP_TAYLOR ? 2
              : method == SG_PROP_RK   ? 1 + order
              : method == SG_PROP_BS   ? 4 + order
                                       : m + 1;
  return SG_OK;
}

// Byte offsets of the work buffers inside one region (each 256-byte
// aligned): v, partials, coef, lz, npart; returns the region's size.
int64_t propagate_layout(int64_t n, int32_t method, int32_t order, int m, int nvec,
                         int64_t off[5]) {
  auto up = [](int64_t b) { return (b + 255) & ~(int64_t)255; };
  int64_t sz[5] = {(int64_t)(nvec + 1) * n * (int64_t)sizeof(double2), 0, 0, 0, 0};
  if (method == SG_PROP_SIL) {
    const int64_t mm = (int64_t)m + 1;
    sz[1] = 2 * mm * dot_partials_per_vector() * (int64_t)sizeof(double);
    sz[2] = 2 * mm * (int64_t)sizeof(double);
    sz[3] = (2 * mm + 1) * (int64_t)sizeof(double);
    sz[4] = (int64_t)lanczos_norm_partials() * (int64_t)sizeof(double);
  } else if (method == SG_PROP_BS || method == SG_PROP_RK) {
    sz[2] = 2 * (int64_t)order * (int64_t)sizeof(double);
  }
  int64_t at = 0;
  for (int i = 0; i < 5; ++i) {
    off[i] = at;
    at += up(sz[i]);
  }
  return at;
}

// The propagation itself, on work buffers B (sized by propagate_layout).
// zero_kernel: clear the work vectors with a fill kernel instead of
// hipMemsetAsync.
sg_status propagate_run(sg_problem *p, void *psi_v, double dt, int32_t nsteps, int32_t method,
                        int32_t order, int m, int nvec, double tol, sg_precision prec,
                        int32_t check_every, sg_prop_stats *stats, double *norm_trace,
                        double *energy_trace, void *stream, PropBuffers &B, bool zero_kernel) {
  hipStream_t s = (hipStream_t)stream;
  double2 *psi = (double2 *)psi_v;
  const int64_t n = p->h.ncs;
  hipError_t e = hipSuccess;
  std::vector<double> wts(2 * (size_t)std::max(order, 1), 0.0);
  if (method == SG_PROP_BS) {
    // extrapolation to h = 0 of the midpoint results at h_i = dt / (2i):
    // Lagrange weights in x = h^2, prod_{j != i} x_j / (x_j - x_i)
    for (int i = 1; i <= order; ++i) {
      double c = 1.0;
      for (int j = 1; j <= order; ++j)
        if (j != i) c *= (double)(i * i) / (double)(i * i - j * j);
      wts[2 * (i - 1)] = c;
    }
    if ((e = hipMemcpyAsync(B.coef, wts.data(), wts.size() * sizeof(double),
                            hipMemcpyHostToDevice, s)) != hipSuccess)
      return hip_fail(e, "upload extrapolation weights");
  } else if (method == SG_PROP_RK) {
    // Runge-Kutta weights as coefficients of H y_i: -i dt b_i
    for (int i = 0; i < order; ++i) {
      wts[2 * i] = 0.0;
      wts[2 * i + 1] = -dt * kRK[order - 1].b[i];
    }
    if ((e = hipMemcpyAsync(B.coef, wts.data(), wts.size() * sizeof(double),
                            hipMemcpyHostToDevice, s)) != hipSuccess)
      return hip_fail(e, "upload Runge-Kutta weights");
  }
  // zero-filled: vector updates read their destination
  e = zero_kernel ? launch_zero(B.v, (int64_t)(nvec + 1) * n, s)
                  : hipMemsetAsync(B.v, 0, (size_t)(nvec + 1) * n * sizeof(double2), s);
  if (e != hipSuccess) return hip_fail(e, "clear work vectors");
  double2 *check_buf = B.v + (size_t)nvec * n;

  sg_prop_stats st{};
  st.cheb_terms = order;
  st.emin = st.emax = std::nan("");
  int ntrace = 0;
  bool have0 = false;
  sg_status ret = SG_OK;
  auto check = [&]() -> sg_status {
    sg_status as = sg_apply_H(p, psi, check_buf, prec, stream);
    if (as != SG_OK) return as;
    double nr, ni, er, ei;
    if ((e = launch_dot(p, psi, psi, s)) != hipSuccess) return hip_fail(e, "dot");
    if ((as = read2(p, s, &nr, &ni)) != SG_OK) return as;
    if ((e = launch_dot(p, psi, check_buf, s)) != hipSuccess) return hip_fail(e, "dot");
    if ((as = read2(p, s, &er, &ei)) != SG_OK) return as;
    st.applies += 1;
    const double nrm = std::sqrt(nr), E = nr > 0.0 ? er / nr : 0.0;
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
    if (tol > 0.0 && std::fabs(nrm - st.norm0) > tol) ret = SG_ETOL;
    return SG_OK;
  };
  double2 *hk[4] = {nullptr, nullptr, nullptr, nullptr};
  for (int i = 0; i < 4 && method == SG_PROP_RK && i < order; ++i) hk[i] = B.v + (size_t)(1 + i) * n;
  sg_status rs = SG_OK;
  for (int step = 0; step < nsteps && ret == SG_OK; ++step) {
    if ((step == 0 || (check_every > 0 && step % check_every == 0)) && (rs = check()) != SG_OK)
      return rs;
    if (ret != SG_OK) break;
    if (method == SG_PROP_TAYLOR) {
      rs = taylor_step(p, psi, dt, order, prec, B.v, B.v + n, s, stream);
      st.applies += order;
    } else if (method == SG_PROP_RK) {
      rs = rk_step(p, psi, dt, kRK[order - 1], prec, B.v, hk, B.coef, s, stream);
      st.applies += order;
    } else if (method == SG_PROP_BS) {
      rs = bs_step(p, psi, dt, order, prec, B.v, B.coef, s, stream);
      st.applies += 1 + order * (order + 1);
    } else {
      int used = 0;   // every step applies H m times, dropped vectors included
      rs = sil_step(p, psi, dt, m, prec, B, B.lz, s, stream, &used);
      st.applies += m;
    }
    if (rs != SG_OK) return rs;
    st.steps_done = step + 1;
  }
  if (ret == SG_OK && (rs = check()) != SG_OK) return rs;
  if ((e = hipStreamSynchronize(s)) != hipSuccess) return hip_fail(e, "propagation");
  if (stats) *stats = st;
  if (ret == SG_ETOL) return fail(SG_ETOL, "norm drift beyond tolerance");
  return SG_OK;
}


}  // namespace sg

extern "C" {

sg_status sg_propagate(sg_problem *p, void *psi_v, double dt, int32_t nsteps, int32_t method,
                       int32_t order, double tol, sg_precision prec, int32_t check_every,
                       sg_prop_stats *stats, double *norm_trace, double *energy_trace,
                       void *stream) {
  int m = 0, nvec = 0;
  sg_status cs = propagate_check(p, psi_v, dt, nsteps, method, order, prec, check_every, &m, &nvec);
  if (cs != SG_OK) return cs;
  const int64_t n = p->h.ncs;
  int64_t off[5];
  propagate_layout(n, method, order, m, nvec, off);
  PropBuffers B;
  hipError_t e = hipMalloc((void **)&B.v, (size_t)(nvec + 1) * n * sizeof(double2));
  if (e == hipSuccess && method == SG_PROP_SIL) {
    const size_t mm = (size_t)m + 1;
    e = hipMalloc((void **)&B.partials, 2 * mm * dot_partials_per_vector() * sizeof(double));
    if (e == hipSuccess) e = hipMalloc((void **)&B.coef, 2 * mm * sizeof(double));
    if (e == hipSuccess) e = hipMalloc((void **)&B.lz, (2 * mm + 1) * sizeof(double));
    if (e == hipSuccess)
      e = hipMalloc((void **)&B.npart, (size_t)lanczos_norm_partials() * sizeof(double));
  }
  if (e == hipSuccess && (method == SG_PROP_BS || method == SG_PROP_RK))
    e = hipMalloc((void **)&B.coef, 2 * (size_t)order * sizeof(double));
  if (e != hipSuccess) return fail(SG_ENOMEM, "propagator work vectors");
  return propagate_run(p, psi_v, dt, nsteps, method, order, m, nvec, tol, prec, check_every,
                       stats, norm_trace, energy_trace, stream, B, false);
}

}  // extern "C"
