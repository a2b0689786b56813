// Lowest eigenpairs of the Smolyak operator by block Davidson (the method the
// paper converges stationary states with, Sec. 3 flowchart text), on the
// operator action sg_apply_H, and the embedding of a level-L' state into the
// nested level-L compact basis that seeds a run from a lower-level solution
// (the paper's Sec. 4 example: a guess from a low-L diagonalization, then
// Davidson at the target level).
//
// H_S is real symmetric; starting vectors are real, so every vector stays
// real (stored as complex128 with zero imaginary parts) and the projected
// matrices are real.  Vector operations run in the library's kernels; only
// the small projected eigenproblem is solved on the host.
#include <algorithm>
#include <cmath>
#include <numeric>
#include <vector>

#include "sg_internal.h"

using namespace sg;

namespace {

struct Work {
  double2 *V = nullptr, *W = nullptr, *X = nullptr, *HX = nullptr;
  double *partials = nullptr, *dots = nullptr, *coef = nullptr;
  ~Work() {
    hipFree(V);
    hipFree(W);
    hipFree(X);
    hipFree(HX);
    hipFree(partials);
    hipFree(dots);
    hipFree(coef);
  }
};

// conj(V_j)^T w for j < m, real parts, on the host (synchronises s)
hipError_t dots(const Work &w, const double2 *V, int64_t n, int m, const double2 *x,
                std::vector<double> *out, hipStream_t s) {
  out->assign(m, 0.0);
  if (m == 0) return hipSuccess;
  std::vector<double> h(2 * (size_t)m);
  hipError_t e = launch_multi_dot(V, n, m, x, n, w.partials, w.dots, s);
  if (e == hipSuccess)
    e = hipMemcpyAsync(h.data(), w.dots, h.size() * sizeof(double), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  for (int j = 0; j < m; ++j) (*out)[j] = h[2 * j];
  return e;
}

// x = beta x + sum_j c_j V_j  (real c)
hipError_t combine(const Work &w, double2 *x, double beta, const double2 *V, int64_t n,
                   const std::vector<double> &c, hipStream_t s) {
  std::vector<double> h(2 * c.size(), 0.0);
  for (size_t j = 0; j < c.size(); ++j) h[2 * j] = c[j];
  hipError_t e = hipSuccess;
  if (!c.empty())
    e = hipMemcpyAsync(w.coef, h.data(), h.size() * sizeof(double), hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = launch_multi_axpy(x, beta, V, n, (int)c.size(), w.coef, n, s);
  // the coefficient buffer is reused by the next call: keep the order
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  return e;
}

// Orthonormalises x against V_0..V_{m-1} (two classical Gram-Schmidt passes)
// and normalises it; returns its norm after the projections.
hipError_t orthonormalise(const Work &w, double2 *x, const double2 *V, int64_t n, int m,
                          double *norm, hipStream_t s) {
  std::vector<double> c;
  hipError_t e = hipSuccess;
  for (int pass = 0; pass < 2 && e == hipSuccess && m > 0; ++pass) {
    e = dots(w, V, n, m, x, &c, s);
    for (double &v : c) v = -v;
    if (e == hipSuccess) e = combine(w, x, 1.0, V, n, c, s);
  }
  std::vector<double> nn;
  if (e == hipSuccess) e = dots(w, x, n, 1, x, &nn, s);
  *norm = e == hipSuccess ? std::sqrt(std::max(nn[0], 0.0)) : 0.0;
  if (e == hipSuccess && *norm > 0.0) e = combine(w, x, 1.0 / *norm, V, n, {}, s);
  return e;
}

}  // namespace

extern "C" {

sg_status sg_eigensolve(sg_problem *p, int32_t nev, int32_t max_basis, int32_t max_iter,
                        double tol, const void *guess, int32_t nguess, double *evals,
                        void *evecs, double *resnorms, sg_eig_stats *stats, void *stream) {
  if (!p || !evals) return fail(SG_EINVAL, "NULL argument");
  if (p->host_only) return fail(SG_EINVAL, "handle was built without device tables");
  const int64_t n = p->h.ncs;
  if (nev < 1 || nev > n) return fail(SG_EINVAL, "need 1 <= nev <= N_cs");
  if (max_basis < 2 * nev || max_basis > 256) return fail(SG_EINVAL, "need 2 nev <= max_basis <= 256");
  if (max_basis > n) max_basis = (int32_t)n;
  if (max_iter < 1 || !(tol > 0.0)) return fail(SG_EINVAL, "need max_iter >= 1 and tol > 0");
  if (nguess < 0 || (nguess > 0 && !guess)) return fail(SG_EINVAL, "bad guess block");
  hipStream_t s = (hipStream_t)stream;
  const int mb = max_basis;
  // Ritz pairs iterated: nev plus as many buffer pairs (corrections for them
  // too), so that a start block with little weight on some wanted state
  // still draws it in before the first nev converge
  const int nblk = std::min<int>(2 * nev, mb / 2);
  const size_t vb = (size_t)n * sizeof(double2);
  Work w;
  hipError_t e = hipMalloc((void **)&w.V, vb * mb);
  if (e == hipSuccess) e = hipMalloc((void **)&w.W, vb * mb);
  if (e == hipSuccess) e = hipMalloc((void **)&w.X, vb * nblk);
  if (e == hipSuccess) e = hipMalloc((void **)&w.HX, vb * nblk);
  if (e == hipSuccess)
    e = hipMalloc((void **)&w.partials, sizeof(double) * 2 * dot_partials_per_vector() * mb);
  if (e == hipSuccess) e = hipMalloc((void **)&w.dots, sizeof(double) * 2 * mb);
  if (e == hipSuccess) e = hipMalloc((void **)&w.coef, sizeof(double) * 2 * mb);
  if (e != hipSuccess) return fail(SG_ENOMEM, "eigensolver workspace allocation failed");
  auto Vc = [&](int j) { return w.V + (size_t)j * n; };
  auto Wc = [&](int j) { return w.W + (size_t)j * n; };

  // starting block: the guess (if any), then unit vectors at the nev lowest
  // diagonal entries of the separable part; vectors that the earlier ones
  // already span are dropped.  The unit vectors keep low-energy directions
  // that a lower-level guess lacks in the subspace.
  int m = 0;
  const int ng = nguess > 0 ? std::min<int>(nguess, mb - 2 * nev) : 0;
  for (int j = 0; j < ng && e == hipSuccess; ++j) {
    double nrm = 0.0;
    e = hipMemcpyAsync(Vc(m), (const double2 *)guess + (size_t)j * n, vb, hipMemcpyDeviceToDevice,
                       s);
    if (e == hipSuccess) e = orthonormalise(w, Vc(m), w.V, n, m, &nrm, s);
    if (e == hipSuccess && nrm > 1e-10) ++m;
  }
  {
    std::vector<int64_t> idx(n);
    std::iota(idx.begin(), idx.end(), 0);
    std::partial_sort(idx.begin(), idx.begin() + nev, idx.end(), [&](int64_t a, int64_t b) {
      return p->h.h0[a] < p->h.h0[b] || (p->h.h0[a] == p->h.h0[b] && a < b);
    });
    const double2 one = make_double2(1.0, 0.0);
    for (int j = 0; j < nev && e == hipSuccess && m < mb - nev; ++j) {
      double nrm = 0.0;
      e = launch_zero(Vc(m), n, s);
      if (e == hipSuccess)
        e = hipMemcpyAsync(Vc(m) + idx[j], &one, sizeof(double2), hipMemcpyHostToDevice, s);
      if (e == hipSuccess) e = hipStreamSynchronize(s);
      if (e == hipSuccess) e = orthonormalise(w, Vc(m), w.V, n, m, &nrm, s);
      if (e == hipSuccess && nrm > 1e-10) ++m;
    }
  }
  // one deterministic pseudo-random vector: symmetries of H (e.g. parity in
  // a mode that only appears squared) leave the unit vectors above in a
  // subset of the invariant subspaces; this vector has weight in all of them
  if (e == hipSuccess && m < mb - nev) {
    std::vector<double2> r(n);
    uint64_t x = 0x9e3779b97f4a7c15ull;
    for (int64_t i = 0; i < n; ++i) {
      x ^= x << 13;
      x ^= x >> 7;
      x ^= x << 17;
      r[i] = make_double2((double)(x >> 11) * 0x1.0p-53 - 0.5, 0.0);
    }
    double nrm = 0.0;
    e = hipMemcpyAsync(Vc(m), r.data(), vb, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e == hipSuccess) e = orthonormalise(w, Vc(m), w.V, n, m, &nrm, s);
    if (e == hipSuccess && nrm > 1e-10) ++m;
  }
  if (e != hipSuccess) return hip_fail(e, "eigensolver start");
  if (m < nev) return fail(SG_EINVAL, "starting block has fewer than nev independent vectors");

  std::vector<double> G((size_t)mb * mb, 0.0), theta, Y, res(nblk, 0.0);
  int have_w = 0;   // columns of W computed
  sg_eig_stats st{};
  for (int it = 0; it < max_iter; ++it) {
    st.iterations = it + 1;
    // W = H V for the new columns, and the new entries of G = V^T H V
    for (int j = have_w; j < m; ++j) {
      sg_status r = sg_apply_H(p, Vc(j), Wc(j), SG_FP64, stream);
      if (r != SG_OK) return r;
      st.applies++;
      std::vector<double> col;
      if ((e = dots(w, w.V, n, j + 1, Wc(j), &col, s)) != hipSuccess)
        return hip_fail(e, "projection");
      for (int i = 0; i <= j; ++i) G[(size_t)i * mb + j] = G[(size_t)j * mb + i] = col[i];
    }
    have_w = m;
    // Rayleigh-Ritz
    std::vector<double> Gm((size_t)m * m);
    for (int i = 0; i < m; ++i)
      for (int j = 0; j < m; ++j) Gm[(size_t)i * m + j] = G[(size_t)i * mb + j];
    jacobi_eigen(Gm, m, &theta, &Y);
    auto ycol = [&](int k) {
      std::vector<double> c(m);
      for (int i = 0; i < m; ++i) c[i] = Y[(size_t)i * m + k];
      return c;
    };
    // Ritz vectors, their images and residual norms
    st.converged = 0;
    const int nk = std::min(nblk, m);
    for (int k = 0; k < nk; ++k) {
      const std::vector<double> c = ycol(k);
      double2 *x = w.X + (size_t)k * n, *hx = w.HX + (size_t)k * n;
      if ((e = combine(w, x, 0.0, w.V, n, c, s)) != hipSuccess) return hip_fail(e, "ritz");
      if ((e = combine(w, hx, 0.0, w.W, n, c, s)) != hipSuccess) return hip_fail(e, "ritz");
      // residual r = H x - theta x, kept in hx
      if ((e = combine(w, hx, 1.0, x, n, {-theta[k]}, s)) != hipSuccess)
        return hip_fail(e, "residual");
      std::vector<double> nn;
      if ((e = dots(w, hx, n, 1, hx, &nn, s)) != hipSuccess) return hip_fail(e, "residual");
      res[k] = std::sqrt(std::max(nn[0], 0.0));
      if (k < nev && res[k] <= tol) st.converged++;
    }
    if (st.converged == nev) break;
    // restart: keep the Ritz block
    if (m + nk > mb) {
      for (int k = 0; k < nk; ++k) {
        double2 *x = w.X + (size_t)k * n;
        if ((e = hipMemcpyAsync(Vc(k), x, vb, hipMemcpyDeviceToDevice, s)) != hipSuccess)
          return hip_fail(e, "restart");
      }
      // images of the kept vectors: H x = residual + theta x
      for (int k = 0; k < nk; ++k) {
        double2 *hx = w.HX + (size_t)k * n;
        if ((e = hipMemcpyAsync(Wc(k), hx, vb, hipMemcpyDeviceToDevice, s)) != hipSuccess)
          return hip_fail(e, "restart");
        if ((e = combine(w, Wc(k), 1.0, Vc(k), n, {theta[k]}, s)) != hipSuccess)
          return hip_fail(e, "restart");
      }
      std::fill(G.begin(), G.end(), 0.0);
      for (int k = 0; k < nk; ++k) G[(size_t)k * mb + k] = theta[k];
      m = have_w = nk;
      st.restarts++;
    }
    // Davidson corrections for the unconverged pairs
    int added = 0;
    for (int k = 0; k < nk && m < mb; ++k) {
      if (res[k] <= tol) continue;
      if ((e = launch_precondition(Vc(m), w.HX + (size_t)k * n, p->d_h0, theta[k], n, s)) !=
          hipSuccess)
        return hip_fail(e, "correction");
      double nrm = 0.0;
      if ((e = orthonormalise(w, Vc(m), w.V, n, m, &nrm, s)) != hipSuccess)
        return hip_fail(e, "correction");
      if (nrm > 1e-12) {
        ++m;
        ++added;
      }
    }
    if (added == 0) break;
  }
  for (int k = 0; k < nev; ++k) {
    evals[k] = theta[k];
    if (resnorms) resnorms[k] = res[k];
  }
  if (evecs) {
    e = hipMemcpyAsync(evecs, w.X, vb * nev, hipMemcpyDeviceToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "eigenvector copy");
  }
  if (stats) *stats = st;
  if (st.converged < nev) return fail(SG_ETOL, "Davidson did not converge every eigenpair");
  return SG_OK;
}

sg_status sg_embed_basis(const sg_problem *from, const sg_problem *to, const void *x, void *y,
                         void *stream) {
  if (!from || !to || !x || !y) return fail(SG_EINVAL, "NULL argument");
  if (from->host_only || to->host_only) return fail(SG_EINVAL, "handles need device tables");
  const Compiled &a = from->h, &b = to->h;
  if (a.D != b.D || a.nbA != b.nbA || a.nbB != b.nbB || a.L > b.L)
    return fail(SG_EINVAL, "bases are not nested (same D and basis map, from L <= to L)");
  const int D = a.D;
  // both compact lists are lexicographic; walk them together
  std::vector<int32_t> map(a.ncs);
  int64_t j = 0;
  for (int64_t i = 0; i < a.ncs; ++i) {
    const uint8_t *u = &a.compact[(size_t)i * D];
    while (j < b.ncs && !std::equal(u, u + D, &b.compact[(size_t)j * D])) ++j;
    if (j == b.ncs) return fail(SG_EINVAL, "basis of the lower level is not contained");
    map[i] = (int32_t)j++;
  }
  hipStream_t s = (hipStream_t)stream;
  int32_t *dmap = nullptr;
  hipError_t e = hipMalloc((void **)&dmap, map.size() * sizeof(int32_t));
  if (e != hipSuccess) return fail(SG_ENOMEM, "embedding map allocation failed");
  e = hipMemcpyAsync(dmap, map.data(), map.size() * sizeof(int32_t), hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = launch_embed((const double2 *)x, dmap, a.ncs, (double2 *)y, b.ncs, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  hipFree(dmap);
  if (e != hipSuccess) return hip_fail(e, "embedding");
  return SG_OK;
}

}  // extern "C"
