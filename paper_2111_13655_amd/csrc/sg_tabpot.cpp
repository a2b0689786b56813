// General coupling potentials V(Q), tabulated per Smolyak term.
//
// Alg. 1 (Sec. 3) applies the operator on each term's direct-product grid.
// With the separable harmonic part split off as the exact diagonal, what a
// term needs of a general V is, per active grid point, the sum over the
// points of its level-0 modes of V times their weights wt_u b_0(Q_u)^2: a
// level-0 mode has one basis function, so its basis -> grid pass multiplies by
// b_0(Q_u) and its grid -> basis pass by wt_u b_0(Q_u).  sg_set_potential
// evaluates the caller's V on every term's literal grid (host, batched),
// forms these per-term tables V_eff,l and uploads them; the problem's term
// sweep then multiplies each grid value by V_eff read along its fiber instead
// of forming the polynomial couplings (the kernel's tabulated instantiation).
#include <algorithm>
#include <cmath>
#include <new>
#include <vector>

#include "sg_internal.h"

namespace sg {

namespace {

constexpr int64_t kBatch = 65536;            // points per call of the caller's V
constexpr double kMaxPoints = 1e11;          // literal grid points evaluated at most

// V_eff of every term on its active grid, mode 0 of the term record fastest
// (the layout of the sweep's grid buffer), from the caller's V.
sg_status tabulate(const Compiled &h, const std::vector<double> &tb, sg_potential_fn fn,
                   void *user, std::vector<double> *veff, std::vector<int64_t> *voff) {
  const int D = h.D;
  const int64_t nt = h.nterms;
  // level-0 points and weights wt_u b_0(Q_u)^2 (standard layout at level 0:
  // b (nq x 1), wt b^T (1 x nq), nodes)
  const int nq0 = h.nqA;
  std::vector<double> x0(nq0), w0(nq0);
  for (int u = 0; u < nq0; ++u) {
    x0[u] = tb[std_table_base(0) + 2 * nq0 + u];
    w0[u] = tb[std_table_base(0) + nq0 + u] * tb[std_table_base(0) + u];
  }
  voff->assign(nt, 0);
  int64_t total = 0;
  for (int64_t t = 0; t < nt; ++t) {
    (*voff)[t] = total;
    total += h.terms[t].ngrid;
  }
  veff->assign(total, 0.0);
  std::vector<double> Q((size_t)kBatch * D), V(kBatch);
  std::vector<int32_t> zero_modes;
  std::vector<char> active(D);
  for (int64_t t = 0; t < nt; ++t) {
    const TermDev &T = h.terms[t];
    const int na = T.na;
    std::fill(active.begin(), active.end(), 0);
    for (int p = 0; p < na; ++p) active[T.mode[p]] = 1;
    zero_modes.clear();
    for (int m = 0; m < D; ++m)
      if (!active[m]) zero_modes.push_back(m);
    const int n0 = (int)zero_modes.size();
    int64_t ncomb = 1;
    for (int i = 0; i < n0; ++i) ncomb *= nq0;
    const int64_t ngrid = T.ngrid, npts = ngrid * ncomb;
    double *out = veff->data() + (*voff)[t];
    // point q = g ncomb + c: active grid point g, level-0 combination c
    // (level-0 mode i's point: digit i of c in base nq0)
    for (int64_t q0 = 0; q0 < npts; q0 += kBatch) {
      const int64_t nb = std::min(kBatch, npts - q0);
      for (int64_t j = 0; j < nb; ++j) {
        const int64_t q = q0 + j;
        int64_t g = q / ncomb, c = q - g * ncomb;
        double *row = Q.data() + (size_t)j * D;
        for (int p = 0; p < na; ++p) {
          const int l = T.lev[p], nq = T.nq[p];
          const int64_t i = g % nq;
          g /= nq;
          row[T.mode[p]] = tb[std_table_base(l) + 2 * T.nb[p] * nq + i];
        }
        for (int i = 0; i < n0; ++i) {
          row[zero_modes[i]] = x0[c % nq0];
          c /= nq0;
        }
      }
      fn(nb, Q.data(), V.data(), user);
      for (int64_t j = 0; j < nb; ++j) {
        if (!std::isfinite(V[j])) return fail(SG_EINVAL, "the potential returned a non-finite value");
        const int64_t q = q0 + j;
        const int64_t g = q / ncomb;
        int64_t c = q - g * ncomb;
        double w = 1.0;
        for (int i = 0; i < n0; ++i) {
          w *= w0[c % nq0];
          c /= nq0;
        }
        out[g] += w * V[j];
      }
    }
  }
  return SG_OK;
}

}  // namespace
}  // namespace sg

using namespace sg;

extern "C" sg_status sg_set_potential(sg_problem *p, sg_potential_fn fn, void *user) {
  if (!p) return fail(SG_EINVAL, "NULL problem");
  if (p->host_only) return fail(SG_EINVAL, "handle was built without device tables");
  if (!fn) {
    if (p->d_veff) {
      hipError_t e = hipDeviceSynchronize();
      if (e != hipSuccess) return hip_fail(e, "synchronize");
      hipFree(p->d_veff);
      hipFree(p->d_voff);
      p->d_veff = nullptr;
      p->d_voff = nullptr;
      return problem_replan(p);
    }
    return SG_OK;
  }
  const Compiled &h = p->h;
  if (!(h.nbA == 1 && h.nbB == 2 && h.nqA == 2 && h.nqB == 2))
    return fail(SG_EINVAL, "a tabulated potential needs the standard size maps");
  if (h.L > 6) return fail(SG_EINVAL, "a tabulated potential takes L <= 6");
  if (!p->plan || !p->plan->fp64_split || p->grid_kinetic)
    return fail(SG_EINVAL, "a tabulated potential needs the split operator form");
  if (!p->plan->sets[kSetSplit64].all_inplace)
    return fail(SG_EINVAL, "a tabulated potential needs every term in place");
  if (p->plan->stab_L < h.L) return fail(SG_EINVAL, "standard-map tables missing");
  if ((double)h.grid_literal > kMaxPoints)
    return fail(SG_EINVAL, "more than 1e11 grid points to evaluate");
  std::vector<double> veff;
  std::vector<int64_t> voff;
  sg_status st = tabulate(h, p->plan->stab64, fn, user, &veff, &voff);
  if (st != SG_OK) return st;
  double *dv = nullptr;
  int64_t *doff = nullptr;
  hipError_t e = hipMalloc((void **)&dv, std::max<size_t>(1, veff.size()) * sizeof(double));
  if (e == hipSuccess) e = hipMalloc((void **)&doff, voff.size() * sizeof(int64_t));
  if (e != hipSuccess) {
    hipFree(dv);
    hipFree(doff);
    return fail(SG_ENOMEM, "device allocation failed");
  }
  e = hipMemcpy(dv, veff.data(), veff.size() * sizeof(double), hipMemcpyHostToDevice);
  if (e == hipSuccess)
    e = hipMemcpy(doff, voff.data(), voff.size() * sizeof(int64_t), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e != hipSuccess) {
    hipFree(dv);
    hipFree(doff);
    return hip_fail(e, "upload potential tables");
  }
  double *old_v = p->d_veff;
  int64_t *old_off = p->d_voff;
  p->d_veff = dv;
  p->d_voff = doff;
  st = problem_replan(p);   // synchronises before it replaces the plan
  if (st != SG_OK) {
    p->d_veff = old_v;
    p->d_voff = old_off;
    hipFree(dv);
    hipFree(doff);
    problem_replan(p);
    return st;
  }
  hipFree(old_v);
  hipFree(old_off);
  return SG_OK;
}
