// Term sweep of a Smolyak operator whose coupling potential is a general
// function V(Q), tabulated per term.
//
// Alg. 1 applies the potential on each term's direct-product grid.  Modes
// at level 0 carry one basis function, and their basis -> grid -> basis
// passes reduce to a weighted sum over their grid points, so each term needs
// V only on the grid of its active modes, averaged with those weights over
// the level-0 points: V_eff,l (built on the host from the caller's V, one
// FP64 value per active grid point, streamed from HBM).  The separable
// harmonic part acts as the exact FP64 diagonal in the reduce, as in the
// polynomial split form.  One term per workgroup (sg_term_group.h); the
// potential step multiplies each grid value by V_eff read along the fiber.
#include "sg_term_group.h"

namespace sg {

namespace {

using namespace grp;

struct TabArgs {
  const TermDev *terms;
  const int32_t *mb;        // M^B, term-major (device order)
  const double *tab;        // standard-map tables (b, wt b^T, nodes per level)
  const double *veff;       // V_eff of all terms, term t's from voff[t]
  const int64_t *voff;      // [nterms]
  const int32_t *order;     // the terms of this launch
  const double2 *vin;       // [N_cs]: the vector H acts on
  double2 *tm;              // [N_s]
  int tab_elems;            // doubles of the table layout in LDS
};

// V_eff along the mode-0 fibers of a term: the term's grid is laid out with
// mode 0 fastest, so fiber f holds points f nq0 .. f nq0 + nq0 - 1.
struct TabPot {
  glb_p<const double> v;
  int nq0;
  using Fiber = glb_p<const double>;
  __device__ __forceinline__ Fiber fiber(int f) const { return v + (int64_t)f * nq0; }
  __device__ __forceinline__ void point(const Fiber &w, int u, const Z (&g)[1], Z (&y)[1]) const {
    const double x = w[u];
    y[0] = Z{x * g[0].x, x * g[0].y};
  }
};

template <int VT, int MAXG, int MAXLEV>
__global__ __launch_bounds__(VT) void tab_sweep_kernel(TabArgs a) {
  extern __shared__ char lds_raw[];
  const int t = a.order[blockIdx.x];
  // read in place: a copy with dynamically indexed arrays would live in scratch
  const TermDev &T = a.terms[t];
  lds_p<double> tab = (lds_p<double>)lds_raw;
  const Bufs<1> B{{(lds_p<Z>)(tab + a.tab_elems)}};
  const int off = T.off;
  copy_tables<VT>(T, tab, a.tab);
  __syncthreads();
  const glb_p<Z> tout[1] = {(glb_p<Z>)a.tm + off};
  const glb_p<const Z> vin[1] = {(glb_p<const Z>)a.vin};
  const glb_p<const double> V = (glb_p<const double>)a.veff + a.voff[t];
  if (T.na == 0) {   // a scalar term: V averaged over the level-0 points
    if (threadIdx.x == 0) {
      const Z x = ldz(vin[0] + a.mb[off]);
      const double w = T.coeff * V[0];
      stz(tout[0], w * x.x, w * x.y);
    }
    return;
  }
  const TabPot pot{V, T.nq[0]};
  run_term<1, VT, MAXG, MAXLEV>(T, tab, B, vin, (glb_p<const int32_t>)a.mb + off, pot, tout);
}

template <int S>
constexpr auto tab_kernel() {
  return &tab_sweep_kernel<kGroupShape[S].vt, kGroupShape[S].max_grid, kGroupShape[S].max_level>;
}

}  // namespace

hipError_t launch_tab_sweep(const TabLaunch &v, const double2 *vin, double2 *tm, hipStream_t s,
                            hipEvent_t ev0, hipEvent_t ev1) {
  static_assert(kGroupShapes == 3, "one kernel per shape");
  static const void *const kernels[kGroupShapes] = {
      (const void *)tab_kernel<0>(), (const void *)tab_kernel<1>(), (const void *)tab_kernel<2>()};
  static bool attr_set = false;
  if (!attr_set) {
    for (int k = 0; k < kGroupShapes; ++k) {
      hipError_t e = hipFuncSetAttribute(kernels[k], hipFuncAttributeMaxDynamicSharedMemorySize,
                                         160 * 1024);
      if (e != hipSuccess) return e;
    }
    attr_set = true;
  }
  TabArgs a;
  a.terms = v.terms;
  a.mb = v.mb;
  a.tab = v.tab;
  a.veff = v.veff;
  a.voff = v.voff;
  a.vin = vin;
  a.tm = tm;
  a.tab_elems = v.tab_elems;
  return launch_term_groups(v.groups, kernels, v.order, a, v.tab_elems * 8, 1, s, ev0, ev1);
}

}  // namespace sg
