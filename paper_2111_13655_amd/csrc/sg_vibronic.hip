// Term sweep of the two-state (vibronic) Smolyak operator for gfx950.
//
// The paper's Sec. 5 pyrazine model has two electronic states: the operator
// at every nuclear configuration is a 2 x 2 matrix.  Alg. 1 per term then
// carries both states through the same one-mode transforms and couples them
// only where the operator acts on the grid: at every grid point
// (y_0, y_1) = [[V_00, V_01], [V_01, V_11]] (g_0, g_1), fused with the first
// grid -> basis contraction.  Along a fiber of the first mode only Q of that
// mode varies, so each potential is A + x (C + B x) with A, B, C formed once
// per fiber from the term's coefficient block (level-0 modes integrated out
// exactly).  The separable harmonic part and the state energies E_s act as
// the exact FP64 diagonal in the reduce, as in the one-state split form.
// One term per workgroup, both states' grids in LDS (sg_term_group.h).
#include "sg_term_group.h"

namespace sg {

namespace {

using namespace grp;

struct VibArgs {
  const TermDev *terms;
  const int32_t *mb;        // M^B, term-major (device order)
  const double *tab;        // standard-map tables (b, wt b^T, nodes per level)
  const double *coef;       // [nterms][kVibCoef] coefficient blocks
  const int32_t *order;     // the terms of this launch
  const double2 *vin;       // [2 N_cs]: the vector H acts on
  double2 *tm;              // [2 N_s]
  int64_t ncs, ns;
  int tab_elems;            // doubles of the table layout in LDS
};

// Coefficient block of a term (kVibCoef doubles), active modes p = 0..na-1 in
// the term record's order: per state s at s * kVibSurf: [0] constant,
// [1 + p] coefficient of Q_p^2, [9 + p] of Q_p, [17 + pair_index(p, q)] of
// Q_p^2 Q_q^2; interstate [2 kVibSurf + p] of Q_p.
struct Coef {
  lds_p<const double> c;
  __device__ double c0(int s) const { return c[s * kVibSurf]; }
  __device__ double a(int s, int p) const { return c[s * kVibSurf + 1 + p]; }
  __device__ double b(int s, int p) const { return c[s * kVibSurf + 9 + p]; }
  __device__ double cc(int s, int p, int q) const { return c[s * kVibSurf + 17 + pair_index(p, q)]; }
  __device__ double lam(int p) const { return c[2 * kVibSurf + p]; }
};

// The 2 x 2 potential along the mode-0 fibers of a term.
struct VibPot {
  const TermDev *T;
  Coef cf;
  lds_p<const double> tab;
  lds_p<const double> x0n;   // nodes of mode 0
  struct Fiber {
    double A[2], B[2], C[2], A01, C01;
  };
  __device__ Fiber fiber(int f) const {
    const int na = T->na;
    // coordinates of the fiber along modes 1..na-1 (mode 1 fastest)
    double xq[kMaxActive];
    int rem = f;
    for (int q = 1; q < na; ++q) {
      const int nq = T->nq[q];
      const int hi = rem / nq;
      xq[q] = tab[std_table_base(T->lev[q]) + 2 * T->nb[q] * nq + (rem - hi * nq)];
      rem = hi;
    }
    Fiber c;
    for (int s = 0; s < 2; ++s) {
      c.A[s] = cf.c0(s);
      c.B[s] = cf.a(s, 0);
      c.C[s] = cf.b(s, 0);
      for (int q = 1; q < na; ++q) {
        const double x2 = xq[q] * xq[q];
        c.A[s] = fma(cf.a(s, q), x2, c.A[s]);
        c.A[s] = fma(cf.b(s, q), xq[q], c.A[s]);
        c.B[s] = fma(cf.cc(s, 0, q), x2, c.B[s]);
        for (int r = q + 1; r < na; ++r) c.A[s] = fma(cf.cc(s, q, r) * x2, xq[r] * xq[r], c.A[s]);
      }
    }
    c.A01 = 0.0;
    for (int q = 1; q < na; ++q) c.A01 = fma(cf.lam(q), xq[q], c.A01);
    c.C01 = cf.lam(0);
    return c;
  }
  __device__ __forceinline__ void point(const Fiber &c, int u, const Z (&g)[2], Z (&y)[2]) const {
    const double x = x0n[u];
    const double V0 = fma(fma(c.B[0], x, c.C[0]), x, c.A[0]);
    const double V1 = fma(fma(c.B[1], x, c.C[1]), x, c.A[1]);
    const double Vx = fma(c.C01, x, c.A01);
    y[0] = Z{fma(V0, g[0].x, Vx * g[1].x), fma(V0, g[0].y, Vx * g[1].y)};
    y[1] = Z{fma(Vx, g[0].x, V1 * g[1].x), fma(Vx, g[0].y, V1 * g[1].y)};
  }
};

// One launch group's terms: VT threads per term, grids of at most MAXG
// points, active levels at most MAXLEV.
template <int VT, int MAXG, int MAXLEV>
__global__ __launch_bounds__(VT) void vib_sweep_kernel(VibArgs a) {
  extern __shared__ char lds_raw[];
  const int t = a.order[blockIdx.x];
  // read in place: a copy with dynamically indexed arrays would live in scratch
  const TermDev &T = a.terms[t];
  lds_p<double> tab = (lds_p<double>)lds_raw;
  lds_p<double> cfl = tab + a.tab_elems;
  const Bufs<2> B{{(lds_p<Z>)(cfl + kVibCoef), (lds_p<Z>)(cfl + kVibCoef) + T.ngrid}};
  const int off = T.off;
  copy_tables<VT>(T, tab, a.tab);
  for (int i = threadIdx.x; i < kVibCoef; i += VT) cfl[i] = a.coef[(size_t)t * kVibCoef + i];
  __syncthreads();
  const Coef cf{cfl};
  const glb_p<Z> tout[2] = {(glb_p<Z>)a.tm + off, (glb_p<Z>)a.tm + a.ns + off};
  const glb_p<const Z> vin[2] = {(glb_p<const Z>)a.vin, (glb_p<const Z>)a.vin + a.ncs};
  if (T.na == 0) {   // a scalar term: only the constants act (linear terms average out)
    if (threadIdx.x == 0) {
      const int c = a.mb[off];
      for (int s = 0; s < 2; ++s) {
        const Z v = ldz(vin[s] + c);
        stz(tout[s], T.coeff * cf.c0(s) * v.x, T.coeff * cf.c0(s) * v.y);
      }
    }
    return;
  }
  const int nb0 = T.nb[0], nq0 = T.nq[0];
  const VibPot pot{&T, cf, tab, tab + std_table_base(T.lev[0]) + 2 * nb0 * nq0};
  run_term<2, VT, MAXG, MAXLEV>(T, tab, B, vin, (glb_p<const int32_t>)a.mb + off, pot, tout);
}

template <int S>
constexpr auto vib_kernel() {
  return &vib_sweep_kernel<kGroupShape[S].vt, kGroupShape[S].max_grid, kGroupShape[S].max_level>;
}

}  // namespace

hipError_t launch_vib_sweep(const VibLaunch &v, const double2 *vin, double2 *tm, hipStream_t s,
                            hipEvent_t ev0, hipEvent_t ev1) {
  static_assert(kGroupShapes == 3, "one kernel per shape");
  static const void *const kernels[kGroupShapes] = {
      (const void *)vib_kernel<0>(), (const void *)vib_kernel<1>(), (const void *)vib_kernel<2>()};
  static bool attr_set = false;
  if (!attr_set) {
    for (int k = 0; k < kGroupShapes; ++k) {
      hipError_t e = hipFuncSetAttribute(kernels[k], hipFuncAttributeMaxDynamicSharedMemorySize,
                                         160 * 1024);
      if (e != hipSuccess) return e;
    }
    attr_set = true;
  }
  VibArgs a;
  a.terms = v.terms;
  a.mb = v.mb;
  a.tab = v.tab;
  a.coef = v.coef;
  a.vin = vin;
  a.tm = tm;
  a.ncs = v.ncs;
  a.ns = v.ns;
  a.tab_elems = v.tab_elems;
  return launch_term_groups(v.groups, kernels, v.order, a, v.tab_elems * 8 + kVibCoef * 8, 2, s,
                            ev0, ev1);
}

}  // namespace sg
