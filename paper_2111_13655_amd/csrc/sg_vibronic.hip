// Term sweep of the two-state (vibronic) Smolyak operator for gfx950.
//
// The paper's Sec. 5 pyrazine model has two electronic states: the operator
// at every nuclear configuration is a 2 x 2 matrix.  Alg. 1 per term then
// carries both states through the same one-mode transforms and couples them
// only where the operator acts on the grid:
//   1. gather both states' coefficients through M^B, fused with the basis ->
//      grid contraction along the first active mode (fibers along that mode
//      are contiguous in the term-major layout);
//   2. basis -> grid along the other active modes (eq_transfer_b_to_g), in
//      place in LDS, both states;
//   3. at every grid point (y_0, y_1) = [[V_00, V_01], [V_01, V_11]] (g_0, g_1),
//      fused with the first grid -> basis contraction: along a fiber of the
//      first mode only Q of that mode varies, so each potential is
//      A + x (C + B x) with A, B, C formed once per fiber from the term's
//      coefficient block (level-0 modes integrated out exactly);
//   4. grid -> basis along the other modes (eq_transfer_g_to_b); the last
//      contraction writes D_l times the result, per state, to the term-major
//      buffer (state s at offset s N_s).
// The separable harmonic part and the state energies E_s act as the exact
// FP64 diagonal in the reduce, as in the one-state split form.
//
// One term per workgroup (256 threads); both states' grids sit in LDS (two
// buffers of the term's grid, 128 KB at a 4096-point term).  A contraction
// loads every input fiber of the group into registers before any output
// overwrites them (at most VibFpt<NI> fibers per thread: grids up to 4096
// points).  Terms are launched in groups of similar LDS need, largest first.
#include <hip/hip_ext.h>

#include "sg_internal.h"

namespace sg {

namespace {

constexpr int kVT = 256;           // threads per term
constexpr int kVibMaxGrid = 4096;  // largest term grid (standard maps, L <= 6)

template <typename T> using lds_p = __attribute__((address_space(3))) T *;
template <typename T> using glb_p = __attribute__((address_space(1))) T *;

struct alignas(16) Z { double x, y; };

template <typename P>
__device__ __forceinline__ Z ldz(P p) {
  Z v;
  v.x = p->x;
  v.y = p->y;
  return v;
}
template <typename P>
__device__ __forceinline__ void stz(P p, double x, double y) {
  p->x = x;
  p->y = y;
}

// fibers of NI values one thread holds in an in-place contraction of a grid
// of at most kVibMaxGrid points
template <int NI>
struct VibFpt {
  static constexpr int value = ((kVibMaxGrid + NI - 1) / NI + kVT - 1) / kVT;
};

struct VibArgs {
  const TermDev *terms;
  const int32_t *mb;        // M^B, term-major (device order)
  const double *tab;        // standard-map tables (b, wt b^T, nodes per level)
  const double *coef;       // [nterms][kVibCoef] coefficient blocks
  const int32_t *order;     // the terms of this launch
  const double2 *vin;       // [2 N_cs]: the vector H acts on
  double2 *tm;              // [2 N_s]
  int64_t ncs, ns;
  int tab_elems;            // doubles of tables copied to LDS
};

// out[lo + stride (u + NO hi)] = sum_k M[u NI + k] in[lo + stride (k + NI hi)]
// for both states, in place (all inputs of the group read before the sync).
template <int NI, int NO>
__device__ __forceinline__ void vib_contract(lds_p<Z> b0, lds_p<Z> b1, lds_p<const double> M,
                                             int stride, int nouter) {
  constexpr int FPT = VibFpt<NI>::value;
  const int F = stride * nouter;
  Z x0[FPT][NI], x1[FPT][NI];
  int ob[FPT];
#pragma unroll
  for (int j = 0; j < FPT; ++j) {
    const int f = threadIdx.x + j * kVT;
    ob[j] = -1;
    if (f < F) {
      const int hi = f / stride;
      const int lo = f - hi * stride;
      const int ib = lo + hi * stride * NI;
      ob[j] = lo + hi * stride * NO;
#pragma unroll
      for (int k = 0; k < NI; ++k) {
        x0[j][k] = ldz(b0 + ib + k * stride);
        x1[j][k] = ldz(b1 + ib + k * stride);
      }
    }
  }
  __syncthreads();
#pragma unroll
  for (int j = 0; j < FPT; ++j) {
    if (ob[j] < 0) continue;
#pragma unroll 1
    for (int u = 0; u < NO; ++u) {
      double r0 = 0, i0 = 0, r1 = 0, i1 = 0;
#pragma unroll
      for (int k = 0; k < NI; ++k) {
        const double m = M[u * NI + k];
        r0 = fma(m, x0[j][k].x, r0);
        i0 = fma(m, x0[j][k].y, i0);
        r1 = fma(m, x1[j][k].x, r1);
        i1 = fma(m, x1[j][k].y, i1);
      }
      stz(b0 + ob[j] + u * stride, r0, i0);
      stz(b1 + ob[j] + u * stride, r1, i1);
    }
  }
  __syncthreads();
}

// the last grid -> basis contraction (nouter = 1): D_l times the result to HBM
template <int NI, int NO>
__device__ __forceinline__ void vib_store(lds_p<Z> b0, lds_p<Z> b1, lds_p<const double> M,
                                          int stride, double dl, glb_p<Z> t0, glb_p<Z> t1) {
  for (int lo = threadIdx.x; lo < stride; lo += kVT) {
    Z x0[NI], x1[NI];
#pragma unroll
    for (int k = 0; k < NI; ++k) {
      x0[k] = ldz(b0 + lo + k * stride);
      x1[k] = ldz(b1 + lo + k * stride);
    }
#pragma unroll 1
    for (int u = 0; u < NO; ++u) {
      double r0 = 0, i0 = 0, r1 = 0, i1 = 0;
#pragma unroll
      for (int k = 0; k < NI; ++k) {
        const double m = M[u * NI + k];
        r0 = fma(m, x0[k].x, r0);
        i0 = fma(m, x0[k].y, i0);
        r1 = fma(m, x1[k].x, r1);
        i1 = fma(m, x1[k].y, i1);
      }
      stz(t0 + lo + u * stride, dl * r0, dl * i0);
      stz(t1 + lo + u * stride, dl * r1, dl * i1);
    }
  }
}

// steps 1 and 2 (first mode): gather both states and transform along mode 0
template <int NB, int NQ>
__device__ __forceinline__ void vib_gather(const VibArgs &a, int off, int nfib,
                                           lds_p<const double> M, lds_p<Z> b0, lds_p<Z> b1) {
  const glb_p<const Z> v0 = (glb_p<const Z>)a.vin;
  const glb_p<const Z> v1 = v0 + a.ncs;
  const glb_p<const int32_t> mb = (glb_p<const int32_t>)a.mb + off;
  for (int f = threadIdx.x; f < nfib; f += kVT) {
    int idx[NB];
#pragma unroll
    for (int k = 0; k < NB; ++k) idx[k] = mb[f * NB + k];
    Z x0[NB], x1[NB];
#pragma unroll
    for (int k = 0; k < NB; ++k) {
      x0[k] = ldz(v0 + idx[k]);
      x1[k] = ldz(v1 + idx[k]);
    }
#pragma unroll 1
    for (int u = 0; u < NQ; ++u) {
      double r0 = 0, i0 = 0, r1 = 0, i1 = 0;
#pragma unroll
      for (int k = 0; k < NB; ++k) {
        const double m = M[u * NB + k];
        r0 = fma(m, x0[k].x, r0);
        i0 = fma(m, x0[k].y, i0);
        r1 = fma(m, x1[k].x, r1);
        i1 = fma(m, x1[k].y, i1);
      }
      stz(b0 + f * NQ + u, r0, i0);
      stz(b1 + f * NQ + u, r1, i1);
    }
  }
}

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

// step 3 fused with the grid -> basis contraction along mode 0 (fibers of NQ
// contiguous points).  STORE: mode 0 is the only active mode; the outputs,
// times D_l, go to HBM.
template <int NQ, int NB, bool STORE>
__device__ __forceinline__ void vib_potential(const TermDev &T, const Coef &cf,
                                              lds_p<const double> tab, lds_p<Z> b0, lds_p<Z> b1,
                                              int nfib, double dl, glb_p<Z> t0, glb_p<Z> t1) {
  constexpr int FPT = VibFpt<NQ>::value;
  const int na = T.na;
  const int l0 = T.lev[0];
  const lds_p<const double> x0n = tab + std_table_base(l0) + 2 * NB * NQ;
  const lds_p<const double> W = tab + std_table_base(l0) + NB * NQ;
  Z y0[FPT][NQ], y1[FPT][NQ];
  int fb[FPT];
#pragma unroll
  for (int j = 0; j < FPT; ++j) {
    const int f = threadIdx.x + j * kVT;
    fb[j] = f < nfib ? f : -1;
    if (fb[j] < 0) continue;
    // coordinates of the fiber along modes 1..na-1 (mode 1 fastest)
    double xq[kMaxActive];
    int rem = f;
    for (int q = 1; q < na; ++q) {
      const int nq = T.nq[q];
      const int hi = rem / nq;
      xq[q] = tab[std_table_base(T.lev[q]) + 2 * T.nb[q] * nq + (rem - hi * nq)];
      rem = hi;
    }
    double A[2], B[2], C[2], A01 = 0.0;
    for (int s = 0; s < 2; ++s) {
      A[s] = cf.c0(s);
      B[s] = cf.a(s, 0);
      C[s] = cf.b(s, 0);
      for (int q = 1; q < na; ++q) {
        const double x2 = xq[q] * xq[q];
        A[s] = fma(cf.a(s, q), x2, A[s]);
        A[s] = fma(cf.b(s, q), xq[q], A[s]);
        B[s] = fma(cf.cc(s, 0, q), x2, B[s]);
        for (int r = q + 1; r < na; ++r) A[s] = fma(cf.cc(s, q, r) * x2, xq[r] * xq[r], A[s]);
      }
    }
    for (int q = 1; q < na; ++q) A01 = fma(cf.lam(q), xq[q], A01);
    const double C01 = cf.lam(0);
#pragma unroll
    for (int u = 0; u < NQ; ++u) {
      const double x = x0n[u];
      const double V0 = fma(fma(B[0], x, C[0]), x, A[0]);
      const double V1 = fma(fma(B[1], x, C[1]), x, A[1]);
      const double Vx = fma(C01, x, A01);
      const Z g0 = ldz(b0 + f * NQ + u), g1 = ldz(b1 + f * NQ + u);
      y0[j][u] = Z{fma(V0, g0.x, Vx * g1.x), fma(V0, g0.y, Vx * g1.y)};
      y1[j][u] = Z{fma(Vx, g0.x, V1 * g1.x), fma(Vx, g0.y, V1 * g1.y)};
    }
  }
  if (!STORE) __syncthreads();
#pragma unroll
  for (int j = 0; j < FPT; ++j) {
    if (fb[j] < 0) continue;
#pragma unroll 1
    for (int v = 0; v < NB; ++v) {
      double r0 = 0, i0 = 0, r1 = 0, i1 = 0;
#pragma unroll
      for (int u = 0; u < NQ; ++u) {
        const double m = W[v * NQ + u];
        r0 = fma(m, y0[j][u].x, r0);
        i0 = fma(m, y0[j][u].y, i0);
        r1 = fma(m, y1[j][u].x, r1);
        i1 = fma(m, y1[j][u].y, i1);
      }
      if (STORE) {
        stz(t0 + fb[j] * NB + v, dl * r0, dl * i0);
        stz(t1 + fb[j] * NB + v, dl * r1, dl * i1);
      } else {
        stz(b0 + fb[j] * NB + v, r0, i0);
        stz(b1 + fb[j] * NB + v, r1, i1);
      }
    }
  }
  if (!STORE) __syncthreads();
}

#define SG_VIB_LEVELS(X) X(1, 3, 4) X(2, 5, 6) X(3, 7, 8) X(4, 9, 10) X(5, 11, 12) X(6, 13, 14)

__global__ __launch_bounds__(kVT) void vib_sweep_kernel(VibArgs a) {
  extern __shared__ char lds_raw[];
  const int t = a.order[blockIdx.x];
  const TermDev T = a.terms[t];
  lds_p<double> tab = (lds_p<double>)lds_raw;
  lds_p<double> cfl = tab + a.tab_elems;
  lds_p<Z> b0 = (lds_p<Z>)(cfl + kVibCoef);
  lds_p<Z> b1 = b0 + T.ngrid;
  for (int i = threadIdx.x; i < a.tab_elems; i += kVT) tab[i] = a.tab[i];
  for (int i = threadIdx.x; i < kVibCoef; i += kVT) cfl[i] = a.coef[(size_t)t * kVibCoef + i];
  __syncthreads();
  const Coef cf{cfl};
  const int na = T.na, off = T.off;
  const double dl = T.coeff;
  const glb_p<Z> t0 = (glb_p<Z>)a.tm + off, t1 = t0 + a.ns;
  if (na == 0) {   // a scalar term: only the constants act (linear terms average out)
    if (threadIdx.x == 0) {
      const int c = a.mb[off];
      const Z v0 = ldz((glb_p<const Z>)a.vin + c), v1 = ldz((glb_p<const Z>)a.vin + a.ncs + c);
      stz(t0, dl * cf.c0(0) * v0.x, dl * cf.c0(0) * v0.y);
      stz(t1, dl * cf.c0(1) * v1.x, dl * cf.c0(1) * v1.y);
    }
    return;
  }
  const int l0 = T.lev[0];
  // steps 1-2
  {
    const lds_p<const double> M0 = tab + std_table_base(l0);
    const int nfib = T.nbasis / T.nb[0];
#define SG_VG(L_, NB_, NQ_) \
  case L_: vib_gather<NB_, NQ_>(a, off, nfib, M0, b0, b1); break;
    switch (l0) { SG_VIB_LEVELS(SG_VG) default: break; }
#undef SG_VG
    __syncthreads();
    int stride = T.nq[0], nouter = nfib;
    for (int p = 1; p < na; ++p) {
      nouter /= T.nb[p];
      const lds_p<const double> M = tab + std_table_base(T.lev[p]);
#define SG_VB(L_, NB_, NQ_) \
  case L_: vib_contract<NB_, NQ_>(b0, b1, M, stride, nouter); break;
      switch (T.lev[p]) { SG_VIB_LEVELS(SG_VB) default: break; }
#undef SG_VB
      stride *= T.nq[p];
    }
  }
  // step 3 + first grid -> basis contraction
  const int nfib = T.ngrid / T.nq[0];
  if (na == 1) {
#define SG_VP1(L_, NB_, NQ_) \
  case L_: vib_potential<NQ_, NB_, true>(T, cf, tab, b0, b1, nfib, dl, t0, t1); break;
    switch (l0) { SG_VIB_LEVELS(SG_VP1) default: break; }
#undef SG_VP1
    return;
  }
#define SG_VP(L_, NB_, NQ_) \
  case L_: vib_potential<NQ_, NB_, false>(T, cf, tab, b0, b1, nfib, dl, t0, t1); break;
  switch (l0) { SG_VIB_LEVELS(SG_VP) default: break; }
#undef SG_VP
  // step 4
  int stride = T.nb[0], nouter = nfib;
  for (int p = 1; p < na - 1; ++p) {
    nouter /= T.nq[p];
    const lds_p<const double> M = tab + std_table_base(T.lev[p]) + T.nb[p] * T.nq[p];
#define SG_VC(L_, NB_, NQ_) \
  case L_: vib_contract<NQ_, NB_>(b0, b1, M, stride, nouter); break;
    switch (T.lev[p]) { SG_VIB_LEVELS(SG_VC) default: break; }
#undef SG_VC
    stride *= T.nb[p];
  }
  const int p = na - 1;
  const lds_p<const double> M = tab + std_table_base(T.lev[p]) + T.nb[p] * T.nq[p];
#define SG_VS(L_, NB_, NQ_) \
  case L_: vib_store<NQ_, NB_>(b0, b1, M, stride, dl, t0, t1); break;
  switch (T.lev[p]) { SG_VIB_LEVELS(SG_VS) default: break; }
#undef SG_VS
}

}  // namespace

hipError_t launch_vib_sweep(const VibLaunch &v, const double2 *vin, double2 *tm, hipStream_t s,
                            hipEvent_t ev0, hipEvent_t ev1) {
  static bool attr_set = false;
  if (!attr_set) {
    hipError_t e = hipFuncSetAttribute((const void *)vib_sweep_kernel,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    if (e != hipSuccess) return e;
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
  const int ngroups = (int)v.groups.size();
  for (int g = 0; g < ngroups; ++g) {
    const VibGroup &G = v.groups[g];
    if (G.count == 0) continue;
    a.order = v.order + G.first;
    const int lds = (int)(v.tab_elems * 8 + kVibCoef * 8 + 2 * G.max_grid * 16);
    hipEvent_t e0 = g == 0 ? ev0 : nullptr, e1 = g == ngroups - 1 ? ev1 : nullptr;
    if (e0 || e1)
      hipExtLaunchKernelGGL(vib_sweep_kernel, dim3((unsigned)G.count), dim3(kVT), lds, s, e0, e1,
                            0, a);
    else
      hipLaunchKernelGGL(vib_sweep_kernel, dim3((unsigned)G.count), dim3(kVT), lds, s, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace sg
