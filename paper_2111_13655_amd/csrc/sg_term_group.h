// Device building blocks of term sweeps that run one Smolyak term per
// workgroup over NS coupled states (the two-state operator: NS = 2).  Alg. 1
// per term, for every state s = 0..NS-1:
//   1. gather the term's coefficients through M^B, fused with the basis ->
//      grid contraction along the first active mode (fibers along that mode
//      are contiguous in the term-major layout);
//   2. basis -> grid along the other active modes (eq_transfer_b_to_g), in
//      place in LDS;
//   3. the operator on the grid (supplied by the kernel), fused with the
//      first grid -> basis contraction;
//   4. grid -> basis along the other modes (eq_transfer_g_to_b); the last
//      contraction writes D_l times the result to the term-major buffer.
//
// Terms are launched in groups of one shape each (threads per workgroup,
// largest grid, highest level), so a kernel instantiates only the
// contraction sizes its terms can have and holds at most kGroupFptCap fibers
// per thread; a contraction over more fibers runs in chunks: every thread
// loads its fibers of the chunk, the group syncs, and the outputs overwrite
// the buffer.  Compacting contractions (NO < NI) take their chunks in
// increasing fiber order and expanding ones in decreasing order: fiber
// f = lo + stride hi reads in[lo + stride (k + NI hi)] and writes
// out[lo + stride (u + NO hi)], the two coincide only for equal lo, and then
// NO < NI puts every output of hi below the inputs of every later hi' > hi
// (NO > NI: above those of every earlier hi'), so no chunk overwrites inputs
// that a later chunk has not read yet.
#pragma once

#include <hip/hip_ext.h>

#include <vector>

#include "sg_internal.h"

namespace sg {
namespace grp {

constexpr int kGroupFptCap = 2;   // fibers per thread and chunk

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

// sizes of a level of the standard maps
template <int L_>
struct VLev {
  static constexpr int NB = 2 * L_ + 1, NQ = 2 * L_ + 2;
};

// calls f(VLev<l>{}) for the levels 1..MAXLEV (other levels do nothing; the
// host never sends a term with a higher level to such a kernel)
template <int MAXLEV, typename F>
__device__ __forceinline__ void by_level(int l, F &&f) {
  switch (l) {
    case 1: if constexpr (MAXLEV >= 1) f(VLev<1>{}); break;
    case 2: if constexpr (MAXLEV >= 2) f(VLev<2>{}); break;
    case 3: if constexpr (MAXLEV >= 3) f(VLev<3>{}); break;
    case 4: if constexpr (MAXLEV >= 4) f(VLev<4>{}); break;
    case 5: if constexpr (MAXLEV >= 5) f(VLev<5>{}); break;
    case 6: if constexpr (MAXLEV >= 6) f(VLev<6>{}); break;
    default: break;
  }
}

// fibers of NI values one thread holds per chunk of a contraction over a grid
// of at most MAXG points
template <int NI, int VT, int MAXG>
struct Fpt {
  static constexpr int raw = ((MAXG + NI - 1) / NI + VT - 1) / VT;
  static constexpr int value = raw < kGroupFptCap ? raw : kGroupFptCap;
};

// The states' grid buffers of one term in LDS.
template <int NS>
struct Bufs {
  lds_p<Z> b[NS];
};

// out[lo + stride (u + NO hi)] = sum_k M[u NI + k] in[lo + stride (k + NI hi)]
// for every state, in place, in chunks (order above).
template <int NS, int NI, int NO, int VT, int MAXG>
__device__ __forceinline__ void contract(const Bufs<NS> &B, lds_p<const double> M, int stride,
                                         int nouter) {
  constexpr int FPT = Fpt<NI, VT, MAXG>::value;
  constexpr int CH = FPT * VT;
  const int F = stride * nouter;
  const int nch = (F + CH - 1) / CH;
  for (int cc = 0; cc < nch; ++cc) {
    const int base = (NO < NI ? cc : nch - 1 - cc) * CH;
    Z x[FPT][NS][NI];
    int ob[FPT];
#pragma unroll
    for (int j = 0; j < FPT; ++j) {
      const int f = base + (int)threadIdx.x + j * VT;
      ob[j] = -1;
      if (f < F) {
        const int hi = f / stride;
        const int lo = f - hi * stride;
        const int ib = lo + hi * stride * NI;
        ob[j] = lo + hi * stride * NO;
#pragma unroll
        for (int s = 0; s < NS; ++s)
#pragma unroll
          for (int k = 0; k < NI; ++k) x[j][s][k] = ldz(B.b[s] + ib + k * stride);
      }
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < FPT; ++j) {
      if (ob[j] < 0) continue;
#pragma unroll 1
      for (int u = 0; u < NO; ++u) {
        double r[NS], i[NS];
#pragma unroll
        for (int s = 0; s < NS; ++s) r[s] = i[s] = 0.0;
#pragma unroll
        for (int k = 0; k < NI; ++k) {
          const double m = M[u * NI + k];
#pragma unroll
          for (int s = 0; s < NS; ++s) {
            r[s] = fma(m, x[j][s][k].x, r[s]);
            i[s] = fma(m, x[j][s][k].y, i[s]);
          }
        }
#pragma unroll
        for (int s = 0; s < NS; ++s) stz(B.b[s] + ob[j] + u * stride, r[s], i[s]);
      }
    }
    __syncthreads();
  }
}

// the last grid -> basis contraction (nouter = 1): D_l times the result to
// HBM, state s at t[s]
template <int NS, int NI, int NO, int VT>
__device__ __forceinline__ void store(const Bufs<NS> &B, lds_p<const double> M, int stride,
                                      double dl, const glb_p<Z> (&t)[NS]) {
  for (int lo = threadIdx.x; lo < stride; lo += VT) {
    Z x[NS][NI];
#pragma unroll
    for (int s = 0; s < NS; ++s)
#pragma unroll
      for (int k = 0; k < NI; ++k) x[s][k] = ldz(B.b[s] + lo + k * stride);
#pragma unroll 1
    for (int u = 0; u < NO; ++u) {
      double r[NS], i[NS];
#pragma unroll
      for (int s = 0; s < NS; ++s) r[s] = i[s] = 0.0;
#pragma unroll
      for (int k = 0; k < NI; ++k) {
        const double m = M[u * NI + k];
#pragma unroll
        for (int s = 0; s < NS; ++s) {
          r[s] = fma(m, x[s][k].x, r[s]);
          i[s] = fma(m, x[s][k].y, i[s]);
        }
      }
#pragma unroll
      for (int s = 0; s < NS; ++s) stz(t[s] + lo + u * stride, dl * r[s], dl * i[s]);
    }
  }
}

// steps 1 and 2 along the first active mode: gather every state (state s of
// the compact vector at v[s]) and transform along mode 0
template <int NS, int NB, int NQ, int VT>
__device__ __forceinline__ void gather(const glb_p<const Z> (&v)[NS], glb_p<const int32_t> mb,
                                       int nfib, lds_p<const double> M, const Bufs<NS> &B) {
  for (int f = threadIdx.x; f < nfib; f += VT) {
    int idx[NB];
#pragma unroll
    for (int k = 0; k < NB; ++k) idx[k] = mb[f * NB + k];
    Z x[NS][NB];
#pragma unroll
    for (int s = 0; s < NS; ++s)
#pragma unroll
      for (int k = 0; k < NB; ++k) x[s][k] = ldz(v[s] + idx[k]);
#pragma unroll 1
    for (int u = 0; u < NQ; ++u) {
      double r[NS], i[NS];
#pragma unroll
      for (int s = 0; s < NS; ++s) r[s] = i[s] = 0.0;
#pragma unroll
      for (int k = 0; k < NB; ++k) {
        const double m = M[u * NB + k];
#pragma unroll
        for (int s = 0; s < NS; ++s) {
          r[s] = fma(m, x[s][k].x, r[s]);
          i[s] = fma(m, x[s][k].y, i[s]);
        }
      }
#pragma unroll
      for (int s = 0; s < NS; ++s) stz(B.b[s] + f * NQ + u, r[s], i[s]);
    }
  }
}

// Step 3 fused with the grid -> basis contraction along mode 0 (fibers of NQ
// contiguous points), in chunks of increasing fiber order (compacting).  The
// operator on the grid comes from `pot`:
//   ctx = pot.fiber(f)         once per fiber, before its points;
//   pot.point(ctx, u, g, y)    y = the operator at point u of the fiber
//                              applied to the states' values g there.
// STORE: mode 0 is the only active mode; the outputs, times D_l, go to HBM.
template <int NS, int NQ, int NB, bool STORE, int VT, int MAXG, typename Pot>
__device__ __forceinline__ void potential(const Pot &pot, const Bufs<NS> &B,
                                          lds_p<const double> W, int nfib, double dl,
                                          const glb_p<Z> (&t)[NS]) {
  constexpr int FPT = Fpt<NQ, VT, MAXG>::value;
  constexpr int CH = FPT * VT;
  const int nch = (nfib + CH - 1) / CH;
  for (int c = 0; c < nch; ++c) {
    Z y[FPT][NS][NQ];
    int fb[FPT];
#pragma unroll
    for (int j = 0; j < FPT; ++j) {
      const int f = c * CH + (int)threadIdx.x + j * VT;
      fb[j] = f < nfib ? f : -1;
      if (fb[j] < 0) continue;
      const typename Pot::Fiber ctx = pot.fiber(f);
#pragma unroll
      for (int u = 0; u < NQ; ++u) {
        Z g[NS], yu[NS];
#pragma unroll
        for (int s = 0; s < NS; ++s) g[s] = ldz(B.b[s] + f * NQ + u);
        pot.point(ctx, u, g, yu);
#pragma unroll
        for (int s = 0; s < NS; ++s) y[j][s][u] = yu[s];
      }
    }
    if (!STORE) __syncthreads();
#pragma unroll
    for (int j = 0; j < FPT; ++j) {
      if (fb[j] < 0) continue;
#pragma unroll 1
      for (int v = 0; v < NB; ++v) {
        double r[NS], i[NS];
#pragma unroll
        for (int s = 0; s < NS; ++s) r[s] = i[s] = 0.0;
#pragma unroll
        for (int u = 0; u < NQ; ++u) {
          const double m = W[v * NQ + u];
#pragma unroll
          for (int s = 0; s < NS; ++s) {
            r[s] = fma(m, y[j][s][u].x, r[s]);
            i[s] = fma(m, y[j][s][u].y, i[s]);
          }
        }
#pragma unroll
        for (int s = 0; s < NS; ++s) {
          if (STORE)
            stz(t[s] + fb[j] * NB + v, dl * r[s], dl * i[s]);
          else
            stz(B.b[s] + fb[j] * NB + v, r[s], i[s]);
        }
      }
    }
    if (!STORE) __syncthreads();
  }
}

// The tables of the levels a term's active modes use, copied from the
// standard layout in HBM to the same places in LDS.
template <int VT>
__device__ __forceinline__ void copy_tables(const TermDev &T, lds_p<double> tab,
                                            const double *gtab) {
  for (int p = 0; p < T.na; ++p) {
    const int l = T.lev[p];
    bool seen = false;
    for (int q = 0; q < p; ++q) seen = seen || T.lev[q] == l;
    if (seen) continue;
    const int base = std_table_base(l), n = 2 * (2 * l + 1) * (2 * l + 2) + (2 * l + 2);
    for (int i = threadIdx.x; i < n; i += VT) tab[base + i] = gtab[base + i];
  }
}

// Steps 1-4 for a term with at least one active mode: its levels' tables are
// in LDS at `tab`, its states' grid buffers in B, state s of the compact
// input at v[s] and of the term-major output at t[s].
template <int NS, int VT, int MAXG, int MAXLEV, typename Pot>
__device__ __forceinline__ void run_term(const TermDev &T, lds_p<const double> tab,
                                         const Bufs<NS> &B, const glb_p<const Z> (&v)[NS],
                                         glb_p<const int32_t> mb, const Pot &pot,
                                         const glb_p<Z> (&t)[NS]) {
  const int na = T.na, l0 = T.lev[0];
  const double dl = T.coeff;
  // steps 1-2
  {
    const lds_p<const double> M0 = tab + std_table_base(l0);
    const int nfib = T.nbasis / T.nb[0];
    by_level<MAXLEV>(l0, [&](auto lv) {
      using V = decltype(lv);
      gather<NS, V::NB, V::NQ, VT>(v, mb, nfib, M0, B);
    });
    __syncthreads();
    int stride = T.nq[0], nouter = nfib;
    for (int p = 1; p < na; ++p) {
      nouter /= T.nb[p];
      const lds_p<const double> M = tab + std_table_base(T.lev[p]);
      by_level<MAXLEV>(T.lev[p], [&](auto lv) {
        using V = decltype(lv);
        contract<NS, V::NB, V::NQ, VT, MAXG>(B, M, stride, nouter);
      });
      stride *= T.nq[p];
    }
  }
  // step 3 + the first grid -> basis contraction
  const int nfib = T.ngrid / T.nq[0];
  if (na == 1) {
    by_level<MAXLEV>(l0, [&](auto lv) {
      using V = decltype(lv);
      potential<NS, V::NQ, V::NB, true, VT, MAXG>(pot, B, tab + std_table_base(l0) + V::NB * V::NQ,
                                                  nfib, dl, t);
    });
    return;
  }
  by_level<MAXLEV>(l0, [&](auto lv) {
    using V = decltype(lv);
    potential<NS, V::NQ, V::NB, false, VT, MAXG>(pot, B, tab + std_table_base(l0) + V::NB * V::NQ,
                                                 nfib, dl, t);
  });
  // step 4
  int stride = T.nb[0], nouter = nfib;
  for (int p = 1; p < na - 1; ++p) {
    nouter /= T.nq[p];
    by_level<MAXLEV>(T.lev[p], [&](auto lv) {
      using V = decltype(lv);
      contract<NS, V::NQ, V::NB, VT, MAXG>(B, tab + std_table_base(T.lev[p]) + V::NB * V::NQ,
                                           stride, nouter);
    });
    stride *= T.nb[p];
  }
  const int p = na - 1;
  by_level<MAXLEV>(T.lev[p], [&](auto lv) {
    using V = decltype(lv);
    store<NS, V::NQ, V::NB, VT>(B, tab + std_table_base(T.lev[p]) + V::NB * V::NQ, stride, dl, t);
  });
}

}  // namespace grp
}  // namespace sg

namespace sg {
namespace grp {

// Launches every non-empty group with its shape's kernel: G.count
// workgroups of the shape's threads, `fixed_lds` bytes of LDS plus ns grid
// buffers of the group's largest term.  The kernel argument block `a` has an
// `order` member pointing at the group's terms; ev0 / ev1 (nullable) attach
// to the first / last dispatch.
template <typename Args>
hipError_t launch_term_groups(const std::vector<TermGroup> &groups,
                              const void *const (&kernels)[kGroupShapes], const int32_t *order,
                              Args &a, int fixed_lds, int ns, hipStream_t s, hipEvent_t ev0,
                              hipEvent_t ev1) {
  int first = -1, last = -1;
  for (int g = 0; g < (int)groups.size(); ++g)
    if (groups[g].count > 0) {
      if (first < 0) first = g;
      last = g;
    }
  for (int g = 0; g < (int)groups.size(); ++g) {
    const TermGroup &G = groups[g];
    if (G.count == 0) continue;
    if (G.shape < 0 || G.shape >= kGroupShapes || G.max_grid > kGroupShape[G.shape].max_grid)
      return hipErrorInvalidValue;
    a.order = order + G.first;
    const size_t lds = (size_t)fixed_lds + (size_t)ns * G.max_grid * 16;
    void *args[] = {&a};
    hipError_t e = hipExtLaunchKernel(kernels[G.shape], dim3((unsigned)G.count),
                                      dim3((unsigned)kGroupShape[G.shape].vt), args, lds, s,
                                      g == first ? ev0 : nullptr, g == last ? ev1 : nullptr, 0);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace grp
}  // namespace sg
