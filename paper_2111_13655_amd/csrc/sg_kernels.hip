// HIP kernels of the Smolyak operator action for gfx950 (MI355X).
//
// sweep_fp64: one workgroup per Smolyak term (Alg. 1, Sec. 3).  The term's
//   coefficients are gathered from the compact vector through M^B into LDS,
//   transformed basis -> grid one active mode at a time (eq_transfer_b_to_g),
//   multiplied by the effective potential evaluated on the fly, given the
//   kinetic second-derivative matrices on the grid (FP64 path), transformed
//   grid -> basis (eq_transfer_g_to_b), scaled by D_l and written to the
//   term-major buffer.  Each mode contraction gives one thread a whole fiber
//   along the contracted mode: the fiber sits in registers and the one-mode
//   matrix is wave-uniform, so its entries come through the scalar cache.
//
// reduce_rows: the scatter-add of Alg. 1's last step as a gather: every
//   compact index sums its term-major contributions through the inverse of
//   M^B in a fixed order (one wavefront per row, butterfly shuffle), so the
//   result is bitwise reproducible.  The Chebyshev recurrence and the norm /
//   energy partial sums are fused into its epilogue.
#include "sg_internal.h"

namespace sg {

namespace {

constexpr int kThreads = 256;

struct SweepArgs {
  const TermDev *terms;
  const int32_t *sched;
  const int32_t *mb;
  const double2 *psi;
  double2 *tm;
  const double *tab;
  const double *cmat;
  const double *kmat;
  DeviceTables td;
  int D;
  int std_maps;  // nb = 1 + 2l, nq = 2 + 2l
  int split;     // mixed-style operator: no harmonic part, no kinetic
  int max_grid;
};

// out[lo + stride*(u + NO*hi)] (+)= scale * sum_k M[u*NI + k] in[lo + stride*(k + NI*hi)]
template <int NI, int NO, bool ACC>
__device__ __forceinline__ void contract_fixed(const double2 *__restrict__ in,
                                               double2 *__restrict__ out,
                                               const double *__restrict__ M, double scale,
                                               int stride, int nouter) {
  const int F = stride * nouter;
  for (int f = threadIdx.x; f < F; f += kThreads) {
    const int hi = f / stride;
    const int lo = f - hi * stride;
    const double2 *src = in + lo + hi * (stride * NI);
    double2 *dst = out + lo + hi * (stride * NO);
    double2 x[NI];
#pragma unroll
    for (int k = 0; k < NI; ++k) x[k] = src[k * stride];
#pragma unroll
    for (int u = 0; u < NO; ++u) {
      double re = 0.0, im = 0.0;
#pragma unroll
      for (int k = 0; k < NI; ++k) {
        const double m = M[u * NI + k];
        re = fma(m, x[k].x, re);
        im = fma(m, x[k].y, im);
      }
      if (ACC) {
        double2 o = dst[u * stride];
        o.x = fma(scale, re, o.x);
        o.y = fma(scale, im, o.y);
        dst[u * stride] = o;
      } else {
        dst[u * stride] = make_double2(re, im);
      }
    }
  }
}

// Same with run-time sizes (any size maps up to kMaxN); fully unrolled with
// guards so the fiber stays in registers.
template <bool ACC>
__device__ __forceinline__ void contract_rt(const double2 *__restrict__ in,
                                            double2 *__restrict__ out,
                                            const double *__restrict__ M, double scale,
                                            int NI, int NO, int stride, int nouter) {
  const int F = stride * nouter;
  for (int f = threadIdx.x; f < F; f += kThreads) {
    const int hi = f / stride;
    const int lo = f - hi * stride;
    const double2 *src = in + lo + hi * (stride * NI);
    double2 *dst = out + lo + hi * (stride * NO);
    double2 x[kMaxN];
#pragma unroll
    for (int k = 0; k < kMaxN; ++k) x[k] = (k < NI) ? src[k * stride] : make_double2(0.0, 0.0);
    for (int u = 0; u < NO; ++u) {
      double re = 0.0, im = 0.0;
#pragma unroll
      for (int k = 0; k < kMaxN; ++k) {
        if (k < NI) {
          const double m = M[u * NI + k];
          re = fma(m, x[k].x, re);
          im = fma(m, x[k].y, im);
        }
      }
      if (ACC) {
        double2 o = dst[u * stride];
        o.x = fma(scale, re, o.x);
        o.y = fma(scale, im, o.y);
        dst[u * stride] = o;
      } else {
        dst[u * stride] = make_double2(re, im);
      }
    }
  }
}

// kind 0: basis -> grid (NI = nb, NO = nq); 1: kinetic on the grid
// (NI = NO = nq); 2: grid -> basis (NI = nq, NO = nb)
template <bool ACC>
__device__ __forceinline__ void contract_level(int kind, int level, int std_maps, int nb, int nq,
                                               const double2 *in, double2 *out,
                                               const double *M, double scale, int stride,
                                               int nouter) {
  if (std_maps) {
#define SG_CASE(L_, NB_, NQ_)                                                             \
  case L_:                                                                                \
    if (kind == 0) contract_fixed<NB_, NQ_, ACC>(in, out, M, scale, stride, nouter);      \
    else if (kind == 1) contract_fixed<NQ_, NQ_, ACC>(in, out, M, scale, stride, nouter); \
    else contract_fixed<NQ_, NB_, ACC>(in, out, M, scale, stride, nouter);                \
    return;
    switch (level) {
      SG_CASE(1, 3, 4)
      SG_CASE(2, 5, 6)
      SG_CASE(3, 7, 8)
      SG_CASE(4, 9, 10)
      SG_CASE(5, 11, 12)
      SG_CASE(6, 13, 14)
      SG_CASE(7, 15, 16)
      default: break;
    }
#undef SG_CASE
  }
  const int NI = kind == 0 ? nb : nq;
  const int NO = kind == 2 ? nb : nq;
  contract_rt<ACC>(in, out, M, scale, NI, NO, stride, nouter);
}

__global__ __launch_bounds__(kThreads) void sweep_kernel(SweepArgs a) {
  extern __shared__ double2 lds[];
  const int t = a.sched[blockIdx.x];
  const TermDev *T = a.terms + t;
  const int na = T->na;
  const int nbasis = T->nbasis;
  const int ngrid = T->ngrid;
  const int off = T->off;
  double2 *A = lds;
  double2 *B = lds + a.max_grid;

  // step 1 of Alg. 1: gather through M^B
  for (int s = threadIdx.x; s < nbasis; s += kThreads) A[s] = a.psi[a.mb[off + s]];
  __syncthreads();

  int nb[kMaxActive], nq[kMaxActive], lv[kMaxActive];
#pragma unroll
  for (int p = 0; p < kMaxActive; ++p) {
    lv[p] = p < na ? T->lev[p] : 0;
    nb[p] = p < na ? a.td.lev[lv[p]].nb : 1;
    nq[p] = p < na ? a.td.lev[lv[p]].nq : 1;
  }

  // step 2: basis -> grid, mode by mode
  double2 *src = A, *dst = B;
  {
    int stride = 1;
    int nouter = nbasis;
    for (int p = 0; p < na; ++p) {
      nouter /= nb[p];
      contract_level<false>(0, lv[p], a.std_maps, nb[p], nq[p], src, dst,
                            a.tab + a.td.lev[lv[p]].bt, 1.0, stride, nouter);
      __syncthreads();
      double2 *tmp = src; src = dst; dst = tmp;
      stride *= nq[p];
    }
  }

  // step 3: operator on the grid.  dst = V_eff * src
  {
    const double c0 = a.split ? T->c0_split : T->c0_full;
    double al[kMaxActive], be[kMaxActive];
#pragma unroll
    for (int p = 0; p < kMaxActive; ++p) {
      al[p] = p < na ? (a.split ? T->alpha_split[p] : T->alpha_full[p]) : 0.0;
      be[p] = p < na ? T->beta[p] : 0.0;
    }
    for (int gidx = threadIdx.x; gidx < ngrid; gidx += kThreads) {
      double x[kMaxActive];
      int rem = gidx;
#pragma unroll
      for (int p = 0; p < kMaxActive; ++p) {
        if (p < na) {
          const int u = rem % nq[p];
          rem /= nq[p];
          x[p] = a.tab[a.td.lev[lv[p]].x + u];
        } else {
          x[p] = 0.0;
        }
      }
      double v = c0;
#pragma unroll
      for (int p = 0; p < kMaxActive; ++p) {
        if (p < na) {
          const double x2 = x[p] * x[p];
          v = fma(al[p], x2, v);
          v = fma(be[p], x[p], v);
#pragma unroll
          for (int q = p + 1; q < kMaxActive; ++q) {
            if (q < na) {
              const int mi = T->mode[p] * a.D + T->mode[q];
              v = fma(a.cmat[mi] * x2, x[q] * x[q], v);
              v = fma(a.kmat[mi] * x2, x[q], v);
            }
          }
        }
      }
      const double2 w = src[gidx];
      dst[gidx] = make_double2(v * w.x, v * w.y);
    }
    __syncthreads();
  }
  // kinetic: dst += (-1/2 omega_p) K_p x_p src, for every active mode
  if (!a.split) {
    int stride = 1;
    int nouter = ngrid;
    for (int p = 0; p < na; ++p) {
      nouter /= nq[p];
      contract_level<true>(1, lv[p], a.std_maps, nb[p], nq[p], src, dst,
                           a.tab + a.td.lev[lv[p]].kg, T->kin[p], stride, nouter);
      __syncthreads();
      stride *= nq[p];
    }
  }
  {
    double2 *tmp = src; src = dst; dst = tmp;
  }
  // step 4: grid -> basis
  {
    int stride = 1;
    int nouter = ngrid;
    for (int p = 0; p < na; ++p) {
      nouter /= nq[p];
      contract_level<false>(2, lv[p], a.std_maps, nb[p], nq[p], src, dst,
                            a.tab + a.td.lev[lv[p]].wt, 1.0, stride, nouter);
      __syncthreads();
      double2 *tmp = src; src = dst; dst = tmp;
      stride *= nb[p];
    }
  }
  // step 5 (first half): D_l times the term result, term-major
  const double cf = T->coeff;
  for (int s = threadIdx.x; s < nbasis; s += kThreads) {
    const double2 r = src[s];
    a.tm[off + s] = make_double2(cf * r.x, cf * r.y);
  }
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
  return v;
}

struct ReduceArgs {
  const int32_t *ptr;
  const int32_t *col;
  const double2 *tm;
  const double *h0;
  const double2 *vin;
  double2 *out;
  int64_t ncs;
  double *partials;
  ChebArgs ca;
  int cheb;
};

// step 5 (second half): compact[r] = sum of its term-major contributions
__global__ __launch_bounds__(kThreads) void reduce_kernel(ReduceArgs a) {
  __shared__ double red[2][kThreads / 64];
  const int wave = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
  const int64_t row = (int64_t)blockIdx.x * (kThreads / 64) + wave;
  double pn = 0.0, pe = 0.0;
  if (row < a.ncs) {
    const int b = a.ptr[row], e = a.ptr[row + 1];
    double sr = 0.0, si = 0.0;
    for (int j = b + lane; j < e; j += 64) {
      const double2 v = a.tm[a.col[j]];
      sr += v.x;
      si += v.y;
    }
    sr = wave_sum(sr);
    si = wave_sum(si);
    if (lane == 0) {
      const double2 vk = a.vin[row];
      if (a.ca.split) {
        const double d = a.h0[row];
        sr = fma(d, vk.x, sr);
        si = fma(d, vk.y, si);
      }
      if (!a.cheb) {
        a.out[row] = make_double2(sr, si);
      } else {
        const ChebArgs &c = a.ca;
        const double zr = (sr - c.ebar * vk.x) * c.inv_half;
        const double zi = (si - c.ebar * vk.y) * c.inv_half;
        double2 phi, accv;
        if (c.first) {
          phi = make_double2(zi, -zr);  // -i z
          accv = make_double2(c.a_0 * vk.x + c.a_k * phi.x, c.a_0 * vk.y + c.a_k * phi.y);
          pn = vk.x * vk.x + vk.y * vk.y;
          pe = vk.x * sr + vk.y * si;  // Re(conj(psi) H psi)
        } else {
          const double2 pr = c.prev[row];
          phi = make_double2(2.0 * zi + pr.x, -2.0 * zr + pr.y);  // -2i z + phi_{k-1}
          const double2 ac = c.acc[row];
          accv = make_double2(ac.x + c.a_k * phi.x, ac.y + c.a_k * phi.y);
        }
        if (c.last) {
          c.final_out[row] = make_double2(c.phase_re * accv.x - c.phase_im * accv.y,
                                          c.phase_re * accv.y + c.phase_im * accv.x);
        } else {
          c.prev[row] = phi;
          c.acc[row] = accv;
        }
      }
    }
  }
  if (a.cheb && a.ca.first && a.ca.want_partials) {
    if (lane == 0) {
      red[0][wave] = pn;
      red[1][wave] = pe;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      double sn = 0.0, se = 0.0;
      for (int w = 0; w < kThreads / 64; ++w) {
        sn += red[0][w];
        se += red[1][w];
      }
      a.partials[2 * blockIdx.x] = sn;
      a.partials[2 * blockIdx.x + 1] = se;
    }
  }
}

// Sums `n` pairs of partials in a fixed order; writes out[0..1].
__global__ __launch_bounds__(kThreads) void finalize_kernel(const double *partials, int n,
                                                            double *out) {
  __shared__ double s0[kThreads], s1[kThreads];
  double a = 0.0, b = 0.0;
  for (int i = threadIdx.x; i < n; i += kThreads) {
    a += partials[2 * i];
    b += partials[2 * i + 1];
  }
  s0[threadIdx.x] = a;
  s1[threadIdx.x] = b;
  __syncthreads();
  for (int w = kThreads / 2; w >= 1; w >>= 1) {
    if (threadIdx.x < w) {
      s0[threadIdx.x] += s0[threadIdx.x + w];
      s1[threadIdx.x] += s1[threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[0] = s0[0];
    out[1] = s1[0];
  }
}

// partials of <a|b> (complex), one pair per block
__global__ __launch_bounds__(kThreads) void dot_kernel(const double2 *x, const double2 *y,
                                                       int64_t n, double *partials) {
  __shared__ double s0[kThreads], s1[kThreads];
  double re = 0.0, im = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kThreads) {
    const double2 u = x[i], v = y[i];
    re += u.x * v.x + u.y * v.y;
    im += u.x * v.y - u.y * v.x;
  }
  s0[threadIdx.x] = re;
  s1[threadIdx.x] = im;
  __syncthreads();
  for (int w = kThreads / 2; w >= 1; w >>= 1) {
    if (threadIdx.x < w) {
      s0[threadIdx.x] += s0[threadIdx.x + w];
      s1[threadIdx.x] += s1[threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    partials[2 * blockIdx.x] = s0[0];
    partials[2 * blockIdx.x + 1] = s1[0];
  }
}

__global__ __launch_bounds__(kThreads) void axpby_kernel(int64_t n, double2 *y, const double2 *x,
                                                         double ar, double ai, double b) {
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kThreads) {
    const double2 u = x[i], v = y[i];
    y[i] = make_double2(ar * u.x - ai * u.y + b * v.x, ar * u.y + ai * u.x + b * v.y);
  }
}

}  // namespace

int sweep_lds_bytes(const sg_problem *p, sg_precision) {
  return (int)(2 * p->h.max_grid * (int64_t)sizeof(double2));
}

hipError_t launch_sweep(const sg_problem *p, const double2 *psi, sg_precision prec,
                        hipStream_t s) {
  SweepArgs a;
  a.terms = p->d_terms;
  a.sched = p->d_sched;
  a.mb = p->d_mb;
  a.psi = psi;
  a.tm = p->d_tm;
  a.tab = p->d_tables;
  a.cmat = p->d_c;
  a.kmat = p->d_k;
  a.td = p->h.tdesc;
  a.D = p->h.D;
  a.std_maps = (p->h.nbA == 1 && p->h.nbB == 2 && p->h.nqA == 2 && p->h.nqB == 2) ? 1 : 0;
  a.split = prec == SG_MIXED ? 1 : 0;
  a.max_grid = (int)p->h.max_grid;
  const int lds = sweep_lds_bytes(p, prec);
  if (lds > 65536) {
    hipError_t e = hipFuncSetAttribute((const void *)sweep_kernel,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, lds);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(sweep_kernel, dim3((unsigned)p->h.nterms), dim3(kThreads), lds, s, a);
  return hipGetLastError();
}

hipError_t launch_reduce(const sg_problem *p, Epi epi, const double2 *psi_in, double2 *out,
                         const ChebArgs *ca, hipStream_t s) {
  ReduceArgs a;
  a.ptr = p->d_inv_ptr;
  a.col = p->d_inv_col;
  a.tm = p->d_tm;
  a.h0 = p->d_h0;
  a.vin = psi_in;
  a.out = out;
  a.ncs = p->h.ncs;
  a.partials = p->d_partials;
  a.ca = ca ? *ca : ChebArgs{};
  a.cheb = epi == Epi::Cheb ? 1 : 0;
  const int64_t blocks = (p->h.ncs + 3) / 4;
  hipLaunchKernelGGL(reduce_kernel, dim3((unsigned)blocks), dim3(kThreads), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_finalize_partials(const sg_problem *p, hipStream_t s) {
  const int n = (int)((p->h.ncs + 3) / 4);
  hipLaunchKernelGGL(finalize_kernel, dim3(1), dim3(kThreads), 0, s,
                     (const double *)p->d_partials, n, p->d_result);
  return hipGetLastError();
}

hipError_t launch_dot(const sg_problem *p, const double2 *x, const double2 *y, hipStream_t s) {
  const int blocks = 256;
  hipLaunchKernelGGL(dot_kernel, dim3(blocks), dim3(kThreads), 0, s, x, y, p->h.ncs,
                     p->d_partials);
  hipLaunchKernelGGL(finalize_kernel, dim3(1), dim3(kThreads), 0, s,
                     (const double *)p->d_partials, blocks, p->d_result);
  return hipGetLastError();
}

hipError_t launch_axpby(int64_t n, double2 *y, const double2 *x, double ar, double ai, double b,
                        hipStream_t s) {
  int64_t blocks = (n + kThreads - 1) / kThreads;
  if (blocks > 4096) blocks = 4096;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(axpby_kernel, dim3((unsigned)blocks), dim3(kThreads), 0, s, n, y, x, ar,
                     ai, b);
  return hipGetLastError();
}

}  // namespace sg
