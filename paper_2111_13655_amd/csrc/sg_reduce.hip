// HIP kernels of the fixed-order scatter-add (the last step of Alg. 1) and the
// small vector kernels of the propagator, for gfx950 (MI355X).
//
// The scatter-add is done as a gather: every compact index sums its
// term-major contributions through the inverse of M^B in a fixed order (a
// whole wavefront for a long row, a group of 8 lanes for each of 8 short
// rows).  Term positions are lexicographic like the compact basis, so the
// contributions of neighbouring rows to one term are neighbours in memory.
// Results are bitwise reproducible and independent of which other instances
// share the launch.  The exact FP64 diagonal of the split operator, the Chebyshev
// recurrence, the series accumulation and the norm / energy partial sums are
// fused into the epilogue.
#include <hip/hip_ext.h>

#include "sg_internal.h"

namespace sg {

namespace {

constexpr int kRedThreads = 256;

template <typename T> using glb_p = __attribute__((address_space(1))) T *;
template <typename T> using cptr = const __attribute__((address_space(4))) T *;

struct alignas(16) Z64 { double x, y; };
template <typename P>
__device__ __forceinline__ Z64 ldz(P p) {
  Z64 v;
  v.x = p->x;
  v.y = p->y;
  return v;
}
template <typename P>
__device__ __forceinline__ void stz(P p, double x, double y) {
  p->x = x;
  p->y = y;
}

struct ReduceArgs {
  cptr<InstDev> inst;
  cptr<RedItem> items;
  int64_t nitems;
  double2 *x0o, *x1o;
  int mode;            // 0 apply, 1 Chebyshev
  int k;               // Chebyshev term produced (1..K-1)
  int want_partials;   // k == 1: norm / energy partial sums
  int split;           // add the exact diagonal part
};

// Sum of tm[col[j]] for j = b + sub, b + sub + G, ... < e, in increasing j.
// Rounds of U entries per lane: U index loads, then U value loads, then the
// adds, so that a row of up to U*G entries costs one dependent pair of loads.
template <int G, int U>
__device__ __forceinline__ void strided_sum(glb_p<const int32_t> col, glb_p<const Z64> tm, int b,
                                            int e, int sub, double *sr, double *si) {
  for (int j = b + sub; j < e; j += U * G) {
    int c[U];
#pragma unroll
    for (int u = 0; u < U; ++u) c[u] = j + u * G < e ? col[j + u * G] : 0;
    Z64 v[U];
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (j + u * G < e) v[u] = ldz(tm + c[u]);
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (j + u * G < e) {
        *sr += v[u].x;
        *si += v[u].y;
      }
    }
  }
}

template <int G>
__device__ __forceinline__ double group_sum(double v) {
#pragma unroll
  for (int m = G / 2; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
  return v;
}

// The row's epilogue inputs, loaded before its sum so that their latency
// overlaps it.
struct RowIn {
  Z64 vk;     // the vector H acts on
  double d;   // exact diagonal (split form)
  Z64 pr;     // phi_{k-2}
  Z64 ac;     // running series sum
};

__device__ __forceinline__ RowIn row_inputs(const ReduceArgs &a, cptr<InstDev> I, int64_t row) {
  RowIn in{};
  double2 *x0 = a.x0o ? a.x0o + I->vec_off : I->x0;
  double2 *x1 = a.x1o ? a.x1o + I->vec_off : I->x1;
  const double2 *vin = (a.mode == 0) ? x0 : (((a.k - 1) & 1) ? x1 : x0);
  in.vk = ldz((glb_p<const Z64>)vin + row);
  in.d = a.split ? ((glb_p<const double>)I->h0)[row] : 0.0;
  if (a.mode == 1 && a.k > 1) {
    const double2 *prev = (a.k & 1) ? x1 : x0;
    in.pr = ldz((glb_p<const Z64>)prev + row);
    in.ac = ldz((glb_p<const Z64>)I->acc + row);
  }
  return in;
}

// Row epilogue: (H psi)[row] = s (+ exact diagonal), then either the plain
// output or one Chebyshev recurrence step phi_k = -2i Hs phi_{k-1} + phi_{k-2}
// (phi_1 = -i Hs phi_0), acc += a_k phi_k, and on the last term
// psi <- exp(-i Ebar dt) acc.
__device__ __forceinline__ void row_epilogue(const ReduceArgs &a, cptr<InstDev> I, int64_t row,
                                             const RowIn &in, double sr, double si, double *pn,
                                             double *pe) {
  double2 *x0 = a.x0o ? a.x0o + I->vec_off : I->x0;
  double2 *x1 = a.x1o ? a.x1o + I->vec_off : I->x1;
  const Z64 vk = in.vk;
  if (a.split) {
    sr = fma(in.d, vk.x, sr);
    si = fma(in.d, vk.y, si);
  }
  if (a.mode == 0) {
    stz((glb_p<Z64>)x1 + row, sr, si);
    return;
  }
  double2 *prev = (a.k & 1) ? x1 : x0;   // phi_{k-2} in, phi_k out
  const double zr = (sr - I->ebar * vk.x) * I->inv_half;
  const double zi = (si - I->ebar * vk.y) * I->inv_half;
  const double ak = I->cheb_a[a.k];
  double phx, phy, acx, acy;
  if (a.k == 1) {
    const double a0 = I->cheb_a[0];
    phx = zi;                              // -i z
    phy = -zr;
    acx = a0 * vk.x + ak * phx;
    acy = a0 * vk.y + ak * phy;
    *pn = vk.x * vk.x + vk.y * vk.y;
    *pe = vk.x * sr + vk.y * si;           // Re(conj(psi) H psi)
  } else {
    phx = 2.0 * zi + in.pr.x;              // -2i z + phi_{k-2}
    phy = -2.0 * zr + in.pr.y;
    acx = in.ac.x + ak * phx;
    acy = in.ac.y + ak * phy;
  }
  if (a.k == I->K - 1) {
    stz((glb_p<Z64>)x0 + row, I->phase_re * acx - I->phase_im * acy,
        I->phase_re * acy + I->phase_im * acx);
  } else {
    stz((glb_p<Z64>)prev + row, phx, phy);
    stz((glb_p<Z64>)I->acc + row, acx, acy);
  }
}

// Workgroups are dealt to the eight XCDs in turn (workgroup i to XCD i mod
// 8).  The item groups are renumbered so that each XCD takes a contiguous run:
// neighbouring rows, whose contributions share cache lines, then meet in one
// L2.  A bijection on [0, nb).
constexpr int kXcds = 8;
__device__ __forceinline__ int64_t xcd_block(int64_t b, int64_t nb) {
  const int64_t x = b % kXcds, q = nb / kXcds, r = nb % kXcds;
  return (x < r ? x * (q + 1) : r * (q + 1) + (x - r) * q) + b / kXcds;
}

// step 5 (second half): compact[r] = sum of its term-major contributions
__global__ __launch_bounds__(kRedThreads) void reduce_kernel(ReduceArgs a) {
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int64_t gw = xcd_block(blockIdx.x, gridDim.x) * (kRedThreads / 64) + wave;
  if (gw >= a.nitems) return;
  const cptr<RedItem> it = a.items + gw;
  const int chunk = it->chunk;
  const int nch = (chunk >> 12) & 0xfff;   // long rows: chunks of the row; short rows: 0
  const glb_p<const int32_t> rowp = (glb_p<const int32_t>)it->rows;
  const glb_p<const int32_t> ptrp = (glb_p<const int32_t>)it->ptr;
  // the item's row and bounds load alongside the instance record (both
  // operands of the test are read, so that neither load waits on the other)
  const cptr<InstDev> I = a.inst + it->inst;
  const bool skip = (I->active == 0) | ((a.mode == 1) & (a.k > I->K - 1));
  // long rows: one row for the workgroup; short rows: one per lane group
  int lrow = 0, lb = 0, le = 0, row = 0, b = 0, e = 0;
  const int r = lane / kShortLanes;
  const bool valid = nch || r < chunk;
  if (nch) {
    lrow = __builtin_amdgcn_readfirstlane(rowp[0]);
    lb = __builtin_amdgcn_readfirstlane(ptrp[0]);
    le = __builtin_amdgcn_readfirstlane(ptrp[1]);
  } else if (valid) {
    row = rowp[r];
    b = ptrp[r];
    e = ptrp[r + 1];
  }
  if (skip) return;
  const glb_p<const Z64> tm = (glb_p<const Z64>)I->tm;
  const glb_p<const int32_t> col = (glb_p<const int32_t>)I->inv_col;
  double pn = 0.0, pe = 0.0;
  if (nch) {
    // a long row on the whole workgroup: wavefront `sub` sums the sub-th of
    // kRowWaves consecutive runs of its entries, the run sums are added in
    // wavefront order through LDS
    __shared__ double wsum[2][kRowWaves];
    const int sub = chunk >> 24;
    row = lrow;
    b = lb;
    e = le;
    RowIn in{};
    if (sub == 0) in = row_inputs(a, I, row);
    const int run = max(kRowRun, (e - b + kRowWaves - 1) / kRowWaves);
    const int cb = min(e, b + sub * run);
    double sr = 0.0, si = 0.0;
    strided_sum<64, 8>(col, tm, cb, min(e, cb + run), lane, &sr, &si);
    sr = group_sum<64>(sr);
    si = group_sum<64>(si);
    if (lane == 0) {
      wsum[0][sub] = sr;
      wsum[1][sub] = si;
    }
    __syncthreads();
    if (sub == 0) {
      sr = wsum[0][0];
      si = wsum[1][0];
#pragma unroll
      for (int w = 1; w < kRowWaves; ++w) {
        sr += wsum[0][w];
        si += wsum[1][w];
      }
      if (lane == 0) row_epilogue(a, I, row, in, sr, si, &pn, &pe);
    }
  } else {
    const int sub = lane % kShortLanes;
    double sr = 0.0, si = 0.0;
    RowIn in{};
    if (valid) {
      in = row_inputs(a, I, row);
      strided_sum<kShortLanes, kLongRow / kShortLanes>(col, tm, b, e, sub, &sr, &si);
    }
    sr = group_sum<kShortLanes>(sr);
    si = group_sum<kShortLanes>(si);
    if (valid && sub == 0) row_epilogue(a, I, row, in, sr, si, &pn, &pe);
  }
  if (a.mode == 1 && a.k == 1 && a.want_partials) {
    pn = group_sum<64>(pn);
    pe = group_sum<64>(pe);
    if (lane == 0) {
      I->partials[2 * it->local] = pn;
      I->partials[2 * it->local + 1] = pe;
    }
  }
}

// One block per instance: sums its item partials in a fixed order.
__global__ __launch_bounds__(256) void finalize_kernel(const InstDev *inst) {
  __shared__ double s0[256], s1[256];
  const InstDev *I = inst + blockIdx.x;
  if (!I->active) return;
  // each thread adds its items in increasing order; the loads of eight are
  // issued before their adds
  double a = 0.0, b = 0.0;
  const int n = I->nitems;
  for (int i0 = threadIdx.x; i0 < n; i0 += 8 * 256) {
    double va[8], vb[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int i = i0 + u * 256;
      va[u] = i < n ? I->partials[2 * i] : 0.0;
      vb[u] = i < n ? I->partials[2 * i + 1] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      if (i0 + u * 256 < n) {
        a += va[u];
        b += vb[u];
      }
    }
  }
  s0[threadIdx.x] = a;
  s1[threadIdx.x] = b;
  __syncthreads();
  for (int w = 128; w >= 1; w >>= 1) {
    if (threadIdx.x < w) {
      s0[threadIdx.x] += s0[threadIdx.x + w];
      s1[threadIdx.x] += s1[threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    I->result[0] = s0[0];
    I->result[1] = s1[0];
  }
}

// Sums n pairs of partials in a fixed order; writes out[0..1].
__global__ __launch_bounds__(256) void sum_pairs_kernel(const double *partials, int n,
                                                        double *out) {
  __shared__ double s0[256], s1[256];
  double a = 0.0, b = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) {
    a += partials[2 * i];
    b += partials[2 * i + 1];
  }
  s0[threadIdx.x] = a;
  s1[threadIdx.x] = b;
  __syncthreads();
  for (int w = 128; w >= 1; w >>= 1) {
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

// partials of <x|y> (complex), one pair per block
__global__ __launch_bounds__(256) void dot_kernel(const double2 *x, const double2 *y, int64_t n,
                                                  double *partials) {
  __shared__ double s0[256], s1[256];
  double re = 0.0, im = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    const double2 u = x[i], v = y[i];
    re += u.x * v.x + u.y * v.y;
    im += u.x * v.y - u.y * v.x;
  }
  s0[threadIdx.x] = re;
  s1[threadIdx.x] = im;
  __syncthreads();
  for (int w = 128; w >= 1; w >>= 1) {
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

__global__ __launch_bounds__(256) void axpby_kernel(int64_t n, double2 *y, const double2 *x,
                                                    double ar, double ai, double b) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    const double2 u = x[i], v = y[i];
    y[i] = make_double2(ar * u.x - ai * u.y + b * v.x, ar * u.y + ai * u.x + b * v.y);
  }
}

}  // namespace

hipError_t launch_reduce(const Plan *pl, const LaunchCtl &c, hipStream_t s) {
  ReduceArgs a;
  a.inst = (cptr<InstDev>)pl->d_inst;
  a.items = (cptr<RedItem>)pl->d_items;
  a.nitems = (int64_t)pl->items.size();
  a.x0o = c.x0o;
  a.x1o = c.x1o;
  a.mode = c.mode == Mode::Cheb ? 1 : 0;
  a.k = c.k;
  a.want_partials = c.want_partials;
  a.split = split_form(pl, c.prec) ? 1 : 0;
  const int64_t blocks = (a.nitems + (kRedThreads / 64) - 1) / (kRedThreads / 64);
  if (blocks == 0) return hipSuccess;
  if (c.ev0 || c.ev1)
    hipExtLaunchKernelGGL(reduce_kernel, dim3((unsigned)blocks), dim3(kRedThreads), 0, s, c.ev0,
                          c.ev1, 0, a);
  else
    hipLaunchKernelGGL(reduce_kernel, dim3((unsigned)blocks), dim3(kRedThreads), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_finalize(const Plan *pl, hipStream_t s) {
  if (pl->inst.empty()) return hipSuccess;
  hipLaunchKernelGGL(finalize_kernel, dim3((unsigned)pl->inst.size()), dim3(256), 0, s,
                     (const InstDev *)pl->d_inst);
  return hipGetLastError();
}

hipError_t launch_dot(const sg_problem *p, const double2 *x, const double2 *y, hipStream_t s) {
  const int blocks = 256;
  hipLaunchKernelGGL(dot_kernel, dim3(blocks), dim3(256), 0, s, x, y, p->h.ncs, p->d_partials);
  hipLaunchKernelGGL(sum_pairs_kernel, dim3(1), dim3(256), 0, s, (const double *)p->d_partials,
                     blocks, p->d_result);
  return hipGetLastError();
}

hipError_t launch_axpby(int64_t n, double2 *y, const double2 *x, double ar, double ai, double b,
                        hipStream_t s) {
  int64_t blocks = (n + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(axpby_kernel, dim3((unsigned)blocks), dim3(256), 0, s, n, y, x, ar, ai, b);
  return hipGetLastError();
}

}  // namespace sg
