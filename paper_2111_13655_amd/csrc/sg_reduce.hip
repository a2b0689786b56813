// HIP kernels of the fixed-order scatter-add (the last step of Alg. 1) and the
// small vector kernels of the propagator, for gfx950 (MI355X).
//
// The scatter-add is done as a gather: every compact index sums its
// term-major contributions through the inverse of M^B in a fixed order (lane
// groups of 8 for short rows, a whole wavefront for long ones), so results
// are bitwise reproducible.  The Chebyshev recurrence and the norm/energy
// partial sums are fused into its epilogue.
#include "sg_internal.h"

namespace sg {

namespace {

constexpr int kRedThreads = 256;
constexpr int kShortLanes = 8;

struct ReduceArgs {
  const int32_t *ptr;
  const int32_t *col;
  const int32_t *rows;     // long rows first, then short rows
  const double2 *tm;
  const double *h0;
  const double2 *vin;
  double2 *out;
  int64_t ncs;
  int64_t nlong;
  double *partials;
  ChebArgs ca;
  int cheb;
};

// Sum of tm[col[j]] for j = b + sub, b + sub + G, ... < e, in increasing j.
// Four index loads and then four value loads are issued before any add, so a
// long row waits for one memory round trip per four entries, not per entry.
template <int G>
__device__ __forceinline__ void strided_sum(const int32_t *__restrict__ col,
                                            const double2 *__restrict__ tm, int b, int e,
                                            int sub, double *sr, double *si) {
  int j = b + sub;
  for (; j + 3 * G < e; j += 4 * G) {
    const int c0 = col[j], c1 = col[j + G], c2 = col[j + 2 * G], c3 = col[j + 3 * G];
    const double2 v0 = tm[c0], v1 = tm[c1], v2 = tm[c2], v3 = tm[c3];
    *sr += v0.x; *si += v0.y;
    *sr += v1.x; *si += v1.y;
    *sr += v2.x; *si += v2.y;
    *sr += v3.x; *si += v3.y;
  }
  for (; j < e; j += G) {
    const double2 v = tm[col[j]];
    *sr += v.x;
    *si += v.y;
  }
}

template <int G>
__device__ __forceinline__ double group_sum(double v) {
#pragma unroll
  for (int m = G / 2; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
  return v;
}

__device__ __forceinline__ void row_epilogue(const ReduceArgs &a, int64_t row, double sr,
                                             double si, double *pn, double *pe) {
  const double2 vk = a.vin[row];
  if (a.ca.split) {
    const double d = a.h0[row];
    sr = fma(d, vk.x, sr);
    si = fma(d, vk.y, si);
  }
  if (!a.cheb) {
    a.out[row] = make_double2(sr, si);
    return;
  }
  const ChebArgs &c = a.ca;
  const double zr = (sr - c.ebar * vk.x) * c.inv_half;
  const double zi = (si - c.ebar * vk.y) * c.inv_half;
  double2 phi, accv;
  if (c.first) {
    phi = make_double2(zi, -zr);  // -i z
    accv = make_double2(c.a_0 * vk.x + c.a_k * phi.x, c.a_0 * vk.y + c.a_k * phi.y);
    *pn = vk.x * vk.x + vk.y * vk.y;
    *pe = vk.x * sr + vk.y * si;  // Re(conj(psi) H psi)
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

// step 5 (second half): compact[r] = sum of its term-major contributions
__global__ __launch_bounds__(kRedThreads) void reduce_kernel(ReduceArgs a) {
  __shared__ double red[2][kRedThreads / 64];
  const int wave = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
  const int64_t gw = (int64_t)blockIdx.x * (kRedThreads / 64) + wave;
  double pn = 0.0, pe = 0.0;
  if (gw < a.nlong) {
    const int64_t row = a.rows[gw];
    const int b = a.ptr[row], e = a.ptr[row + 1];
    double sr = 0.0, si = 0.0;
    strided_sum<64>(a.col, a.tm, b, e, lane, &sr, &si);
    sr = group_sum<64>(sr);
    si = group_sum<64>(si);
    if (lane == 0) row_epilogue(a, row, sr, si, &pn, &pe);
  } else {
    const int64_t sidx = (gw - a.nlong) * (64 / kShortLanes) + lane / kShortLanes;
    const int sub = lane % kShortLanes;
    const bool valid = a.nlong + sidx < a.ncs;
    double sr = 0.0, si = 0.0;
    int64_t row = 0;
    if (valid) {
      row = a.rows[a.nlong + sidx];
      const int b = a.ptr[row], e = a.ptr[row + 1];
      strided_sum<kShortLanes>(a.col, a.tm, b, e, sub, &sr, &si);
    }
    sr = group_sum<kShortLanes>(sr);
    si = group_sum<kShortLanes>(si);
    if (valid && sub == 0) row_epilogue(a, row, sr, si, &pn, &pe);
  }
  if (a.cheb && a.ca.first && a.ca.want_partials) {
    pn = group_sum<64>(pn);
    pe = group_sum<64>(pe);
    if (lane == 0) {
      red[0][wave] = pn;
      red[1][wave] = pe;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      double sn = 0.0, se = 0.0;
      for (int w = 0; w < kRedThreads / 64; ++w) {
        sn += red[0][w];
        se += red[1][w];
      }
      a.partials[2 * blockIdx.x] = sn;
      a.partials[2 * blockIdx.x + 1] = se;
    }
  }
}

// Sums `n` pairs of partials in a fixed order; writes out[0..1].
__global__ __launch_bounds__(256) void finalize_kernel(const double *partials, int n,
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

int64_t reduce_blocks(const sg_problem *p) {
  const int64_t nshort = p->h.ncs - p->h.n_long_rows;
  const int64_t waves = p->h.n_long_rows + (nshort + (64 / kShortLanes) - 1) / (64 / kShortLanes);
  return (waves + (kRedThreads / 64) - 1) / (kRedThreads / 64);
}

hipError_t launch_reduce(const sg_problem *p, Epi epi, const double2 *psi_in, double2 *out,
                         const ChebArgs *ca, hipStream_t s) {
  ReduceArgs a;
  a.ptr = p->d_inv_ptr;
  a.col = p->d_inv_col;
  a.rows = p->d_rows;
  a.tm = p->d_tm;
  a.h0 = p->d_h0;
  a.vin = psi_in;
  a.out = out;
  a.ncs = p->h.ncs;
  a.nlong = p->h.n_long_rows;
  a.partials = p->d_partials;
  a.ca = ca ? *ca : ChebArgs{};
  a.cheb = epi == Epi::Cheb ? 1 : 0;
  hipLaunchKernelGGL(reduce_kernel, dim3((unsigned)reduce_blocks(p)), dim3(kRedThreads), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_finalize_partials(const sg_problem *p, hipStream_t s) {
  const int n = (int)reduce_blocks(p);
  hipLaunchKernelGGL(finalize_kernel, dim3(1), dim3(256), 0, s, (const double *)p->d_partials, n,
                     p->d_result);
  return hipGetLastError();
}

hipError_t launch_dot(const sg_problem *p, const double2 *x, const double2 *y, hipStream_t s) {
  const int blocks = 256;
  hipLaunchKernelGGL(dot_kernel, dim3(blocks), dim3(256), 0, s, x, y, p->h.ncs, p->d_partials);
  hipLaunchKernelGGL(finalize_kernel, dim3(1), dim3(256), 0, s, (const double *)p->d_partials,
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
