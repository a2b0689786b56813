// Vector kernels of the eigensolver (gfx950): block inner products with a
// fixed-order second stage (bitwise reproducible), block linear combinations,
// the diagonal (Davidson) correction and the basis embedding of the
// level-to-level restart.  All are HBM-bound streams over N_cs complex values.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "sg_internal.h"

namespace sg {

namespace {

constexpr int kBlasThreads = 256;
constexpr int kDotBlocks = 128;   // partial sums per inner product

template <typename T> using glb_p = __attribute__((address_space(1))) T *;

// partials[(j * kDotBlocks + b) * 2 + {0,1}] = sum over block b's share of
// conj(V_j[i]) w[i]   (V_j = V + j * ld)
__global__ __launch_bounds__(kBlasThreads) void multi_dot_kernel(const double2 *V, int64_t ld,
                                                                 const double2 *w, int64_t n,
                                                                 double *partials) {
  __shared__ double s0[kBlasThreads], s1[kBlasThreads];
  const int b = blockIdx.x, j = blockIdx.y;
  const glb_p<const double2> v = (glb_p<const double2>)(V + (size_t)j * ld);
  const glb_p<const double2> x = (glb_p<const double2>)w;
  double re = 0.0, im = 0.0;
  for (int64_t i = (int64_t)b * kBlasThreads + threadIdx.x; i < n;
       i += (int64_t)kDotBlocks * kBlasThreads) {
    const double vr = v[i].x, vi = v[i].y, xr = x[i].x, xi = x[i].y;
    re += vr * xr + vi * xi;
    im += vr * xi - vi * xr;
  }
  s0[threadIdx.x] = re;
  s1[threadIdx.x] = im;
  __syncthreads();
  for (int s = kBlasThreads / 2; s >= 1; s >>= 1) {
    if (threadIdx.x < s) {
      s0[threadIdx.x] += s0[threadIdx.x + s];
      s1[threadIdx.x] += s1[threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    partials[((size_t)j * kDotBlocks + b) * 2] = s0[0];
    partials[((size_t)j * kDotBlocks + b) * 2 + 1] = s1[0];
  }
}

// out[j] = sum_b partials[j][b], in block order (one thread per j)
__global__ void multi_dot_finish(const double *partials, int m, double *out) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= m) return;
  double re = 0.0, im = 0.0;
  for (int b = 0; b < kDotBlocks; ++b) {
    re += partials[((size_t)j * kDotBlocks + b) * 2];
    im += partials[((size_t)j * kDotBlocks + b) * 2 + 1];
  }
  out[2 * j] = re;
  out[2 * j + 1] = im;
}

// x[i] = beta x[i] + sum_j c_j V_j[i]   (c complex, j in order)
__global__ __launch_bounds__(kBlasThreads) void multi_axpy_kernel(double2 *x, double beta,
                                                                  const double2 *V, int64_t ld,
                                                                  int m, const double *c,
                                                                  int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * kBlasThreads + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kBlasThreads) {
    // beta = 0 overwrites x (which may hold anything)
    double re = beta == 0.0 ? 0.0 : beta * x[i].x, im = beta == 0.0 ? 0.0 : beta * x[i].y;
    for (int j = 0; j < m; ++j) {
      const double2 v = V[(size_t)j * ld + i];
      const double cr = c[2 * j], ci = c[2 * j + 1];
      re += cr * v.x - ci * v.y;
      im += cr * v.y + ci * v.x;
    }
    x[i] = make_double2(re, im);
  }
}

// t[i] = r[i] / (theta - d[i]), with |theta - d[i]| kept away from zero
__global__ __launch_bounds__(kBlasThreads) void precondition_kernel(double2 *t, const double2 *r,
                                                                    const double *d,
                                                                    double theta, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * kBlasThreads + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kBlasThreads) {
    double den = theta - d[i];
    if (fabs(den) < 1e-8) den = den < 0 ? -1e-8 : 1e-8;
    t[i] = make_double2(r[i].x / den, r[i].y / den);
  }
}

__global__ __launch_bounds__(kBlasThreads) void zero_kernel(double2 *y, int64_t ny) {
  for (int64_t i = (int64_t)blockIdx.x * kBlasThreads + threadIdx.x; i < ny;
       i += (int64_t)gridDim.x * kBlasThreads)
    y[i] = make_double2(0.0, 0.0);
}

__global__ __launch_bounds__(kBlasThreads) void scatter_kernel(const double2 *x,
                                                               const int32_t *map, int64_t nx,
                                                               double2 *y) {
  for (int64_t i = (int64_t)blockIdx.x * kBlasThreads + threadIdx.x; i < nx;
       i += (int64_t)gridDim.x * kBlasThreads)
    y[map[i]] = x[i];
}

int grid_for(int64_t n) {
  const int64_t b = (n + kBlasThreads - 1) / kBlasThreads;
  return (int)std::max<int64_t>(1, std::min<int64_t>(b, 4096));
}

// Lanczos on the device (no host round trip per Krylov vector).
// coef[j] = -sum_b partials[j][b] (block order, as multi_dot_finish) for
// j < m; alpha = (accumulate ? alpha : 0) + the real part of the last sum
__global__ void lanczos_project_kernel(const double *partials, int m, double *coef, double *alpha,
                                       int accumulate) {
  const int j = threadIdx.x;
  if (j >= m) return;
  double re = 0.0, im = 0.0;
  for (int b = 0; b < kDotBlocks; ++b) {
    re += partials[((size_t)j * kDotBlocks + b) * 2];
    im += partials[((size_t)j * kDotBlocks + b) * 2 + 1];
  }
  coef[2 * j] = -re;
  coef[2 * j + 1] = -im;
  if (j == m - 1) *alpha = (accumulate ? *alpha : 0.0) + re;
}

// x += sum_j c_j V_j (c complex, j in order), and npart[block] = the block's
// sum of |x_new|^2 (tree order)
__global__ __launch_bounds__(kBlasThreads) void multi_axpy_norm_kernel(double2 *x, const double2 *V,
                                                                       int64_t ld, int m,
                                                                       const double *c, int64_t n,
                                                                       double *npart) {
  __shared__ double s0[kBlasThreads];
  double acc = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * kBlasThreads + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kBlasThreads) {
    double re = x[i].x, im = x[i].y;
    for (int j = 0; j < m; ++j) {
      const double2 v = V[(size_t)j * ld + i];
      const double cr = c[2 * j], ci = c[2 * j + 1];
      re += cr * v.x - ci * v.y;
      im += cr * v.y + ci * v.x;
    }
    x[i] = make_double2(re, im);
    acc += re * re + im * im;
  }
  s0[threadIdx.x] = acc;
  __syncthreads();
  for (int s = kBlasThreads / 2; s >= 1; s >>= 1) {
    if (threadIdx.x < s) s0[threadIdx.x] += s0[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) npart[blockIdx.x] = s0[0];
}

// beta from multi_axpy_norm's block sums (fixed order), as lanczos_norm_kernel
__global__ __launch_bounds__(256) void lanczos_norm_partials_kernel(const double *npart, int nb,
                                                                    double *beta,
                                                                    const double *beta0,
                                                                    double thr, double *scale) {
  __shared__ double s0[256];
  double a = 0.0;
  for (int i = threadIdx.x; i < nb; i += 256) a += npart[i];
  s0[threadIdx.x] = a;
  __syncthreads();
  for (int s = 128; s >= 1; s >>= 1) {
    if (threadIdx.x < s) s0[threadIdx.x] += s0[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double b = sqrt(fmax(s0[0], 0.0));
    const bool keep = !(b < thr * beta0[0]);
    beta[0] = keep ? b : 0.0;
    scale[0] = keep ? 1.0 / b : 0.0;
  }
}

// beta = |w| from nrm2 = <w|w>, kept (scale = 1/beta) unless below
// thr * beta0 (beta0 null: unless zero); a dropped vector gets beta = 0 and
// scale 0, which zeroes it and every later Krylov vector
__global__ void lanczos_norm_kernel(const double *nrm2, double *beta, const double *beta0,
                                    double thr, double *scale) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const double b = sqrt(fmax(nrm2[0], 0.0));
  const bool keep = beta0 ? !(b < thr * beta0[0]) : b > 0.0;
  beta[0] = keep ? b : 0.0;
  scale[0] = keep ? 1.0 / b : 0.0;
}

// dst = scale[0] * src (dst may be src)
__global__ __launch_bounds__(kBlasThreads) void scale_copy_kernel(double2 *dst, const double2 *src,
                                                                  const double *scale, int64_t n) {
  const double c = scale[0];
  for (int64_t i = (int64_t)blockIdx.x * kBlasThreads + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kBlasThreads) {
    const double2 v = src[i];
    dst[i] = make_double2(c * v.x, c * v.y);
  }
}

// y = c0 x0 + c1 x1 (+ c2 x2 when x2 is not null), complex coefficients;
// y may be one of the x
__global__ __launch_bounds__(kBlasThreads) void comb3_kernel(int64_t n, double2 *y,
                                                             const double2 *x0, double2 c0,
                                                             const double2 *x1, double2 c1,
                                                             const double2 *x2, double2 c2) {
  for (int64_t i = (int64_t)blockIdx.x * kBlasThreads + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kBlasThreads) {
    const double2 u = x0[i], v = x1[i];
    double re = c0.x * u.x - c0.y * u.y + (c1.x * v.x - c1.y * v.y);
    double im = c0.x * u.y + c0.y * u.x + (c1.x * v.y + c1.y * v.x);
    if (x2) {
      const double2 w = x2[i];
      re += c2.x * w.x - c2.y * w.y;
      im += c2.x * w.y + c2.y * w.x;
    }
    y[i] = make_double2(re, im);
  }
}

// t = c x, then acc += t (one pass; the Taylor term and its sum)
__global__ __launch_bounds__(kBlasThreads) void scale_accumulate_kernel(int64_t n, double2 *t,
                                                                        const double2 *x,
                                                                        double2 c, double2 *acc) {
  for (int64_t i = (int64_t)blockIdx.x * kBlasThreads + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kBlasThreads) {
    const double2 u = x[i], a = acc[i];
    const double re = c.x * u.x - c.y * u.y, im = c.x * u.y + c.y * u.x;
    t[i] = make_double2(re, im);
    acc[i] = make_double2(a.x + re, a.y + im);
  }
}

}  // namespace

hipError_t launch_comb3(int64_t n, double2 *y, const double2 *x0, double2 c0, const double2 *x1,
                        double2 c1, const double2 *x2, double2 c2, hipStream_t s) {
  hipLaunchKernelGGL(comb3_kernel, dim3(grid_for(n)), dim3(kBlasThreads), 0, s, n, y, x0, c0, x1,
                     c1, x2, c2);
  return hipGetLastError();
}

hipError_t launch_scale_accumulate(int64_t n, double2 *t, const double2 *x, double2 c,
                                   double2 *acc, hipStream_t s) {
  hipLaunchKernelGGL(scale_accumulate_kernel, dim3(grid_for(n)), dim3(kBlasThreads), 0, s, n, t,
                     x, c, acc);
  return hipGetLastError();
}

hipError_t launch_lanczos_project(const double2 *V, int64_t ld, int m, const double2 *w,
                                  int64_t n, double *partials, double *coef, double *alpha,
                                  bool accumulate, hipStream_t s) {
  if (m < 1 || m > 64) return hipErrorInvalidValue;
  hipLaunchKernelGGL(multi_dot_kernel, dim3(kDotBlocks, m), dim3(kBlasThreads), 0, s, V, ld, w, n,
                     partials);
  hipLaunchKernelGGL(lanczos_project_kernel, dim3(1), dim3(64), 0, s, (const double *)partials, m,
                     coef, alpha, accumulate ? 1 : 0);
  return hipGetLastError();
}

int lanczos_norm_partials() { return 4096; }

hipError_t launch_multi_axpy_norm(double2 *x, const double2 *V, int64_t ld, int m,
                                  const double *c, int64_t n, double *npart, hipStream_t s) {
  hipLaunchKernelGGL(multi_axpy_norm_kernel, dim3(grid_for(n)), dim3(kBlasThreads), 0, s, x, V,
                     ld, m, c, n, npart);
  return hipGetLastError();
}

hipError_t launch_lanczos_norm_partials(const double *npart, int64_t n, double *beta,
                                        const double *beta0, double thr, double *scale,
                                        hipStream_t s) {
  hipLaunchKernelGGL(lanczos_norm_partials_kernel, dim3(1), dim3(256), 0, s, npart, grid_for(n),
                     beta, beta0, thr, scale);
  return hipGetLastError();
}

hipError_t launch_lanczos_norm(const double *nrm2, double *beta, const double *beta0, double thr,
                               double *scale, hipStream_t s) {
  hipLaunchKernelGGL(lanczos_norm_kernel, dim3(1), dim3(64), 0, s, nrm2, beta, beta0, thr, scale);
  return hipGetLastError();
}

int dot_partials_per_vector() { return kDotBlocks; }

hipError_t launch_multi_dot(const double2 *V, int64_t ld, int m, const double2 *w, int64_t n,
                            double *partials, double *out, hipStream_t s) {
  if (m <= 0) return hipSuccess;
  hipLaunchKernelGGL(multi_dot_kernel, dim3(kDotBlocks, m), dim3(kBlasThreads), 0, s, V, ld, w, n,
                     partials);
  hipLaunchKernelGGL(multi_dot_finish, dim3((m + 63) / 64), dim3(64), 0, s,
                     (const double *)partials, m, out);
  return hipGetLastError();
}

hipError_t launch_multi_axpy(double2 *x, double beta, const double2 *V, int64_t ld, int m,
                             const double *c, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(multi_axpy_kernel, dim3(grid_for(n)), dim3(kBlasThreads), 0, s, x, beta, V,
                     ld, m, c, n);
  return hipGetLastError();
}

hipError_t launch_precondition(double2 *t, const double2 *r, const double *d, double theta,
                               int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(precondition_kernel, dim3(grid_for(n)), dim3(kBlasThreads), 0, s, t, r, d,
                     theta, n);
  return hipGetLastError();
}

hipError_t launch_scale_copy(double2 *dst, const double2 *src, const double *scale, int64_t n,
                             hipStream_t s) {
  hipLaunchKernelGGL(scale_copy_kernel, dim3(grid_for(n)), dim3(kBlasThreads), 0, s, dst, src,
                     scale, n);
  return hipGetLastError();
}

hipError_t launch_zero(double2 *y, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(zero_kernel, dim3(grid_for(n)), dim3(kBlasThreads), 0, s, y, n);
  return hipGetLastError();
}

hipError_t launch_embed(const double2 *x, const int32_t *map, int64_t nx, double2 *y, int64_t ny,
                        hipStream_t s) {
  hipLaunchKernelGGL(zero_kernel, dim3(grid_for(ny)), dim3(kBlasThreads), 0, s, y, ny);
  hipLaunchKernelGGL(scatter_kernel, dim3(grid_for(nx)), dim3(kBlasThreads), 0, s, x, map, nx, y);
  return hipGetLastError();
}

}  // namespace sg
