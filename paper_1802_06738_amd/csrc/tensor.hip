// Layout kernels: strided 4-index permutation with accumulate, axpby, fill, casts.
// All are HBM-bound grid-stride loops; consecutive threads write consecutive
// output elements.
#include "common.h"

namespace pnoeom {
namespace {

template <typename I>
__global__ void permute4_kernel(Perm4 p, double alpha, const double* __restrict__ in, double beta,
                                double* __restrict__ out, I per, I total) {
  const I d1 = (I)p.d[1], d2 = (I)p.d[2], d3 = (I)p.d[3];
  for (I e = blockIdx.x * (I)blockDim.x + threadIdx.x; e < total; e += (I)gridDim.x * blockDim.x) {
    const I q = e / per;
    I r = e - q * per;
    const I i3 = r % d3; r /= d3;
    const I i2 = r % d2; r /= d2;
    const I i1 = r % d1;
    const I i0 = r / d1;
    const double x = in[q * p.ibs + i0 * p.is[0] + i1 * p.is[1] + i2 * p.is[2] + i3 * p.is[3]];
    double* y = out + (q * p.obs + i0 * p.os[0] + i1 * p.os[1] + i2 * p.os[2] + i3 * p.os[3]);
    double val = alpha * x;
    if (beta != 0.0) val += beta * (*y);
    *y = val;
  }
}

__global__ void axpby_kernel(int64_t n, double alpha, const double* __restrict__ x, double beta,
                             double* __restrict__ y) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
    double val = alpha * x[e];
    if (beta != 0.0) val += beta * y[e];
    y[e] = val;
  }
}

__global__ void fill_kernel(int64_t n, double val, double* __restrict__ y) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
    y[e] = val;
}

__global__ void to_float_kernel(int64_t n, const double* __restrict__ x, float* __restrict__ y) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
    y[e] = (float)x[e];
}

__global__ void to_double_kernel(int64_t n, const float* __restrict__ x, double* __restrict__ y, double beta) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
    double val = (double)x[e];
    if (beta != 0.0) val += beta * y[e];
    y[e] = val;
  }
}

unsigned grid_for(int64_t n) {
  int64_t b = (n + 255) / 256;
  if (b > 65536) b = 65536;
  if (b < 1) b = 1;
  return (unsigned)b;
}

}  // namespace

void permute4(hipStream_t s, const Perm4& p, double alpha, const double* in, double beta, double* out) {
  const int64_t per = p.d[0] * p.d[1] * p.d[2] * p.d[3];
  const int64_t total = per * p.nb;
  if (total == 0) return;
  // 32-bit index arithmetic when the element count allows it (integer division is
  // the cost of this kernel besides the HBM traffic)
  if (total < (1ll << 31))
    hipLaunchKernelGGL(permute4_kernel<uint32_t>, dim3(grid_for(total)), dim3(256), 0, s, p, alpha, in, beta, out,
                       (uint32_t)per, (uint32_t)total);
  else
    hipLaunchKernelGGL(permute4_kernel<int64_t>, dim3(grid_for(total)), dim3(256), 0, s, p, alpha, in, beta, out,
                       per, total);
  PNO_HIP(hipGetLastError());
}

void permute_c(hipStream_t s, const int64_t in_dims[4], const int perm[4], double alpha, const double* in,
               double beta, double* out, int64_t nb) {
  int64_t in_str[4];
  in_str[3] = 1;
  for (int k = 2; k >= 0; --k) in_str[k] = in_str[k + 1] * in_dims[k + 1];
  Perm4 p;
  for (int k = 0; k < 4; ++k) {
    p.d[k] = in_dims[perm[k]];
    p.is[k] = in_str[perm[k]];
  }
  p.os[3] = 1;
  for (int k = 2; k >= 0; --k) p.os[k] = p.os[k + 1] * p.d[k + 1];
  p.nb = nb;
  p.ibs = p.obs = in_dims[0] * in_dims[1] * in_dims[2] * in_dims[3];
  permute4(s, p, alpha, in, beta, out);
}

void axpby(hipStream_t s, int64_t n, double alpha, const double* x, double beta, double* y) {
  if (n == 0) return;
  hipLaunchKernelGGL(axpby_kernel, dim3(grid_for(n)), dim3(256), 0, s, n, alpha, x, beta, y);
  PNO_HIP(hipGetLastError());
}

void fill(hipStream_t s, int64_t n, double val, double* y) {
  if (n == 0) return;
  hipLaunchKernelGGL(fill_kernel, dim3(grid_for(n)), dim3(256), 0, s, n, val, y);
  PNO_HIP(hipGetLastError());
}

void to_float(hipStream_t s, int64_t n, const double* x, float* y) {
  if (n == 0) return;
  hipLaunchKernelGGL(to_float_kernel, dim3(grid_for(n)), dim3(256), 0, s, n, x, y);
  PNO_HIP(hipGetLastError());
}

void to_double(hipStream_t s, int64_t n, const float* x, double* y, double beta) {
  if (n == 0) return;
  hipLaunchKernelGGL(to_double_kernel, dim3(grid_for(n)), dim3(256), 0, s, n, x, y, beta);
  PNO_HIP(hipGetLastError());
}

}  // namespace pnoeom
