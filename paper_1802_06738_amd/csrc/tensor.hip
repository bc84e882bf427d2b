// Layout kernels: strided 4-index permutation with accumulate, axpby, fill, casts.
// All are HBM-bound grid-stride loops; consecutive threads write consecutive
// output elements.
#include <algorithm>

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

// The same permutation when the output's innermost axis L (unit output stride) is not the
// input's unit-stride axis K: 32 x 32 tiles over (K, L) pass through LDS, read with lanes
// along K and written with lanes along L, so both sides move contiguous row segments.  The
// other two axes U, W and the batch are enumerated by blockIdx.y (grid-stride).
template <typename I>
__global__ __launch_bounds__(256) void permute4_tiled_kernel(Perm4 p, int K, int L, int U, int W, double alpha,
                                                             const double* __restrict__ in, double beta,
                                                             double* __restrict__ out, I nrest) {
  __shared__ double tile[32][33];
  const I dK = (I)p.d[K], dL = (I)p.d[L], dU = (I)p.d[U], dW = (I)p.d[W];
  const I ntl = (dL + 31) / 32;
  const I k0 = (I)(blockIdx.x / ntl) * 32, l0 = (I)(blockIdx.x % ntl) * 32;
  const int tx = threadIdx.x % 32, ty = threadIdx.x / 32;  // 32 x 8
  for (I rest = blockIdx.y; rest < nrest; rest += gridDim.y) {
    const I iw = rest % dW;
    const I t = rest / dW;
    const I iu = t % dU;
    const I q = t / dU;
    const int64_t ib = (int64_t)q * p.ibs + (int64_t)iu * p.is[U] + (int64_t)iw * p.is[W];
    const int64_t ob = (int64_t)q * p.obs + (int64_t)iu * p.os[U] + (int64_t)iw * p.os[W];
    for (int l = ty; l < 32; l += 8) {
      const I ik = k0 + tx, il = l0 + l;
      if (ik < dK && il < dL) tile[l][tx] = in[ib + (int64_t)ik * p.is[K] + (int64_t)il * p.is[L]];
    }
    __syncthreads();
    for (int kk = ty; kk < 32; kk += 8) {
      const I ik = k0 + kk, il = l0 + tx;
      if (ik < dK && il < dL) {
        double* y = out + ob + (int64_t)ik * p.os[K] + (int64_t)il * p.os[L];
        double val = alpha * tile[tx][kk];
        if (beta != 0.0) val += beta * (*y);
        *y = val;
      }
    }
    __syncthreads();
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
  // tiled path: L = innermost output axis of extent > 1 (unit output stride), K = an axis
  // of unit input stride, both at least 8 long
  int L = -1, K = -1;
  for (int k = 3; k >= 0; --k)
    if (p.d[k] > 1) { L = k; break; }
  if (L >= 0 && p.os[L] == 1 && p.is[L] != 1)
    for (int k = 0; k < 4; ++k)
      if (k != L && p.d[k] > 1 && p.is[k] == 1) K = k;
  if (L >= 0 && K >= 0 && p.d[L] >= 8 && p.d[K] >= 8) {
    int rest_ax[2], nr = 0;
    for (int k = 0; k < 4; ++k)
      if (k != K && k != L) rest_ax[nr++] = k;
    const int U = rest_ax[0], W = rest_ax[1];
    const int64_t nrest = p.nb * p.d[U] * p.d[W];
    const int64_t tiles = ((p.d[K] + 31) / 32) * ((p.d[L] + 31) / 32);
    if (tiles <= 0x7fffffff) {
      const unsigned gy = (unsigned)std::min<int64_t>(nrest, 65535);
      if (total < (1ll << 31))
        hipLaunchKernelGGL(permute4_tiled_kernel<uint32_t>, dim3((unsigned)tiles, gy), dim3(256), 0, s, p, K, L, U, W,
                           alpha, in, beta, out, (uint32_t)nrest);
      else
        hipLaunchKernelGGL(permute4_tiled_kernel<int64_t>, dim3((unsigned)tiles, gy), dim3(256), 0, s, p, K, L, U, W,
                           alpha, in, beta, out, nrest);
      PNO_HIP(hipGetLastError());
      return;
    }
  }
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
