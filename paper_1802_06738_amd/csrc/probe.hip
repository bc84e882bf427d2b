// Micro-benchmarks of the chip's ceilings, run by the measurement harness next to the
// published figures: dense MFMA rates (FP64 16x16x4, FP32 16x16x4, BF16 16x16x32 with
// FP32 accumulation) from register-only loops of 16 independent accumulators per
// wave on every CU, and HBM bandwidth from a plain device copy (read + write counted).
// The copy kernel is also the reference for scaling hardware byte counters.
#include <algorithm>

#include "context.h"

namespace pnoeom {
namespace {

typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

template <int KIND>
__global__ __launch_bounds__(256) void mfma_loop_kernel(int iters, float* out) {
  // lane-varying operands (random-looking bits) so that the multipliers toggle
  unsigned x = threadIdx.x * 2654435761u + blockIdx.x * 97u + 1u;
  auto rnd = [&]() {
    x ^= x << 13;
    x ^= x >> 17;
    x ^= x << 5;
    return (float)(x & 0xffff) * 1e-5f - 0.3f;
  };
  float sum = 0.f;
  if (KIND == 0) {
    f64x4 acc[16];
    double a[4], b[4];
    for (int i = 0; i < 16; ++i) acc[i] = f64x4{0, 0, 0, 0};
    for (int i = 0; i < 4; ++i) a[i] = rnd();
    for (int i = 0; i < 4; ++i) b[i] = rnd();
    for (int it = 0; it < iters; ++it)
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j)
          acc[i * 4 + j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j], acc[i * 4 + j], 0, 0, 0);
    for (int i = 0; i < 16; ++i) sum += (float)(acc[i][0] + acc[i][1] + acc[i][2] + acc[i][3]);
  } else if (KIND == 1) {
    f32x4 acc[16];
    float a[4], b[4];
    for (int i = 0; i < 16; ++i) acc[i] = f32x4{0, 0, 0, 0};
    for (int i = 0; i < 4; ++i) a[i] = rnd();
    for (int i = 0; i < 4; ++i) b[i] = rnd();
    for (int it = 0; it < iters; ++it)
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j)
          acc[i * 4 + j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i], b[j], acc[i * 4 + j], 0, 0, 0);
    for (int i = 0; i < 16; ++i) sum += acc[i][0] + acc[i][1] + acc[i][2] + acc[i][3];
  } else {
    f32x4 acc[16];
    bf16x8 a[4], b[4];
    for (int i = 0; i < 16; ++i) acc[i] = f32x4{0, 0, 0, 0};
    for (int i = 0; i < 4; ++i)
      for (int e = 0; e < 8; ++e) a[i][e] = (__bf16)rnd();
    for (int i = 0; i < 4; ++i)
      for (int e = 0; e < 8; ++e) b[i][e] = (__bf16)rnd();
    for (int it = 0; it < iters; ++it)
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j)
          acc[i * 4 + j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i * 4 + j], 0, 0, 0);
    for (int i = 0; i < 16; ++i) sum += acc[i][0] + acc[i][1] + acc[i][2] + acc[i][3];
  }
  out[blockIdx.x * 256 + threadIdx.x] = sum;
}

typedef double d2 __attribute__((ext_vector_type(2)));

__global__ __launch_bounds__(256) void copy_kernel(int64_t n2, const d2* __restrict__ x, d2* __restrict__ y) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n2; e += (int64_t)gridDim.x * blockDim.x)
    y[e] = x[e];
}

}  // namespace

void probe_peaks(hipStream_t s, double* fp64_tflops, double* fp32_tflops, double* bf16_tflops, double* copy_gbs) {
  const int blocks = 1024, iters = 4000;
  DBuf<float> out;
  out.alloc((int64_t)blocks * 256);
  hipEvent_t e0, e1;
  PNO_HIP(hipEventCreate(&e0));
  PNO_HIP(hipEventCreate(&e1));
  double* dst[3] = {fp64_tflops, fp32_tflops, bf16_tflops};
  const double flops_per_mfma[3] = {2.0 * 16 * 16 * 4, 2.0 * 16 * 16 * 4, 2.0 * 16 * 16 * 32};
  for (int kind = 0; kind < 3; ++kind) {
    if (!dst[kind]) continue;
    float best = 1e30f;
    for (int rep = 0; rep < 3; ++rep) {  // first launch warms the clocks up
      PNO_HIP(hipEventRecord(e0, s));
      if (kind == 0)
        hipLaunchKernelGGL(mfma_loop_kernel<0>, dim3(blocks), dim3(256), 0, s, iters, (float*)out);
      else if (kind == 1)
        hipLaunchKernelGGL(mfma_loop_kernel<1>, dim3(blocks), dim3(256), 0, s, iters, (float*)out);
      else
        hipLaunchKernelGGL(mfma_loop_kernel<2>, dim3(blocks), dim3(256), 0, s, iters, (float*)out);
      PNO_HIP(hipGetLastError());
      PNO_HIP(hipEventRecord(e1, s));
      PNO_HIP(hipEventSynchronize(e1));
      float ms = 0.f;
      PNO_HIP(hipEventElapsedTime(&ms, e0, e1));
      if (rep > 0) best = std::min(best, ms);
    }
    const double fl = flops_per_mfma[kind] * 16.0 * iters * 4.0 * blocks;  // 16 per step, 4 waves per block
    *dst[kind] = fl / (best * 1e-3) / 1e12;
  }
  if (copy_gbs) {
    const int64_t bytes = (int64_t)1 << 30;  // per buffer
    DBuf<double> a, b;
    a.alloc(bytes / 8);
    b.alloc(bytes / 8);
    fill(s, bytes / 8, 1.0, a);
    float best = 1e30f;
    for (int rep = 0; rep < 4; ++rep) {
      PNO_HIP(hipEventRecord(e0, s));
      hipLaunchKernelGGL(copy_kernel, dim3(8192), dim3(256), 0, s, bytes / 16, (const d2*)a.p, (d2*)b.p);
      PNO_HIP(hipGetLastError());
      PNO_HIP(hipEventRecord(e1, s));
      PNO_HIP(hipEventSynchronize(e1));
      float ms = 0.f;
      PNO_HIP(hipEventElapsedTime(&ms, e0, e1));
      if (rep > 0) best = std::min(best, ms);
    }
    *copy_gbs = 2.0 * bytes / (best * 1e-3) / 1e9;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
}

}  // namespace pnoeom
