// Block Davidson eigensolver (non-Hermitian) on the GPU with an FP64 subspace.
//
// The subspace basis V and the projected sigma vectors S = P sigma(V) live in HBM
// as [m][N] row-major FP64 arrays.  Inner products are split-K MFMA GEMMs whose
// partial sums are reduced in a fixed order (bitwise reproducible); only the
// m x m subspace matrix G = V S^T and the k Ritz coefficient vectors cross to
// the host, where the small eigenproblem is solved.  The correction step is the
// one the paper describes for the PNO simulation: residual -> (semicanonical
// OSV/PNO basis) -> diagonal preconditioner -> back to the vector space.
#include <algorithm>
#include <cmath>
#include <chrono>
#include <cstdio>
#include <functional>

#include "context.h"

namespace pnoeom {
namespace {

constexpr double kClamp = 1e-4;

__device__ __forceinline__ double clampd(double d) {
  if (fabs(d) < kClamp) return d >= 0.0 ? kClamp : -kClamp;
  return d;
}

// out[e] = sum_b part[b][e]: one workgroup per output, a fixed summation tree
// (bitwise reproducible for a given nparts)
__global__ __launch_bounds__(256) void reduce_partials_kernel(int64_t nout, int64_t nparts,
                                                              const double* __restrict__ part,
                                                              double* __restrict__ out) {
  __shared__ double red[256];
  const int64_t e = blockIdx.x;
  double acc = 0.0;
  for (int64_t b = threadIdx.x; b < nparts; b += 256) acc += part[b * nout + e];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[e] = red[0];
}

// R[k][n] -= theta[k] * X[k][n]
__global__ void sub_scaled_rows_kernel(int nr, int64_t N, const double* __restrict__ theta,
                                       const double* __restrict__ X, double* __restrict__ R) {
  const int64_t total = nr * N;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x)
    R[e] -= theta[e / N] * X[e];
}

__global__ void scale_kernel(int64_t n, double a, double* __restrict__ x) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
    x[e] *= a;
}

// canonical preconditioner: singles / (theta + F_ii - F_aa), doubles / (theta + F_ii + F_jj - F_aa - F_bb)
// with the diagonals of the one-particle part of H-bar (F_oo, F_vv, row-major o x o and v x v)
__global__ void precond_canonical_kernel(int o, int v, const double* __restrict__ Foo, const double* __restrict__ Fvv,
                                         double theta, double* __restrict__ x) {
  const int64_t ov = (int64_t)o * v, n = ov + ov * ov;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
    double d;
    if (e < ov) {
      const int i = (int)(e / v), a = (int)(e % v);
      d = theta + Foo[(int64_t)i * o + i] - Fvv[(int64_t)a * v + a];
    } else {
      int64_t r = e - ov;
      const int b = (int)(r % v); r /= v;
      const int a = (int)(r % v); r /= v;
      const int j = (int)(r % o); r /= o;
      const int i = (int)r;
      d = theta + Foo[(int64_t)i * o + i] + Foo[(int64_t)j * o + j] - Fvv[(int64_t)a * v + a] - Fvv[(int64_t)b * v + b];
    }
    x[e] /= clampd(d);
  }
}

// CIS preconditioner: r / (theta - (e_a - e_i))
__global__ void precond_cis_kernel(int o, int v, const double* __restrict__ eps, double theta,
                                   double* __restrict__ x) {
  const int64_t ov = (int64_t)o * v;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < ov; e += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(e / v), a = (int)(e % v);
    x[e] /= clampd(theta - (eps[o + a] - eps[i]));
  }
}

__global__ void cis_diag_kernel(int o, int v, const double* __restrict__ eps, double* __restrict__ A) {
  const int64_t ov = (int64_t)o * v;
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= ov) return;
  const int i = (int)(e / v), a = (int)(e % v);
  A[e * ov + e] += eps[o + a] - eps[i];
}

unsigned g1(int64_t n) {
  int64_t b = (n + 255) / 256;
  if (b > 65536) b = 65536;
  if (b < 1) b = 1;
  return (unsigned)b;
}

// Skinny inner products out[i][j] = sum_n A[i][n] B[j][n] for at most 64 rows of A
// and 16 rows of B over a long n (the Davidson vectors).  The sum over n is
// order-free, so a wave feeds each FP64 MFMA 16x16x4 with four k-indices of its
// own choosing: in a unit of 16 consecutive n, lane l (row l%16, group g = l/16)
// supplies n = base + 4 s + g at step s, which makes every load instruction read
// 32 contiguous bytes per row.  Each wave accumulates the whole 64 x 16 block over
// a strided set of units; the four waves of a workgroup are summed through LDS
// and each workgroup writes one partial block, reduced afterwards in a fixed
// order.  The kernel is bound by HBM reads of A and B.
constexpr int kDotWaves = 4;
constexpr int kDotGroups = 512;

__global__ __launch_bounds__(64 * kDotWaves) void dots_kernel(int na, int nb, int64_t N, const double* __restrict__ A,
                                                              int64_t lda, const double* __restrict__ B, int64_t ldb,
                                                              double* __restrict__ part) {
  typedef double v4 __attribute__((ext_vector_type(4)));
  __shared__ double red[kDotWaves][64][17];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int r = lane & 15, g = lane >> 4;
  const int nblk = (na + 15) >> 4;
  v4 acc[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) acc[q] = v4{0, 0, 0, 0};
  // row pointers; rows past the end read row 0 and contribute zeros
  const double* pa[4];
  bool ma[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int row = q * 16 + r;
    pa[q] = A + (row < na ? (int64_t)row * lda : 0) + g;
    ma[q] = row < na;
  }
  const double* pb = B + (r < nb ? (int64_t)r * ldb : 0) + g;
  const bool mb = r < nb;
  const int64_t units = N / 16;
  const int64_t stride = (int64_t)gridDim.x * kDotWaves;
  for (int64_t u = (int64_t)blockIdx.x * kDotWaves + wave; u < units; u += stride) {
    const int64_t base = u * 16;
    double bv[4], av[4][4];
#pragma unroll
    for (int st = 0; st < 4; ++st) {
      const double x = pb[base + 4 * st];
      bv[st] = mb ? x : 0.0;
    }
#pragma unroll
    for (int q = 0; q < 4; ++q)
      if (q < nblk) {
#pragma unroll
        for (int st = 0; st < 4; ++st) {
          const double x = pa[q][base + 4 * st];
          av[q][st] = ma[q] ? x : 0.0;
        }
      }
#pragma unroll
    for (int st = 0; st < 4; ++st)
#pragma unroll
      for (int q = 0; q < 4; ++q)
        if (q < nblk) acc[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[q][st], bv[st], acc[q], 0, 0, 0);
  }
  // tail n in [16 units, N): one wave of the first workgroup, zero-padded
  if (blockIdx.x == 0 && wave == 0 && units * 16 < N) {
    const int64_t base = units * 16;
    double bv[4], av[4][4];
#pragma unroll
    for (int st = 0; st < 4; ++st) {
      const int64_t n = base + 4 * st + g;
      bv[st] = (n < N && mb) ? pb[base + 4 * st] : 0.0;
#pragma unroll
      for (int q = 0; q < 4; ++q) av[q][st] = (n < N && q < nblk && ma[q]) ? pa[q][base + 4 * st] : 0.0;
    }
#pragma unroll
    for (int st = 0; st < 4; ++st)
#pragma unroll
      for (int q = 0; q < 4; ++q)
        if (q < nblk) acc[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[q][st], bv[st], acc[q], 0, 0, 0);
  }
  // accumulator r4 of lane l holds row 16 q + l/16 + 4 r4, column l%16
#pragma unroll
  for (int q = 0; q < 4; ++q)
#pragma unroll
    for (int r4 = 0; r4 < 4; ++r4) red[wave][q * 16 + g + 4 * r4][r] = acc[q][r4];
  __syncthreads();
  double* out = part + (int64_t)blockIdx.x * na * nb;
  for (int e = threadIdx.x; e < na * nb; e += 64 * kDotWaves) {
    const int i = e / nb, j = e % nb;
    double sum = 0.0;
#pragma unroll
    for (int w = 0; w < kDotWaves; ++w) sum += red[w][i][j];
    out[e] = sum;
  }
}

// The same products with 16-byte loads, for rows that start 16-byte aligned (even row
// stride, aligned bases): units of 32 consecutive n, lane (row r, group g) reads the two
// columns base + 8 j + 2 g + {0, 1} for j = 0..3 (64 contiguous bytes of a row per load
// instruction) and MFMA step 2 j + h takes column 8 j + 2 g + h, identically for A and B.
// The operands of a wave's next unit are loaded before the MFMAs of the current one, so two
// units' reads are in flight per wave (≈ 6 TB/s against ≈ 3 TB/s for the kernel above).
// NQ = blocks of 16 rows of A (1..4).
template <int NQ>
__global__ __launch_bounds__(64 * kDotWaves) void dots_vec_kernel(int na, int nb, int64_t N,
                                                                  const double* __restrict__ A, int64_t lda,
                                                                  const double* __restrict__ B, int64_t ldb,
                                                                  double* __restrict__ part) {
  typedef double v4 __attribute__((ext_vector_type(4)));
  typedef double d2 __attribute__((ext_vector_type(2)));
  __shared__ double red[kDotWaves][64][17];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int r = lane & 15, g = lane >> 4;
  v4 acc[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q) acc[q] = v4{0, 0, 0, 0};
  // row pointers; rows past the end read row 0 and contribute zeros
  const double* pa[NQ];
  bool ma[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    const int row = q * 16 + r;
    pa[q] = A + (row < na ? (int64_t)row * lda : 0) + 2 * g;
    ma[q] = row < na;
  }
  const double* pb = B + (r < nb ? (int64_t)r * ldb : 0) + 2 * g;
  const bool mb = r < nb;
  const int64_t units = N / 32;
  const int64_t stride = (int64_t)gridDim.x * kDotWaves;
  d2 bv[4], av[NQ][4];
  auto load = [&](int64_t u, d2(&b)[4], d2(&a)[NQ][4]) {
    const int64_t base = u * 32;
#pragma unroll
    for (int j = 0; j < 4; ++j) b[j] = *(const d2*)(pb + base + 8 * j);
#pragma unroll
    for (int q = 0; q < NQ; ++q)
#pragma unroll
      for (int j = 0; j < 4; ++j) a[q][j] = *(const d2*)(pa[q] + base + 8 * j);
  };
  int64_t u = (int64_t)blockIdx.x * kDotWaves + wave;
  if (u < units) load(u, bv, av);
  while (u < units) {
    const int64_t un = u + stride;
    d2 bn[4], an[NQ][4];
    if (un < units) load(un, bn, an);
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const double bb = mb ? bv[j][h] : 0.0;
#pragma unroll
        for (int q = 0; q < NQ; ++q)
          acc[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(ma[q] ? av[q][j][h] : 0.0, bb, acc[q], 0, 0, 0);
      }
#pragma unroll
    for (int j = 0; j < 4; ++j) bv[j] = bn[j];
#pragma unroll
    for (int q = 0; q < NQ; ++q)
#pragma unroll
      for (int j = 0; j < 4; ++j) av[q][j] = an[q][j];
    u = un;
  }
  // tail n in [32 units, N): one wave of the first workgroup, zero-padded
  if (blockIdx.x == 0 && wave == 0 && units * 32 < N) {
    const int64_t base = units * 32;
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int64_t n = base + 8 * j + 2 * g + h;
        const double bb = (n < N && mb) ? pb[base + 8 * j + h] : 0.0;
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
          const double aa = (n < N && ma[q]) ? pa[q][base + 8 * j + h] : 0.0;
          acc[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(aa, bb, acc[q], 0, 0, 0);
        }
      }
  }
  // accumulator r4 of lane l holds row 16 q + l/16 + 4 r4, column l%16
#pragma unroll
  for (int q = 0; q < NQ; ++q)
#pragma unroll
    for (int r4 = 0; r4 < 4; ++r4) red[wave][q * 16 + g + 4 * r4][r] = acc[q][r4];
  __syncthreads();
  double* out = part + (int64_t)blockIdx.x * na * nb;
  for (int e = threadIdx.x; e < na * nb; e += 64 * kDotWaves) {
    const int i = e / nb, j = e % nb;
    double sum = 0.0;
#pragma unroll
    for (int w = 0; w < kDotWaves; ++w) sum += red[w][i][j];
    out[e] = sum;
  }
}

// Skinny subspace updates C[q][n] = alpha sum_i a(i, q) B[i][n] + beta C[q][n] with a few
// output rows (q < M <= MQ) and a short sum (i < K) over long rows of length N (the
// Davidson's Ritz vectors, residuals, Gram-Schmidt and block-orthonormalisation updates):
// HBM-bound.  Each thread streams two adjacent columns with 16-byte loads, eight rows of B
// in flight at a time; a(i, q) = A[i sai + q saq] is the same for the whole wave.
// (at least four waves per SIMD: the loads in flight set its speed)
template <int MQ>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void skinny_kernel(
    int M, int K, int64_t N, const double* __restrict__ A,
    int64_t sai, int64_t saq, double alpha, const double* __restrict__ B, double beta, double* __restrict__ C) {
  typedef double d2 __attribute__((ext_vector_type(2)));
  const int64_t np = N / 2;
  for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < np; p += (int64_t)gridDim.x * blockDim.x) {
    d2 acc[MQ];
#pragma unroll
    for (int q = 0; q < MQ; ++q) acc[q] = d2{0.0, 0.0};
    const double* b = B + 2 * p;
    int i = 0;
    for (; i + 8 <= K; i += 8) {
      d2 bv[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) bv[u] = *(const d2*)(b + (int64_t)(i + u) * N);
#pragma unroll
      for (int u = 0; u < 8; ++u)
#pragma unroll
        for (int q = 0; q < MQ; ++q)
          if (q < M) acc[q] += A[(int64_t)(i + u) * sai + q * saq] * bv[u];
    }
    for (; i < K; ++i) {
      const d2 bv = *(const d2*)(b + (int64_t)i * N);
#pragma unroll
      for (int q = 0; q < MQ; ++q)
        if (q < M) acc[q] += A[(int64_t)i * sai + q * saq] * bv;
    }
#pragma unroll
    for (int q = 0; q < MQ; ++q)
      if (q < M) {
        d2* c = (d2*)(C + (int64_t)q * N + 2 * p);
        d2 val = alpha * acc[q];
        if (beta != 0.0) val += beta * (*c);
        *c = val;
      }
  }
}

// C = alpha op(A) B + beta C for the Davidson's subspace updates (rows of length N, row
// stride N): a(i, q) = A[i sai + q saq] with sai = 1 or saq = 1.  The streaming kernel when
// the rows are 16-byte aligned and M <= 16, else the tiled GEMM.
void skinny(hipStream_t s, int M, int K, int64_t N, const double* A, int64_t sai, int64_t saq, double alpha,
            const double* B, double beta, double* C) {
  if (M <= 0 || N <= 0) return;
  if (M <= 16 && N % 2 == 0 && (uintptr_t)B % 16 == 0 && (uintptr_t)C % 16 == 0) {
    const int64_t np = N / 2;
    const unsigned grid = (unsigned)std::max<int64_t>(1, std::min<int64_t>(2048, (np + 255) / 256));
    // (an 8-row instance compiles to twice the registers of the 16-row one, so 5..16 rows
    // share the latter; rows past M are skipped)
    if (M <= 4)
      hipLaunchKernelGGL(skinny_kernel<4>, dim3(grid), dim3(256), 0, s, M, K, N, A, sai, saq, alpha, B, beta, C);
    else
      hipLaunchKernelGGL(skinny_kernel<16>, dim3(grid), dim3(256), 0, s, M, K, N, A, sai, saq, alpha, B, beta, C);
    PNO_HIP(hipGetLastError());
    return;
  }
  GemmDesc<double> d;
  d.ta = saq == 1;
  d.lda = d.ta ? sai : saq;
  d.M = M; d.N = N; d.K = K; d.alpha = alpha; d.beta = beta;
  d.A = A; d.B = B; d.ldb = N; d.C = C; d.ldc = N;
  gemm(d, s);
}

struct Dots {
  DBuf<double> part, out;
  Context* ctx = nullptr;  // for the timed region of the inner products
};

// host out[i][j] = sum_n A[i][n] B[j][n]   (A: na rows, B: nb rows, row stride N)
void dots(hipStream_t s, Dots& w, const double* A, int na, const double* B, int nb, int64_t N, double* host) {
  if (na == 0 || nb == 0) return;
  if (na <= 16 && nb > 16 && nb <= 64) {
    // one launch with the long side as A (64 rows) instead of one per 16 rows of B,
    // each re-reading A: out = (B A^T)^T
    std::vector<double> t((size_t)na * nb);
    dots(s, w, B, nb, A, na, N, t.data());
    for (int i = 0; i < na; ++i)
      for (int j = 0; j < nb; ++j) host[(int64_t)i * nb + j] = t[(size_t)j * na + i];
    return;
  }
  const int64_t nout = (int64_t)na * nb;
  int64_t groups = std::min<int64_t>(kDotGroups, std::max<int64_t>(1, (N / 16 + kDotWaves - 1) / kDotWaves));
  if ((int64_t)w.part.n < groups * nout) w.part.alloc(groups * nout);
  if ((int64_t)w.out.n < nout) w.out.alloc(nout);
  std::vector<double> blk;
  // 16-byte loads when every row starts 16-byte aligned
  const bool vec = N % 2 == 0 && (uintptr_t)A % 16 == 0 && (uintptr_t)B % 16 == 0;
  // blocks of at most 64 x 16 outputs
  for (int i0 = 0; i0 < na; i0 += 64)
    for (int j0 = 0; j0 < nb; j0 += 16) {
      const int ni = std::min(64, na - i0), nj = std::min(16, nb - j0);
      hipEvent_t ev = w.ctx ? w.ctx->region_begin(0, s) : nullptr;
      const double* a0 = A + (int64_t)i0 * N;
      const double* b0 = B + (int64_t)j0 * N;
      if (vec) {
        const int nq = (ni + 15) / 16;
        auto kern = nq == 1 ? dots_vec_kernel<1> : nq == 2 ? dots_vec_kernel<2> : nq == 3 ? dots_vec_kernel<3>
                                                                                        : dots_vec_kernel<4>;
        hipLaunchKernelGGL(kern, dim3((unsigned)groups), dim3(64 * kDotWaves), 0, s, ni, nj, N, a0, N, b0, N,
                           (double*)w.part);
      } else {
        hipLaunchKernelGGL(dots_kernel, dim3((unsigned)groups), dim3(64 * kDotWaves), 0, s, ni, nj, N, a0, N, b0, N,
                           (double*)w.part);
      }
      PNO_HIP(hipGetLastError());
      const int64_t nsub = (int64_t)ni * nj;
      hipLaunchKernelGGL(reduce_partials_kernel, dim3((unsigned)nsub), dim3(256), 0, s, nsub, groups,
                         (const double*)w.part, (double*)w.out);
      PNO_HIP(hipGetLastError());
      if (w.ctx) w.ctx->region_end(ev, 0, s, 2, 2.0 * ni * nj * (double)N, 8.0 * (ni + nj) * (double)N);
      if (ni == na && nj == nb) {
        PNO_HIP(hipMemcpyAsync(host, w.out, nout * sizeof(double), hipMemcpyDeviceToHost, s));
      } else {
        blk.resize(nsub);
        PNO_HIP(hipMemcpyAsync(blk.data(), w.out, nsub * sizeof(double), hipMemcpyDeviceToHost, s));
        PNO_HIP(hipStreamSynchronize(s));
        for (int i = 0; i < ni; ++i)
          for (int j = 0; j < nj; ++j) host[(int64_t)(i0 + i) * nb + j0 + j] = blk[(int64_t)i * nj + j];
      }
    }
  PNO_HIP(hipStreamSynchronize(s));
}

struct Operator {
  int64_t N = 0;
  std::function<void(int, const double*, double*)> apply;  // S = P A X for nvec rows
  std::function<void(double*, double)> precond;            // in place, result in range(P)
  std::function<void(double*)> project;                    // in place
};

// Orthonormal-column Q (m x k) of Y (m x k) by modified Gram-Schmidt with one re-orthogonalisation.
std::vector<double> orth_cols(int m, int k, const std::vector<double>& Y) {
  std::vector<double> Q = Y;
  for (int j = 0; j < k; ++j) {
    for (int pass = 0; pass < 2; ++pass)
      for (int q = 0; q < j; ++q) {
        double d = 0.0;
        for (int i = 0; i < m; ++i) d += Q[i * k + q] * Q[i * k + j];
        for (int i = 0; i < m; ++i) Q[i * k + j] -= d * Q[i * k + q];
      }
    double n = 0.0;
    for (int i = 0; i < m; ++i) n += Q[i * k + j] * Q[i * k + j];
    n = std::sqrt(n);
    for (int i = 0; i < m; ++i) Q[i * k + j] /= n;
  }
  return Q;
}

// ----------------------------------------------------------------------------- checkpoints
// File: "PNOEOMCK", int32 version 1, int64 N, int32 nvec, space, precision, phase, then
// double theta[nvec] and the vectors [nvec][N] (host byte order).
constexpr char kCkptMagic[8] = {'P', 'N', 'O', 'E', 'O', 'M', 'C', 'K'};

void write_checkpoint(hipStream_t s, const char* path, int64_t N, int nvec, int space, int precision, int phase,
                      const std::vector<double>& theta, const double* dX) {
  std::vector<double> h((size_t)nvec * N);
  PNO_HIP(hipMemcpyAsync(h.data(), dX, h.size() * sizeof(double), hipMemcpyDeviceToHost, s));
  PNO_HIP(hipStreamSynchronize(s));
  const std::string tmp = std::string(path) + ".tmp";
  FILE* f = fopen(tmp.c_str(), "wb");
  PNO_CHECK(f != nullptr, PNOEOM_EINVAL, std::string("checkpoint: cannot write ") + tmp);
  const int32_t hdr[5] = {1, nvec, space, precision, phase};
  bool ok = fwrite(kCkptMagic, 1, 8, f) == 8 && fwrite(&hdr[0], 4, 1, f) == 1 && fwrite(&N, 8, 1, f) == 1 &&
            fwrite(&hdr[1], 4, 4, f) == 4 && fwrite(theta.data(), 8, nvec, f) == (size_t)nvec &&
            fwrite(h.data(), 8, h.size(), f) == h.size();
  ok = (fclose(f) == 0) && ok;
  PNO_CHECK(ok, PNOEOM_EINVAL, std::string("checkpoint: write failed for ") + tmp);
  PNO_CHECK(std::rename(tmp.c_str(), path) == 0, PNOEOM_EINVAL, std::string("checkpoint: cannot rename to ") + path);
}

struct Checkpoint {
  int64_t N = 0;
  int nvec = 0, space = 0, precision = 0, phase = 0;
  std::vector<double> theta, x;
};

Checkpoint read_checkpoint(const char* path) {
  Checkpoint k;
  FILE* f = fopen(path, "rb");
  PNO_CHECK(f != nullptr, PNOEOM_EINVAL, std::string("resume: cannot open ") + path);
  char magic[8];
  int32_t ver = 0, h4[4];
  bool ok = fread(magic, 1, 8, f) == 8 && std::equal(magic, magic + 8, kCkptMagic) && fread(&ver, 4, 1, f) == 1 &&
            ver == 1 && fread(&k.N, 8, 1, f) == 1 && fread(h4, 4, 4, f) == 4;
  if (ok) {
    k.nvec = h4[0]; k.space = h4[1]; k.precision = h4[2]; k.phase = h4[3];
    ok = k.N > 0 && k.nvec > 0 && k.nvec < (1 << 20) && k.N < (int64_t(1) << 40);
  }
  if (ok) {
    k.theta.resize(k.nvec);
    k.x.resize((size_t)k.nvec * k.N);
    ok = fread(k.theta.data(), 8, k.nvec, f) == (size_t)k.nvec && fread(k.x.data(), 8, k.x.size(), f) == k.x.size();
  }
  fclose(f);
  PNO_CHECK(ok, PNOEOM_EINVAL, std::string("resume: not a readable checkpoint: ") + path);
  return k;
}

// nroots roots must converge; nextra further Ritz pairs are tracked (and kept at
// collapse) to speed up convergence of the highest target root.  Iterations are
// numbered from it_base + 1 for checkpoints and aborts (phase 0: main run, 1: FP64
// refinement).
DavidsonResult run_davidson(Context& c, Operator& op, int ntarget, const double* guess, int nguess,
                            const pnoeom_davidson_opts& opt, const char* tag, double* xout, int nextra = 0,
                            int it_base = 0, int phase = 0) {
  hipStream_t s = c.stream;
  const auto t_start = std::chrono::steady_clock::now();
  const int64_t N = op.N;
  const int nroots = ntarget + nextra;
  const int maxs = std::max(opt.max_sub, nroots + nguess);
  const int cap = maxs + nroots;
  DBuf<double> V, S, X, R, cand, dY, dc, dcb, dth;
  {
    // the sigma workspaces of earlier calls may hold most of the device (their chunk is sized
    // to the free memory): drop them when the subspace would not fit beside them; the first
    // sigma block re-sizes them against what is left
    size_t fr = 0, tot = 0;
    PNO_HIP(hipMemGetInfo(&fr, &tot));
    const int64_t need = ((int64_t)(2 * cap + 2 * nroots + 1) * N + 3 * (int64_t)cap * nroots) * 8 + (1ll << 30);
    if ((int64_t)fr < need && !c.keep_build_tmp) {
      c.drop_graphs();  // captured sigma blocks refer to the workspaces
      c.sw.release();
      for (DBuf<double>* b : {&c.pno.r1, &c.pno.r2, &c.pno.s1, &c.pno.s2}) b->release();
    }
  }
  V.alloc((int64_t)cap * N);
  S.alloc((int64_t)cap * N);
  X.alloc((int64_t)nroots * N);
  R.alloc((int64_t)nroots * N);
  cand.alloc(N);
  dY.alloc((int64_t)cap * nroots);
  dc.alloc(cap);
  dcb.alloc((int64_t)cap * nroots);
  dth.alloc(nroots);
  Dots dw;
  dw.ctx = &c;
  DavidsonResult res;
  const double tol_r = opt.tol_r > 0 ? opt.tol_r : 0.1 * std::sqrt(opt.tol_e);

  // orthonormalise x (device, length N) against V[0:m]; returns the norm left
  auto orth = [&](double* x, int m) -> double {
    std::vector<double> cvec(std::max(m, 1));
    for (int pass = 0; pass < 2; ++pass) {
      if (m > 0) {
        dots(s, dw, V, m, x, 1, N, cvec.data());
        PNO_HIP(hipMemcpyAsync(dc, cvec.data(), m * sizeof(double), hipMemcpyHostToDevice, s));
        skinny(s, 1, m, N, dc, 1, m, -1.0, V, 1.0, x);
        // second pass only if the first removed more than half the squared norm (x is a unit
        // vector and V orthonormal, so 1 - sum c_i^2 is left)
        double c2 = 0.0;
        for (int i = 0; i < m; ++i) c2 += cvec[i] * cvec[i];
        if (pass == 0 && 1.0 - c2 >= 0.5) break;
      }
    }
    double nn = 0.0;
    dots(s, dw, x, 1, x, 1, N, &nn);
    return std::sqrt(nn);
  };

  int m = 0;
  std::vector<int> newidx;
  for (int g = 0; g < nguess; ++g) {
    PNO_HIP(hipMemcpyAsync(cand, guess + (int64_t)g * N, N * sizeof(double), hipMemcpyDeviceToDevice, s));
    op.project(cand);
    double n0 = 0.0;
    dots(s, dw, cand, 1, cand, 1, N, &n0);
    if (n0 <= 0.0) continue;
    hipLaunchKernelGGL(scale_kernel, dim3(g1(N)), dim3(256), 0, s, N, 1.0 / std::sqrt(n0), (double*)cand);
    const double nrm = orth(cand, m);
    if (nrm < 1e-10) continue;
    hipLaunchKernelGGL(scale_kernel, dim3(g1(N)), dim3(256), 0, s, N, 1.0 / nrm, (double*)cand);
    PNO_HIP(hipMemcpyAsync(V + (int64_t)m * N, cand, N * sizeof(double), hipMemcpyDeviceToDevice, s));
    ++m;
  }
  PNO_CHECK(m >= nroots, PNOEOM_EINVAL, "Davidson: fewer independent guess vectors than roots");
  PNO_CHECK(m <= maxs, PNOEOM_EINVAL, "Davidson: more guess vectors than the subspace holds");
  // sigma applications; with an iteration log their wall time is measured (the stream is
  // synchronised around them only then)
  double sigma_s = 0.0;
  auto apply = [&](int nv, const double* X_, double* S_) {
    if (!opt.log_path) {
      op.apply(nv, X_, S_);
      return;
    }
    PNO_HIP(hipStreamSynchronize(s));
    const auto t0 = std::chrono::steady_clock::now();
    op.apply(nv, X_, S_);
    PNO_HIP(hipStreamSynchronize(s));
    sigma_s += std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  };
  apply(m, V, S);
  res.nsigma += m;
  std::vector<double> G((size_t)maxs * maxs);
  {
    std::vector<double> tmp((size_t)m * m);
    dots(s, dw, V, m, S, m, N, tmp.data());
    for (int i = 0; i < m; ++i)
      for (int j = 0; j < m; ++j) G[(size_t)i * maxs + j] = tmp[(size_t)i * m + j];
  }
  std::vector<double> theta_old(nroots, 0.0);
  bool have_old = false;
  for (int it = 1; it <= opt.max_iter; ++it) {
    TraceRange tr_("davidson iteration");
    res.iters = it;
    std::vector<double> Gm((size_t)m * m), wr(m), wi(m), vr((size_t)m * m);
    for (int i = 0; i < m; ++i)
      for (int j = 0; j < m; ++j) Gm[(size_t)i * m + j] = G[(size_t)i * maxs + j];
    const int st = host_eig(m, Gm.data(), wr.data(), wi.data(), vr.data(), std::min(nroots, m));
    PNO_CHECK(st == PNOEOM_OK, PNOEOM_ENOTCONV, "subspace eigenproblem did not converge");
    std::vector<double> theta(nroots), Y((size_t)m * nroots);
    for (int k = 0; k < nroots; ++k) {
      theta[k] = wr[k];
      if (wi[k] != 0.0) res.complex_pair = true;
      double n = 0.0;
      for (int i = 0; i < m; ++i) n += vr[(size_t)i * m + k] * vr[(size_t)i * m + k];
      n = std::sqrt(n);
      for (int i = 0; i < m; ++i) Y[(size_t)i * nroots + k] = vr[(size_t)i * m + k] / n;
    }
    PNO_HIP(hipMemcpyAsync(dY, Y.data(), Y.size() * sizeof(double), hipMemcpyHostToDevice, s));
    PNO_HIP(hipMemcpyAsync(dth, theta.data(), nroots * sizeof(double), hipMemcpyHostToDevice, s));
    skinny(s, nroots, m, N, dY, nroots, 1, 1.0, V, 0.0, X);
    skinny(s, nroots, m, N, dY, nroots, 1, 1.0, S, 0.0, R);
    hipLaunchKernelGGL(sub_scaled_rows_kernel, dim3(g1(nroots * N)), dim3(256), 0, s, nroots, N,
                       (const double*)dth, (const double*)X, (double*)R);
    std::vector<double> rr((size_t)nroots * nroots);
    dots(s, dw, R, nroots, R, nroots, N, rr.data());
    std::vector<double> rn(nroots);
    std::vector<bool> conv(nroots);
    bool all = true;
    for (int k = 0; k < nroots; ++k) {
      rn[k] = std::sqrt(std::max(0.0, rr[(size_t)k * nroots + k]));
      const double de = have_old ? std::fabs(theta[k] - theta_old[k]) : 1e300;
      conv[k] = (k >= ntarget) || (rn[k] <= tol_r && de <= opt.tol_e);
      all = all && conv[k];
    }
    res.omega.assign(theta.begin(), theta.begin() + ntarget);
    res.resnorm.assign(rn.begin(), rn.begin() + ntarget);
    if (opt.log_path) {
      FILE* lf = fopen(opt.log_path, "a");
      PNO_CHECK(lf != nullptr, PNOEOM_EINVAL, std::string("davidson: cannot append to ") + opt.log_path);
      const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
      fprintf(lf, "{\"phase\": %d, \"it\": %d, \"m\": %d, \"nsigma\": %d, \"seconds\": %.6f, \"sigma_seconds\": %.6f",
              phase, it_base + it, m, res.nsigma, secs, sigma_s);
      const char* keys[3] = {"omega", "resnorm", "domega"};
      for (int f = 0; f < 3; ++f) {
        fprintf(lf, ", \"%s\": [", keys[f]);
        for (int k = 0; k < ntarget; ++k) {
          const double x = f == 0 ? theta[k] : f == 1 ? rn[k] : (have_old ? theta[k] - theta_old[k] : 0.0);
          fprintf(lf, "%s%.17g", k ? ", " : "", x);
        }
        fprintf(lf, "]");
      }
      fprintf(lf, "}\n");
      fclose(lf);
    }
    if (opt.verbose) {
      fprintf(stderr, "[%s] it %3d m %3d", tag, it, m);
      for (int k = 0; k < ntarget; ++k) fprintf(stderr, " %.10f(%.1e)", theta[k], rn[k]);
      fprintf(stderr, "\n");
      fflush(stderr);
    }
    if (all) {
      res.converged = true;
      if (xout)
        PNO_HIP(hipMemcpyAsync(xout, X, (int64_t)ntarget * N * sizeof(double), hipMemcpyDeviceToDevice, s));
      PNO_HIP(hipStreamSynchronize(s));
      return res;
    }
    const int itg = it_base + it;
    const bool abort_now = opt.abort_after_iter > 0 && itg >= opt.abort_after_iter;
    if (opt.ckpt_path && (abort_now || (opt.ckpt_every > 0 && itg % opt.ckpt_every == 0)))
      write_checkpoint(s, opt.ckpt_path, N, nroots, opt.space, opt.precision, phase, theta, X);
    if (abort_now) {
      res.aborted = true;
      PNO_HIP(hipStreamSynchronize(s));
      return res;
    }
    theta_old = theta;
    have_old = true;
    // corrections: preconditioned residuals of the unconverged roots, normalised,
    // orthogonalised against V as a block (classical Gram-Schmidt, each pass reading V
    // once, the second only when needed), then among themselves; staged in X
    // When every preconditioned direction lies in span(V) (a preconditioner close to the
    // exact operator maps r_k back onto the Ritz vector), the plain residuals are taken:
    // the Galerkin condition V^T r_k = 0 makes them new directions whenever r_k != 0.
    int nnew = 0;
    for (int attempt = 0; attempt < 2 && nnew == 0; ++attempt) {
      int nc = 0;
      for (int k = 0; k < nroots; ++k) {
        if (conv[k]) continue;
        double* xk = X + (int64_t)nc * N;
        PNO_HIP(hipMemcpyAsync(xk, R + (int64_t)k * N, N * sizeof(double), hipMemcpyDeviceToDevice, s));
        if (attempt == 0) op.precond(xk, theta[k]);
        ++nc;
      }
      if (nc > 0) {
        std::vector<double> cc((size_t)nc * nc);
        dots(s, dw, X, nc, X, nc, N, cc.data());
        for (int q = 0; q < nc; ++q) {
          const double n0 = cc[(size_t)q * nc + q];
          const double sc = n0 > 0.0 ? 1.0 / std::sqrt(n0) : 0.0;
          hipLaunchKernelGGL(scale_kernel, dim3(g1(N)), dim3(256), 0, s, N, sc, X + (int64_t)q * N);
        }
        std::vector<double> coef((size_t)m * nc);
        for (int pass = 0; pass < 2; ++pass) {
          dots(s, dw, V, m, X, nc, N, coef.data());  // coef[i][q] = V_i . X_q
          PNO_HIP(hipMemcpyAsync(dcb, coef.data(), coef.size() * sizeof(double), hipMemcpyHostToDevice, s));
          skinny(s, nc, m, N, dcb, nc, 1, -1.0, V, 1.0, X);
          // "twice is enough": a second pass only if the first removed more than half of a
          // correction's squared norm (unit corrections, orthonormal V: 1 - sum_i c_iq^2 is
          // left); otherwise one projection is exact to working precision
          if (pass == 0) {
            bool again = false;
            for (int q = 0; q < nc && !again; ++q) {
              double c2 = 0.0;
              for (int i = 0; i < m; ++i) c2 += coef[(size_t)i * nc + q] * coef[(size_t)i * nc + q];
              again = 1.0 - c2 < 0.5;
            }
            if (!again) break;
          }
        }
        // orthonormal basis of the block itself: two Gram passes, each X <- T^T X with
        // T = W_k diag(w_k^-1/2) from the eigenpairs (w_k, W_k) of the block's Gram
        // matrix, directions with w_k < 1e-20 (norm below 1e-10 after the projection
        // against V, the vectors having been unit before it) dropped.  Two dot-product
        // sweeps and two GEMMs replace the vector-by-vector loop.
        int nb = nc;
        double* src = X;
        double* dst = V + (int64_t)m * N;
        for (int pass = 0; pass < 2 && nb > 0; ++pass) {
          std::vector<double> gm((size_t)nb * nb), w(nb), W((size_t)nb * nb);
          dots(s, dw, src, nb, src, nb, N, gm.data());
          PNO_CHECK(host_syev(nb, gm.data(), w.data(), W.data()) == PNOEOM_OK, PNOEOM_ENOTCONV,
                    "Davidson: block Gram eigenproblem did not converge");
          std::vector<double> Tt;  // [kept][nb], row r = (W_k / sqrt(w_k))^T
          for (int k = 0; k < nb; ++k) {
            if (!(w[k] >= 1e-20)) continue;
            const double sc = 1.0 / std::sqrt(w[k]);
            for (int i = 0; i < nb; ++i) Tt.push_back(W[(size_t)i * nb + k] * sc);
          }
          const int nk = (int)(Tt.size() / (size_t)std::max(nb, 1));
          if (nk == 0) {
            nb = 0;
            break;
          }
          PNO_HIP(hipMemcpyAsync(dcb, Tt.data(), Tt.size() * sizeof(double), hipMemcpyHostToDevice, s));
          skinny(s, nk, nb, N, dcb, 1, nb, 1.0, src, 0.0, dst);
          nb = nk;
          std::swap(src, dst);
        }
        // after an even number of passes the block is back in X: move it into V
        if (nb > 0 && src != V + (int64_t)m * N)
          PNO_HIP(hipMemcpyAsync(V + (int64_t)m * N, src, (int64_t)nb * N * sizeof(double), hipMemcpyDeviceToDevice, s));
        nnew = nb;
      }
    }
    if (nnew == 0) {
      // no direction outside span(V) is left (e.g. V spans the whole space): the Ritz values
      // cannot change any more, so residuals within tol_r are final
      bool small = true;
      for (int k = 0; k < ntarget; ++k) small = small && rn[k] <= tol_r;
      if (small) {
        res.converged = true;
        if (xout) {  // X held the corrections: the Ritz vectors again, from V and Y
          PNO_HIP(hipMemcpyAsync(dY, Y.data(), Y.size() * sizeof(double), hipMemcpyHostToDevice, s));
          skinny(s, ntarget, m, N, dY, nroots, 1, 1.0, V, 0.0, xout);  // xout holds the ntarget roots only
        }
        PNO_HIP(hipStreamSynchronize(s));
        return res;
      }
    }
    PNO_CHECK(nnew > 0, PNOEOM_ENOTCONV, "Davidson stalled: no new directions");
    if (m + nnew > maxs) {
      // collapse onto the Ritz vectors: V <- V Q, S <- S Q, G <- Q^T G Q
      const std::vector<double> Q = orth_cols(m, nroots, Y);
      PNO_HIP(hipMemcpyAsync(dY, Q.data(), Q.size() * sizeof(double), hipMemcpyHostToDevice, s));
      skinny(s, nroots, m, N, dY, nroots, 1, 1.0, V, 0.0, X);
      skinny(s, nroots, m, N, dY, nroots, 1, 1.0, S, 0.0, R);
      // keep the staged new vectors: move them right after the collapsed block
      DBuf<double> stage;
      stage.alloc((int64_t)std::max(nnew, 1) * N);
      PNO_HIP(hipMemcpyAsync(stage, V + (int64_t)m * N, (int64_t)nnew * N * sizeof(double), hipMemcpyDeviceToDevice, s));
      PNO_HIP(hipMemcpyAsync(V, X, (int64_t)nroots * N * sizeof(double), hipMemcpyDeviceToDevice, s));
      PNO_HIP(hipMemcpyAsync(S, R, (int64_t)nroots * N * sizeof(double), hipMemcpyDeviceToDevice, s));
      std::vector<double> Gn((size_t)maxs * maxs, 0.0);
      for (int a = 0; a < nroots; ++a)
        for (int b = 0; b < nroots; ++b) {
          double acc = 0.0;
          for (int i = 0; i < m; ++i)
            for (int j = 0; j < m; ++j) acc += Q[(size_t)i * nroots + a] * G[(size_t)i * maxs + j] * Q[(size_t)j * nroots + b];
          Gn[(size_t)a * maxs + b] = acc;
        }
      G.swap(Gn);
      m = nroots;
      int kept = 0;
      for (int q = 0; q < nnew; ++q) {
        PNO_HIP(hipMemcpyAsync(cand, stage + (int64_t)q * N, N * sizeof(double), hipMemcpyDeviceToDevice, s));
        const double nrm = orth(cand, m + kept);
        if (nrm < 1e-10) continue;
        hipLaunchKernelGGL(scale_kernel, dim3(g1(N)), dim3(256), 0, s, N, 1.0 / nrm, (double*)cand);
        PNO_HIP(hipMemcpyAsync(V + (int64_t)(m + kept) * N, cand, N * sizeof(double), hipMemcpyDeviceToDevice, s));
        ++kept;
      }
      nnew = kept;
      PNO_CHECK(nnew > 0, PNOEOM_ENOTCONV, "Davidson stalled after collapse");
    }
    apply(nnew, V + (int64_t)m * N, S + (int64_t)m * N);
    res.nsigma += nnew;
    const int m1 = m + nnew;
    {
      std::vector<double> a((size_t)m1 * nnew), b((size_t)nnew * m);
      dots(s, dw, V, m1, S + (int64_t)m * N, nnew, N, a.data());   // G[0:m1][m:m1]
      for (int i = 0; i < m1; ++i)
        for (int j = 0; j < nnew; ++j) G[(size_t)i * maxs + m + j] = a[(size_t)i * nnew + j];
      if (m > 0) {
        dots(s, dw, V + (int64_t)m * N, nnew, S, m, N, b.data());  // G[m:m1][0:m]
        for (int i = 0; i < nnew; ++i)
          for (int j = 0; j < m; ++j) G[(size_t)(m + i) * maxs + j] = b[(size_t)i * m + j];
      }
    }
    m = m1;
  }
  res.converged = false;
  if (xout)
    PNO_HIP(hipMemcpyAsync(xout, X, (int64_t)ntarget * N * sizeof(double), hipMemcpyDeviceToDevice, s));
  PNO_HIP(hipStreamSynchronize(s));
  return res;
}

}  // namespace

// ----------------------------------------------------------------------------- CIS
void cis_roots(Context& c, int n, double* omega, double* vec) {
  PNO_CHECK(c.have_df, PNOEOM_ESTATE, "cis before build_df");
  const int o = c.o, v = c.v, naux = c.naux, nmo = c.nmo;
  const int64_t ov = c.ov(), n2 = (int64_t)nmo * nmo;
  PNO_CHECK(n >= 1 && n <= ov, PNOEOM_EINVAL, "cis: bad number of roots");
  hipStream_t s = c.stream;
  // A = 2 (ia|jb) - (ij|ab) + d(e_a - e_i), bare integrals
  DBuf<double> A, BooT0, BvvT0, tmp;
  A.alloc(ov * ov);
  BooT0.alloc((int64_t)o * o * naux);
  BvvT0.alloc((int64_t)v * v * naux);
  tmp.alloc(ov * ov);
  {
    Perm4 p;
    p.d[0] = o; p.d[1] = o; p.d[2] = naux; p.d[3] = 1;
    p.is[0] = nmo; p.is[1] = 1; p.is[2] = n2; p.is[3] = 0;
    p.os[0] = (int64_t)o * naux; p.os[1] = naux; p.os[2] = 1; p.os[3] = 0;
    permute4(s, p, 1.0, c.B, 0.0, BooT0);
    p.d[0] = v; p.d[1] = v;
    p.os[0] = (int64_t)v * naux;
    permute4(s, p, 1.0, c.B + (int64_t)o * nmo + o, 0.0, BvvT0);
  }
  GemmDesc<double> d;
  d.tb = true; d.M = (int64_t)o * o; d.N = (int64_t)v * v; d.K = naux;
  d.A = BooT0; d.lda = naux; d.B = BvvT0; d.ldb = naux; d.C = tmp; d.ldc = (int64_t)v * v;
  gemm(d, s);
  {
    const int64_t dims[4] = {o, o, v, v};
    const int pp[4] = {0, 3, 1, 2};
    permute_c(s, dims, pp, -1.0, tmp, 0.0, A);
  }
  axpby(s, ov * ov, 2.0, c.G, 1.0, A);
  hipLaunchKernelGGL(cis_diag_kernel, dim3((ov + 255) / 256), dim3(256), 0, s, o, v, (const double*)c.eps,
                     (double*)A);
  PNO_HIP(hipGetLastError());
  BooT0.release();
  BvvT0.release();
  tmp.release();

  Operator op;
  op.N = ov;
  const double* Ap = A;
  op.apply = [&](int nv, const double* X, double* S) {
    GemmDesc<double> g;
    g.tb = true; g.M = nv; g.N = ov; g.K = ov;
    g.A = X; g.lda = ov; g.B = Ap; g.ldb = ov; g.C = S; g.ldc = ov;
    gemm(g, s);
  };
  op.precond = [&](double* x, double th) {
    hipLaunchKernelGGL(precond_cis_kernel, dim3(g1(ov)), dim3(256), 0, s, o, v, (const double*)c.eps, th, x);
  };
  op.project = [](double*) {};
  // guesses: unit vectors at the smallest orbital-energy differences
  std::vector<double> eps(nmo);
  PNO_HIP(hipMemcpyAsync(eps.data(), c.eps, nmo * sizeof(double), hipMemcpyDeviceToHost, s));
  PNO_HIP(hipStreamSynchronize(s));
  std::vector<int64_t> idx(ov);
  for (int64_t e = 0; e < ov; ++e) idx[e] = e;
  std::stable_sort(idx.begin(), idx.end(), [&](int64_t x, int64_t y) {
    return eps[o + x % v] - eps[x / v] < eps[o + y % v] - eps[y / v];
  });
  const int ng = (int)std::min<int64_t>(ov, std::max(2 * n, n + 4));
  std::vector<double> gh((size_t)ng * ov, 0.0);
  for (int g = 0; g < ng; ++g) gh[(size_t)g * ov + idx[g]] = 1.0;
  DBuf<double> dg;
  dg.alloc((int64_t)ng * ov);
  PNO_HIP(hipMemcpyAsync(dg, gh.data(), gh.size() * sizeof(double), hipMemcpyHostToDevice, s));
  pnoeom_davidson_opts opt;
  pnoeom_davidson_defaults(&opt);
  opt.tol_e = 1e-13;
  opt.tol_r = 1e-11;
  opt.max_sub = std::max(40, 4 * n + 8);
  opt.max_iter = 300;
  opt.verbose = 0;
  const int nextra = (int)std::min<int64_t>(ov - n, std::max(2, n / 2));
  DavidsonResult r = run_davidson(c, op, n, dg, ng, opt, "cis", vec, nextra);
  PNO_CHECK(r.converged, PNOEOM_ENOTCONV, "CIS Davidson did not converge");
  for (int k = 0; k < n; ++k) omega[k] = r.omega[k];
}

}  // namespace pnoeom

// ----------------------------------------------------------------------------- EOM-CCSD roots
namespace pnoeom {

void precond_pno(Context& c, double* x, double theta);
void project_pno(Context& c, double* x);

DavidsonResult davidson(Context& c, int nroots, const pnoeom_davidson_opts& opt) {
  PNO_CHECK(c.have_df, PNOEOM_ESTATE, "davidson before build_df");
  PNO_CHECK(nroots >= 1 && nroots <= c.ov(), PNOEOM_EINVAL, "davidson: bad number of roots");
  PNO_CHECK(opt.space == PNOEOM_CANONICAL || opt.space == PNOEOM_PNO, PNOEOM_EINVAL, "davidson: bad space");
  PNO_CHECK(opt.precision == PNOEOM_FP64 || opt.precision == PNOEOM_FP32 || opt.precision == PNOEOM_BF16,
            PNOEOM_EINVAL, "davidson: precision must be FP64, FP32 or BF16");
  PNO_CHECK(opt.space == PNOEOM_CANONICAL || c.pno.built, PNOEOM_ESTATE, "PNO Davidson before build_sapno");
  PNO_CHECK(opt.nextra >= 0 && nroots + opt.nextra <= c.ov(), PNOEOM_EINVAL, "davidson: bad nextra");
  const int nk = nroots + opt.nextra;
  PNO_CHECK(opt.max_sub >= 2 * nk, PNOEOM_EINVAL, "davidson: max_sub must be >= 2*(nroots+nextra)");
  hipStream_t s = c.stream;
  const int o = c.o, v = c.v;
  const int64_t ov = c.ov();
  // guess: CIS vectors (singles only), one per tracked root
  std::vector<double> w(nk);
  DBuf<double> cisv;
  cisv.alloc((int64_t)nk * ov);
  cis_roots(c, nk, w.data(), cisv);

  Operator op;
  DBuf<double> guess;
  if (opt.space == PNOEOM_CANONICAL) {
    op.N = c.vlen();
    guess.alloc((int64_t)nk * op.N);
    fill(s, (int64_t)nk * op.N, 0.0, guess);
    for (int k = 0; k < nk; ++k)
      PNO_HIP(hipMemcpyAsync(guess + (int64_t)k * op.N, cisv + (int64_t)k * ov, ov * sizeof(double),
                             hipMemcpyDeviceToDevice, s));
    op.project = [&](double* x) { symmetrize_r2(s, o, v, x + ov); };
    op.precond = [&](double* x, double th) {
      hipLaunchKernelGGL(precond_canonical_kernel, dim3(g1(op.N)), dim3(256), 0, s, o, v, (const double*)c.Foo,
                         (const double*)c.Fvv, th, x);
      PNO_HIP(hipGetLastError());
      symmetrize_r2(s, o, v, x + ov);
    };
  } else {
    op.N = c.pno.len;
    guess.alloc((int64_t)nk * op.N);
    DBuf<double> z2;
    z2.alloc(c.oovv());
    fill(s, c.oovv(), 0.0, z2);
    for (int k = 0; k < nk; ++k) pno_compress(c, 1, cisv + (int64_t)k * ov, z2, guess + (int64_t)k * op.N);
    PNO_HIP(hipStreamSynchronize(s));
    op.project = [&](double* x) { project_pno(c, x); };
    op.precond = [&](double* x, double th) { precond_pno(c, x, th); };
  }
  int prec = opt.precision;
  op.apply = [&](int nv, const double* X, double* S) {
    sigma_apply(c, opt.space, nv, X, S, op.N, prec);
    if (opt.space == PNOEOM_CANONICAL)
      for (int q = 0; q < nv; ++q) symmetrize_r2(s, o, v, S + (int64_t)q * op.N + ov);
  };
  // resume: the Ritz vectors of a checkpoint replace the CIS guess
  int phase0 = 0, nguess = nk;
  if (opt.resume_path) {
    const Checkpoint k = read_checkpoint(opt.resume_path);
    PNO_CHECK(k.N == op.N && k.space == opt.space, PNOEOM_EINVAL,
              "resume: the checkpoint is of another space or vector length");
    nguess = std::min(k.nvec, nk);
    PNO_HIP(hipMemcpyAsync(guess, k.x.data(), (size_t)nguess * op.N * sizeof(double), hipMemcpyHostToDevice, s));
    PNO_HIP(hipStreamSynchronize(s));
    phase0 = k.phase;
  }
  DBuf<double> xr;
  xr.alloc((int64_t)nroots * op.N);
  // a mixed phase that is refined afterwards stops at its own (looser) bounds
  pnoeom_davidson_opts mopt = opt;
  if (prec != PNOEOM_FP64 && opt.refine_fp64) {
    if (opt.mixed_tol_e > 0) mopt.tol_e = opt.mixed_tol_e;
    if (opt.mixed_tol_r > 0) mopt.tol_r = opt.mixed_tol_r;
  }
  const bool refine = prec != PNOEOM_FP64 && opt.refine_fp64;
  if (refine && phase0 == 1) {
    // a checkpoint of the refinement phase: continue there
    prec = PNOEOM_FP64;
    return run_davidson(c, op, nroots, guess, std::min(nguess, nroots), opt, "eom-fp64-refine", nullptr, 0, 0, 1);
  }
  auto record = [&](int ph, const DavidsonResult& rr, double secs) {
    Context::PhaseRecord& pr = c.dav_phase[ph];
    pr.omega = rr.omega;
    pr.resnorm = rr.resnorm;
    pr.iters = rr.iters;
    pr.nsigma = rr.nsigma;
    pr.n = (int)rr.omega.size();
    pr.seconds = secs;
  };
  c.dav_phase[0] = Context::PhaseRecord();
  c.dav_phase[1] = Context::PhaseRecord();
  const auto t0 = std::chrono::steady_clock::now();
  DavidsonResult r = run_davidson(c, op, nroots, guess, nguess, mopt,
                                  prec == PNOEOM_FP32 ? "eom-fp32" : prec == PNOEOM_BF16 ? "eom-bf16" : "eom", xr,
                                  opt.nextra);
  PNO_HIP(hipStreamSynchronize(s));
  const auto t1 = std::chrono::steady_clock::now();
  record(0, r, std::chrono::duration<double>(t1 - t0).count());
  if (refine && r.converged) {
    prec = PNOEOM_FP64;
    DavidsonResult r2 = run_davidson(c, op, nroots, xr, nroots, opt, "eom-fp64-refine", nullptr, 0, r.iters, 1);
    PNO_HIP(hipStreamSynchronize(s));
    record(1, r2, std::chrono::duration<double>(std::chrono::steady_clock::now() - t1).count());
    r2.iters += r.iters;
    r2.nsigma += r.nsigma;
    r = r2;
  }
  return r;
}

}  // namespace pnoeom
