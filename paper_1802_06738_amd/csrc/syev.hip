// Batched symmetric eigensolver for matrices above the size the one-workgroup Jacobi kernel
// handles (Methods: the per-pair eigenproblems of the averaged pair densities, whose kept
// eigenvectors are the PNOs, and the semicanonical rotations of the kept spaces).  Only the
// eigenvectors whose eigenvalue passes the truncation test are formed:
//   1. Householder reduction to tridiagonal form, one workgroup per matrix;
//   2. every eigenvalue by bisection on Sturm-sequence counts, one thread per eigenvalue;
//   3. the eigenvectors of the kept eigenvalues (|lambda| >= cut) of the tridiagonal matrix by
//      inverse iteration (partial-pivoting LU of T - lambda I, three solves from a fixed
//      pseudo-random start), each iterate orthogonalised (classical Gram-Schmidt; twice after
//      the last solve) against the earlier vectors of its cluster of close eigenvalues;
//   4. back-transform of those vectors by the stored reflectors, one wave per vector.
// The reduction reads the trailing block twice and writes it once per column (HBM/L2 bound,
// 4/3 n^3 flops); bisection is O(n^2) per matrix, inverse iteration O(n) per kept vector plus
// O(n c) for the c earlier vectors of its cluster.
#include <cfloat>
#include <cmath>

#include "context.h"

namespace pnoeom {
namespace {

constexpr int kTriThreads = 512;
constexpr int kMaxN = kSyevMaxN;
constexpr int kSlots = kMaxN / 64;   // vector elements per lane in the back-transform
constexpr int kInvIters = 3;

__device__ __forceinline__ double wave_sum(double x) {
  for (int m = 32; m > 0; m >>= 1) x += __shfl_xor(x, m, 64);
  return x;
}

// Sum over the workgroup, returned to every thread; red holds one entry per wave.
template <int NT>
__device__ __forceinline__ double block_sum(double x, double* red) {
  x = wave_sum(x);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = x;
  __syncthreads();
  double t = 0.0;
#pragma unroll
  for (int w = 0; w < NT / 64; ++w) t += red[w];
  return t;
}

template <int NT>
__device__ __forceinline__ double block_max(double x, double* red) {
  for (int m = 32; m > 0; m >>= 1) x = fmax(x, __shfl_xor(x, m, 64));
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = x;
  __syncthreads();
  double t = red[0];
#pragma unroll
  for (int w = 1; w < NT / 64; ++w) t = fmax(t, red[w]);
  return t;
}

// 1. A (n x n, row-major, leading dimension ld) -> T = Q^T A Q with Q = H_0 H_1 ... H_{n-2},
// H_k = I - tau_k v_k v_k^T acting on indices k+1..n-1.  On exit d[k] = T_kk, e[k] = T_{k,k+1},
// tau[k], and row k of A holds v_k in columns k+1..n-1 (v_k[k+1] = 1, stored).  The trailing
// block is kept in full (both triangles), so every row access is contiguous.
__global__ __launch_bounds__(kTriThreads) void tridiag_kernel(int ld, const int* __restrict__ nsz,
                                                              double* __restrict__ Aall, double* __restrict__ dall,
                                                              double* __restrict__ eall, double* __restrict__ tall) {
  constexpr int NW = kTriThreads / 64;
  const int mat = blockIdx.x;
  const int n = nsz[mat];
  double* A = Aall + (int64_t)mat * ld * ld;
  double* d = dall + (int64_t)mat * ld;
  double* e = eall + (int64_t)mat * ld;
  double* tau = tall + (int64_t)mat * ld;
  __shared__ double vs[kMaxN], ws[kMaxN];
  __shared__ double red[NW];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  if (n <= 0) return;
  for (int k = 0; k + 1 < n; ++k) {
    const int m = n - k - 1;
    double* xk = A + (int64_t)k * ld + k + 1;
    double s2 = 0.0;
    for (int i = 1 + tid; i < m; i += kTriThreads) s2 += xk[i] * xk[i];
    s2 = block_sum<kTriThreads>(s2, red);
    const double alpha = xk[0];
    double t = 0.0, beta = alpha, scal = 0.0;
    if (s2 > 0.0) {
      const double mu = sqrt(alpha * alpha + s2);
      beta = alpha >= 0.0 ? -mu : mu;
      t = (beta - alpha) / beta;
      scal = 1.0 / (alpha - beta);
    }
    for (int i = tid; i < m; i += kTriThreads) vs[i] = i == 0 ? 1.0 : xk[i] * scal;
    if (tid == 0) {
      d[k] = A[(int64_t)k * ld + k];
      e[k] = beta;
      tau[k] = t;
    }
    __syncthreads();
    for (int i = tid; i < m; i += kTriThreads) xk[i] = vs[i];
    if (t == 0.0) continue;  // H_k = I (uniform over the workgroup)
    double* A22 = A + (int64_t)(k + 1) * ld + (k + 1);
    // p = tau A22 v
    for (int r = wv; r < m; r += NW) {
      const double* row = A22 + (int64_t)r * ld;
      double acc = 0.0;
      for (int c = lane; c < m; c += 64) acc += row[c] * vs[c];
      acc = wave_sum(acc);
      if (lane == 0) ws[r] = t * acc;
    }
    __syncthreads();
    // w = p - (tau/2)(p.v) v
    double pv = 0.0;
    for (int i = tid; i < m; i += kTriThreads) pv += ws[i] * vs[i];
    pv = block_sum<kTriThreads>(pv, red);
    const double g = 0.5 * t * pv;
    for (int i = tid; i < m; i += kTriThreads) ws[i] -= g * vs[i];
    __syncthreads();
    // A22 -= v w^T + w v^T
    for (int r = wv; r < m; r += NW) {
      double* row = A22 + (int64_t)r * ld;
      const double vr = vs[r], wr = ws[r];
      for (int c = lane; c < m; c += 64) row[c] -= vr * ws[c] + wr * vs[c];
    }
    __syncthreads();
  }
  if (tid == 0) {
    d[n - 1] = A[(int64_t)(n - 1) * ld + (n - 1)];
    e[n - 1] = 0.0;
    tau[n - 1] = 0.0;
  }
}

// Number of eigenvalues of the tridiagonal (d, e2 = e^2) below x: the count of negative
// pivots of the LDL^T factorisation of T - x I, a pivot smaller than pivmin taken as -pivmin.
__device__ int sturm_count(int n, const double* d, const double* e2, double x, double pivmin) {
  double q = d[0] - x;
  if (fabs(q) < pivmin) q = -pivmin;
  int cnt = q < 0.0;
  for (int i = 1; i < n; ++i) {
    q = d[i] - x - e2[i - 1] / q;
    if (fabs(q) < pivmin) q = -pivmin;
    cnt += q < 0.0;
  }
  return cnt;
}

// 2. eigenvalue k (ascending) of matrix blockIdx.y, thread k of the grid row.  The interval
// starts from the Gershgorin bounds and is halved until it is below 2 eps ||T|| (the
// accuracy of the counts) or 2 eps |lambda|.
__global__ __launch_bounds__(256) void bisect_kernel(int ld, const int* __restrict__ nsz, const double* __restrict__ dall,
                                                     const double* __restrict__ eall, double* __restrict__ evall) {
  const int mat = blockIdx.y;
  const int n = nsz[mat];
  __shared__ double d[kMaxN], e2[kMaxN], ea[kMaxN];
  for (int i = threadIdx.x; i < n; i += 256) {
    d[i] = dall[(int64_t)mat * ld + i];
    const double x = i + 1 < n ? eall[(int64_t)mat * ld + i] : 0.0;
    e2[i] = x * x;
    ea[i] = fabs(x);
  }
  __syncthreads();
  const int k = blockIdx.x * 256 + threadIdx.x;
  if (k >= n) return;
  double lo = d[0], hi = d[0], maxe2 = 0.0;
  for (int i = 0; i < n; ++i) {
    const double r = ea[i] + (i > 0 ? ea[i - 1] : 0.0);
    lo = fmin(lo, d[i] - r);
    hi = fmax(hi, d[i] + r);
    maxe2 = fmax(maxe2, e2[i]);
  }
  const double tn = fmax(fabs(lo), fabs(hi));
  const double pivmin = DBL_MIN * fmax(1.0, maxe2);
  const double atol = 2.0 * DBL_EPSILON * tn;
  lo -= atol + 2.0 * pivmin;
  hi += atol + 2.0 * pivmin;
  for (int it = 0; it < 256; ++it) {
    const double mid = 0.5 * (lo + hi);
    if (hi - lo <= fmax(atol, 2.0 * DBL_EPSILON * fmax(fabs(lo), fabs(hi))) || mid <= lo || mid >= hi) break;
    if (sturm_count(n, d, e2, mid, pivmin) > k) hi = mid;
    else lo = mid;
  }
  evall[(int64_t)mat * ld + k] = 0.5 * (lo + hi);
}

__device__ __forceinline__ double start_value(int i, int k) {
  uint32_t h = (uint32_t)i * 0x9E3779B1u ^ ((uint32_t)k * 0x85EBCA77u + 0x27D4EB2Fu);
  h ^= h >> 16;
  h *= 0x7FEB352Du;
  h ^= h >> 15;
  h *= 0x846CA68Bu;
  h ^= h >> 16;
  return (double)h * (2.0 / 4294967296.0) - 1.0;
}

// 3. one workgroup per matrix: for each kept eigenvalue in ascending order, the eigenvector of
// the tridiagonal matrix into row k of Vt (rows of the eigenvalues not kept are zeroed).  A new
// cluster starts where the gap to the previous kept eigenvalue exceeds 1e-3 ||T||_1; inside a
// cluster a repeated eigenvalue is nudged up by 10 eps |lambda| + eps ||T|| so that the
// factorisations differ, and each iterate is orthogonalised against the cluster's earlier
// vectors (a zero matrix is one cluster).  Pivots below eps ||T|| are replaced by
// +-eps ||T||; each solve is rescaled to max |x| = 1 before the projections and normalised
// after them.
template <int NS>
__global__ __launch_bounds__(256) void inviter_kernel(int ld, const int* __restrict__ nsz, const double* __restrict__ dall,
                                                      const double* __restrict__ eall, const double* __restrict__ evall,
                                                      double cut, double* __restrict__ Vtall) {
  const int mat = blockIdx.x;
  const int n = nsz[mat];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  __shared__ double d[kMaxN], e[kMaxN];
  __shared__ double fd[kMaxN], fu[kMaxN], fu2[kMaxN], fl[kMaxN];
  __shared__ unsigned char pv[kMaxN];
  __shared__ double x[kMaxN];
  __shared__ int mem[kMaxN];
  __shared__ double red[4];
  if (n <= 0) return;
  const double* ev = evall + (int64_t)mat * ld;
  double* Vt = Vtall + (int64_t)mat * ld * ld;
  double tloc = 0.0;
  for (int i = tid; i < n; i += 256) {
    d[i] = dall[(int64_t)mat * ld + i];
    e[i] = i + 1 < n ? eall[(int64_t)mat * ld + i] : 0.0;
  }
  __syncthreads();
  for (int i = tid; i < n; i += 256) tloc = fmax(tloc, fabs(d[i]) + fabs(e[i]) + (i > 0 ? fabs(e[i - 1]) : 0.0));
  const double tn = block_max<256>(tloc, red);
  const double tiny = fmax(DBL_EPSILON * tn, DBL_MIN);
  const double ortol = 1e-3 * tn;
  int nclus = 0;
  double prev = 0.0, prev_used = 0.0;
  for (int k = 0; k < n; ++k) {
    const double lam = ev[k];
    double* row = Vt + (int64_t)k * ld;
    if (!(fabs(lam) >= cut)) {
      for (int i = tid; i < n; i += 256) row[i] = 0.0;
      continue;
    }
    if (nclus > 0 && lam - prev > fmax(ortol, tiny)) nclus = 0;
    double lu = lam;
    const double pert = 10.0 * DBL_EPSILON * fabs(lam) + tiny;
    if (nclus > 0 && lu < prev_used + pert) lu = prev_used + pert;
    prev = lam;
    prev_used = lu;
    if (tid == 0) {
      // LU with partial pivoting of T - lu I; the running pivot row is carried in registers
      // (dc: its diagonal, uc: its superdiagonal), the reciprocal pivots go to fd
      double dc = d[0] - lu, uc = n > 1 ? e[0] : 0.0;
#pragma unroll 4
      for (int i = 0; i + 1 < n; ++i) {
        const double l = e[i], dn = d[i + 1] - lu, un = i + 2 < n ? e[i + 1] : 0.0;
        double piv;
        if (fabs(dc) >= fabs(l)) {
          if (dc == 0.0) dc = tiny;
          const double f = l / dc;
          piv = dc;
          fl[i] = f;
          fu[i] = uc;
          fu2[i] = 0.0;
          pv[i] = 0;
          dc = dn - f * uc;
          uc = un;
        } else {
          const double f = dc / l;
          piv = l;
          fl[i] = f;
          fu[i] = dn;
          fu2[i] = un;
          pv[i] = 1;
          dc = uc - f * dn;
          uc = -f * un;
        }
        if (fabs(piv) < tiny) piv = piv >= 0.0 ? tiny : -tiny;
        fd[i] = 1.0 / piv;
      }
      if (fabs(dc) < tiny) dc = dc >= 0.0 ? tiny : -tiny;
      fd[n - 1] = 1.0 / dc;
    }
    for (int i = tid; i < n; i += 256) x[i] = start_value(i, k);
    __syncthreads();
    for (int it = 0; it < kInvIters; ++it) {
      if (tid == 0) {
        // forward: the row interchanges and multipliers, the running entry in a register
        double cur = x[0];
#pragma unroll 4
        for (int i = 0; i + 1 < n; ++i) {
          const double nx = x[i + 1];
          if (!pv[i]) {
            x[i] = cur;
            cur = nx - fl[i] * cur;
          } else {
            x[i] = nx;
            cur = cur - fl[i] * nx;
          }
        }
        // backward: the upper factor with two superdiagonals
        double x2 = cur * fd[n - 1], x1 = 0.0;
        x[n - 1] = x2;
        if (n > 1) {
          x1 = (x[n - 2] - fu[n - 2] * x2) * fd[n - 2];
          x[n - 2] = x1;
        }
#pragma unroll 4
        for (int i = n - 3; i >= 0; --i) {
          const double xi = (x[i] - fu[i] * x1 - fu2[i] * x2) * fd[i];
          x[i] = xi;
          x2 = x1;
          x1 = xi;
        }
      }
      __syncthreads();
      // scale to max |x| = 1 before the projections
      double mx = 0.0;
      for (int i = tid; i < n; i += 256) mx = fmax(mx, fabs(x[i]));
      mx = block_max<256>(mx, red);
      const double inv = mx > 0.0 ? 1.0 / mx : 0.0;
      for (int i = tid; i < n; i += 256) x[i] *= inv;
      __syncthreads();
      // x -= Z Z^T x over the cluster's earlier vectors Z (rows mem[] of Vt): once per
      // iteration, twice in the last.  Wave w takes members w, w + 4, ..., four at a time: one
      // coalesced read of each member row gives both its coefficient (against the x of this
      // pass, held in registers) and its share of the update; the four waves' shares are
      // subtracted in turn.
      const int passes = it + 1 < kInvIters ? 1 : 2;
      for (int pass = 0; pass < passes && nclus > 0; ++pass) {
        double xr[NS], up[NS];
#pragma unroll
        for (int q = 0; q < NS; ++q) {
          const int i = lane + 64 * q;
          xr[q] = i < n ? x[i] : 0.0;
          up[q] = 0.0;
        }
        for (int p = wv; p < nclus; p += 16) {
          double z[4][NS], a[4];
#pragma unroll
          for (int m = 0; m < 4; ++m) {
            const int pm = p + 4 * m;
            const double* zr = Vt + (int64_t)mem[pm < nclus ? pm : p] * ld;
            a[m] = 0.0;
#pragma unroll
            for (int q = 0; q < NS; ++q) {
              const int i = lane + 64 * q;
              z[m][q] = (pm < nclus && i < n) ? zr[i] : 0.0;
              a[m] += z[m][q] * xr[q];
            }
          }
#pragma unroll
          for (int m = 0; m < 4; ++m) a[m] = wave_sum(a[m]);
#pragma unroll
          for (int q = 0; q < NS; ++q) up[q] += a[0] * z[0][q] + a[1] * z[1][q] + a[2] * z[2][q] + a[3] * z[3][q];
        }
        for (int w = 0; w < 4; ++w) {
          if (wv == w) {
#pragma unroll
            for (int q = 0; q < NS; ++q) {
              const int i = lane + 64 * q;
              if (i < n) x[i] -= up[q];
            }
          }
          __syncthreads();
        }
      }
      double s = 0.0;
      for (int i = tid; i < n; i += 256) s += x[i] * x[i];
      s = block_sum<256>(s, red);
      const double sc = s > 0.0 ? 1.0 / sqrt(s) : 0.0;
      for (int i = tid; i < n; i += 256) x[i] *= sc;
      __syncthreads();
    }
    for (int i = tid; i < n; i += 256) row[i] = x[i];
    if (tid == 0) mem[nclus] = k;
    ++nclus;
    __syncthreads();
  }
}

// 4. row k of Vt (an eigenvector of T, wave w of workgroup (mat, y) takes k = 4 y + w) ->
// Q times it, applying H_{n-2}, ..., H_0; the vector stays in registers, kSlots per lane.
__global__ __launch_bounds__(256) void backxf_kernel(int ld, const int* __restrict__ nsz, const double* __restrict__ Aall,
                                                     const double* __restrict__ tall, const double* __restrict__ evall,
                                                     double cut, double* __restrict__ Vtall) {
  const int mat = blockIdx.x;
  const int n = nsz[mat];
  const int lane = threadIdx.x & 63;
  const int k = blockIdx.y * 4 + (threadIdx.x >> 6);
  if (k >= n || !(fabs(evall[(int64_t)mat * ld + k]) >= cut)) return;
  const double* A = Aall + (int64_t)mat * ld * ld;
  const double* tau = tall + (int64_t)mat * ld;
  double* row = Vtall + ((int64_t)mat * ld + k) * ld;
  double y[kSlots];
#pragma unroll
  for (int s = 0; s < kSlots; ++s) {
    const int i = lane + 64 * s;
    y[s] = i < n ? row[i] : 0.0;
  }
  for (int j = n - 2; j >= 0; --j) {
    const double t = tau[j];
    if (t == 0.0) continue;
    const double* v = A + (int64_t)j * ld;
    double vr[kSlots];
    double acc = 0.0;
#pragma unroll
    for (int s = 0; s < kSlots; ++s) {
      vr[s] = 0.0;
      if (64 * s + 63 > j && 64 * s < n) {
        const int i = lane + 64 * s;
        if (i > j && i < n) vr[s] = v[i];
        acc += vr[s] * y[s];
      }
    }
    acc = t * wave_sum(acc);
#pragma unroll
    for (int s = 0; s < kSlots; ++s) y[s] -= acc * vr[s];
  }
#pragma unroll
  for (int s = 0; s < kSlots; ++s) {
    const int i = lane + 64 * s;
    if (i < n) row[i] = y[s];
  }
}

}  // namespace

void syev_tridiag(hipStream_t s, int nmat, const int* dn, int nmax, int ld, double* A, double* Vt, double* ev,
                  double cut) {
  PNO_CHECK(nmax <= kSyevMaxN && nmax <= ld, PNOEOM_EINVAL, "syev: matrix larger than the tridiagonal solver's limit");
  if (nmat <= 0 || nmax <= 0) return;
  DBuf<double> d, e, t;
  d.alloc((int64_t)nmat * ld);
  e.alloc((int64_t)nmat * ld);
  t.alloc((int64_t)nmat * ld);
  hipLaunchKernelGGL(tridiag_kernel, dim3(nmat), dim3(kTriThreads), 0, s, ld, dn, A, (double*)d, (double*)e,
                     (double*)t);
  PNO_HIP(hipGetLastError());
  hipLaunchKernelGGL(bisect_kernel, dim3((nmax + 255) / 256, nmat), dim3(256), 0, s, ld, dn, (const double*)d,
                     (const double*)e, ev);
  PNO_HIP(hipGetLastError());
  if (nmax <= 512)
    hipLaunchKernelGGL(inviter_kernel<8>, dim3(nmat), dim3(256), 0, s, ld, dn, (const double*)d, (const double*)e,
                       (const double*)ev, cut, Vt);
  else
    hipLaunchKernelGGL(inviter_kernel<kSlots>, dim3(nmat), dim3(256), 0, s, ld, dn, (const double*)d,
                       (const double*)e, (const double*)ev, cut, Vt);
  PNO_HIP(hipGetLastError());
  hipLaunchKernelGGL(backxf_kernel, dim3(nmat, (nmax + 3) / 4), dim3(256), 0, s, ld, dn, (const double*)A,
                     (const double*)t, (const double*)ev, cut, Vt);
  PNO_HIP(hipGetLastError());
  PNO_HIP(hipStreamSynchronize(s));
}

}  // namespace pnoeom
