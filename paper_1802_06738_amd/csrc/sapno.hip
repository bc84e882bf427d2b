// State-averaged PNOs and the PNO-projected Davidson space (Methods: CIS(D) doubles,
// state-specific pair densities, their state average, PNO truncation, OSVs from the
// diagonal pairs, semicanonical bases; the residual projection / back-transform of
// the PNO simulation).
//
// Densities: for each averaged CIS root k the doubles B_(k) = K_(k) / (w_k + e_i + e_j
// - e_a - e_b) come from the DF factors (K is the sigma-doubles of R1 = b_k at T = 0,
// i.e. the (ai|bj) response to the one-index transformation by b_k); the pair
// densities D^{ij} += 2/(1+d_ij)/N (B Bt^T + B^T Bt), Bt = 2B - B^T, are batched MFMA
// GEMMs over all pairs.  Per-pair eigenproblems up to n = 128 use a batched cyclic parallel
// Jacobi method (one workgroup per matrix, Brent-Luk round-robin ordering), which keeps
// small occupation numbers to high relative accuracy; larger ones the batched tridiagonal
// solver of syev.hip, which forms only the eigenvectors the truncation keeps (occupations
// to eps times the largest).  Compressed vectors hold the
// singles blocks U^i^T r^i, then the pair blocks w_p U^p^T R^{ij} U^p for i <= j
// (w_p = sqrt 2 for i < j, 1 for i = j), so plain dot products are the full-array
// Frobenius inner product.
#include <algorithm>
#include <cmath>

#include <thread>

#include "context.h"

namespace pnoeom {
namespace {

constexpr double kClamp = 1e-4;

__device__ __forceinline__ double clampd(double d) {
  if (fabs(d) < kClamp) return d >= 0.0 ? kClamp : -kClamp;
  return d;
}

unsigned gsz(int64_t n) {
  int64_t b = (n + 255) / 256;
  if (b > 65536) b = 65536;
  if (b < 1) b = 1;
  return (unsigned)b;
}

void gm(hipStream_t s, bool ta, bool tb, int64_t M, int64_t N, int64_t K, double alpha, const double* A,
        int64_t lda, int64_t sA, const double* B, int64_t ldb, int64_t sB, double beta, double* C, int64_t ldc,
        int64_t sC, int64_t batch) {
  GemmDesc<double> d;
  d.ta = ta; d.tb = tb; d.M = M; d.N = N; d.K = K; d.alpha = alpha; d.beta = beta;
  d.A = A; d.lda = lda; d.sA = sA; d.B = B; d.ldb = ldb; d.sB = sB; d.C = C; d.ldc = ldc; d.sC = sC;
  d.batch = batch;
  gemm(d, s);
}

void perm(hipStream_t s, const double* in, int64_t a, int64_t b, int64_t c, int64_t d, int p0, int p1, int p2,
          int p3, double* out, double alpha = 1.0, double beta = 0.0) {
  const int64_t dims[4] = {a, b, c, d};
  const int pp[4] = {p0, p1, p2, p3};
  permute_c(s, dims, pp, alpha, in, beta, out);
}

// t[i][j][a][b] = K / clamp(w + e_i + e_j - e_a - e_b)
__global__ void cisd_div_kernel(int o, int v, const double* __restrict__ eps, double w, const double* __restrict__ K,
                                double* __restrict__ t) {
  const int64_t n = (int64_t)o * o * v * v;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
    int64_t r = e;
    const int b = (int)(r % v); r /= v;
    const int a = (int)(r % v); r /= v;
    const int j = (int)(r % o); r /= o;
    const int i = (int)r;
    t[e] = K[e] / clampd(w + eps[i] + eps[j] - eps[o + a] - eps[o + b]);
  }
}

// Dp[p] = scale_p * D[i_p][j_p] for the pairs i <= j
__global__ void gather_pairs_kernel(int o, int v, int npair, const int* __restrict__ pi, const int* __restrict__ pj,
                                    double inv_n, const double* __restrict__ D, double* __restrict__ Dp) {
  const int64_t vv = (int64_t)v * v;
  const int64_t n = (int64_t)npair * vv;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
    const int p = (int)(e / vv);
    const int64_t r = e % vv;
    const int i = pi[p], j = pj[p];
    const double sc = (i == j ? 1.0 : 2.0) * inv_n;
    Dp[e] = sc * D[((int64_t)i * o + j) * vv + r];
  }
}

// Batched symmetric eigensolver: cyclic parallel Jacobi, one 256-thread workgroup per
// matrix.  A[m] (n_m x n_m, leading dimension ld, stride ld*ld) is overwritten; on exit
// eval[m*ld + k] holds eigenvalue k and Vt[m] row k the unit eigenvector k.
__global__ __launch_bounds__(256) void jacobi_kernel(int ld, const int* __restrict__ nsz, double* __restrict__ Aall,
                                                     double* __restrict__ Vtall, double* __restrict__ evall,
                                                     int max_sweeps) {
  const int m = blockIdx.x;
  const int n = nsz[m];
  double* A = Aall + (int64_t)m * ld * ld;
  double* Vt = Vtall + (int64_t)m * ld * ld;
  double* ev = evall + (int64_t)m * ld;
  const int tid = threadIdx.x;
  __shared__ double cs[1024], sn[1024];
  __shared__ int pp[1024], qq[1024];
  __shared__ double red[256];
  __shared__ int done;
  if (n <= 0) return;
  for (int64_t e = tid; e < (int64_t)n * n; e += 256) Vt[(e / n) * ld + (e % n)] = (e / n == e % n) ? 1.0 : 0.0;
  const int np = (n + 1) & ~1;  // players, padded to even
  const int half = np / 2;
  __syncthreads();
  for (int sweep = 0; sweep < max_sweeps; ++sweep) {
    // convergence test: off-diagonal Frobenius norm vs the whole matrix
    double off = 0.0, all = 0.0;
    for (int64_t e = tid; e < (int64_t)n * n; e += 256) {
      const int i = (int)(e / n), j = (int)(e % n);
      const double x = A[(int64_t)i * ld + j];
      all += x * x;
      if (i != j) off += x * x;
    }
    red[tid] = off;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
      if (tid < w) red[tid] += red[tid + w];
      __syncthreads();
    }
    const double offs = red[0];
    __syncthreads();
    red[tid] = all;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
      if (tid < w) red[tid] += red[tid + w];
      __syncthreads();
    }
    if (tid == 0) done = (offs <= 1e-30 * red[0] || offs == 0.0) ? 1 : 0;
    __syncthreads();
    if (done) break;
    for (int round = 0; round < np - 1; ++round) {
      for (int k = tid; k < half; k += 256) {
        int p, q;
        if (k == 0) { p = np - 1; q = round; }
        else { p = (round + k) % (np - 1); q = (round - k + (np - 1)) % (np - 1); }
        if (p > q) { const int t = p; p = q; q = t; }
        double c = 1.0, s = 0.0;
        if (q < n) {
          const double apq = A[(int64_t)p * ld + q];
          if (apq != 0.0) {
            const double app = A[(int64_t)p * ld + p], aqq = A[(int64_t)q * ld + q];
            const double th = (aqq - app) / (2.0 * apq);
            const double t = (th >= 0 ? 1.0 : -1.0) / (fabs(th) + sqrt(th * th + 1.0));
            c = 1.0 / sqrt(t * t + 1.0);
            s = t * c;
          }
        }
        pp[k] = p; qq[k] = q; cs[k] = c; sn[k] = s;
      }
      __syncthreads();
      // rows: A <- J^T A ; Vt <- J^T Vt
      for (int64_t e = tid; e < (int64_t)half * n; e += 256) {
        const int k = (int)(e / n), j = (int)(e % n);
        const int p = pp[k], q = qq[k];
        if (q >= n || sn[k] == 0.0) continue;
        const double c = cs[k], s = sn[k];
        double* ap = A + (int64_t)p * ld;
        double* aq = A + (int64_t)q * ld;
        const double x = ap[j], y = aq[j];
        ap[j] = c * x - s * y;
        aq[j] = s * x + c * y;
        double* vp = Vt + (int64_t)p * ld;
        double* vq = Vt + (int64_t)q * ld;
        const double vx = vp[j], vy = vq[j];
        vp[j] = c * vx - s * vy;
        vq[j] = s * vx + c * vy;
      }
      __syncthreads();
      // columns: A <- A J
      for (int64_t e = tid; e < (int64_t)half * n; e += 256) {
        const int k = (int)(e % half), i = (int)(e / half);
        const int p = pp[k], q = qq[k];
        if (q >= n || sn[k] == 0.0) continue;
        const double c = cs[k], s = sn[k];
        double* ai = A + (int64_t)i * ld;
        const double x = ai[p], y = ai[q];
        ai[p] = c * x - s * y;
        ai[q] = s * x + c * y;
      }
      __syncthreads();
    }
  }
  for (int k = tid; k < n; k += 256) ev[k] = A[(int64_t)k * ld + k];
}

// U0[a][c] = Vt[m][idx[c]][a] for the kept columns of each matrix (rows of Vt)
__global__ void gather_kept_kernel(int ld, int v, int nsel, const int* __restrict__ mat, const int* __restrict__ row,
                                   const int64_t* __restrict__ off, const int* __restrict__ col, const int* __restrict__ ncol,
                                   const double* __restrict__ Vt, double* __restrict__ U) {
  const int64_t total = (int64_t)nsel * v;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int t = (int)(e / v), a = (int)(e % v);
    U[off[t] + (int64_t)a * ncol[t] + col[t]] = Vt[((int64_t)mat[t] * ld + row[t]) * ld + a];
  }
}

// Second stage of the back-transform, one pair block per workgroup row and one 64 x 64 tile
// (a, b) of it per workgroup: R^{ij}[a][b] = w sum_d T_p[a][d] U_p[b][d] (T_p = U_p X_p, both
// v x n_p row-major; w = 1 on diagonal pairs, 1/sqrt 2 off the diagonal), written into
// r2[i][j][a][b] and, for i < j, into r2[j][i][b][a] through an LDS copy of the tile so that
// both writes run along rows.  Every element of r2 belongs to one tile of one pair (a pair
// with n_p = 0 writes zeros), so the array needs no clearing and no mirror pass.
// FP64 MFMA 16x16x4: 4 waves in 2 x 2, each a 32 x 32 block; operand lane l supplies
// A[l%16][k0 + l/16] and B[k0 + l/16][l%16], accumulator r holds row l/16 + 4 r, column l%16.
constexpr int kXT = 64, kXK = 16;
__global__ __launch_bounds__(256) void expand_pairs_kernel(int o, int v, const int64_t* __restrict__ xpair,
                                                           const double* __restrict__ Tw,
                                                           const double* __restrict__ U, double w_off,
                                                           double* __restrict__ r2) {
  typedef double v4 __attribute__((ext_vector_type(4)));
  __shared__ double As[kXK][kXT + 1];
  __shared__ double Bs[kXK][kXT + 1];
  __shared__ double Cs[kXT][kXT + 1];
  const int64_t* d = xpair + 5 * (int64_t)blockIdx.y;
  const int i = (int)d[0], j = (int)d[1], n = (int)d[2];
  const double* T = Tw + d[3];
  const double* Up = U + d[4];
  const int nt = (v + kXT - 1) / kXT;
  const int a0 = (int)(blockIdx.x / nt) * kXT, b0 = (int)(blockIdx.x % nt) * kXT;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, wm = wave >> 1, wn = wave & 1;
  const int lr = lane & 15, lk = lane >> 4;
  v4 acc[2][2];
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y) acc[x][y] = v4{0.0, 0.0, 0.0, 0.0};
  // the next K-step's operands are loaded into registers while the current one is used
  constexpr int kL = kXT * kXK / 256;
  double ra[kL], rb[kL];
  auto gload = [&](int k0) {
#pragma unroll
    for (int q = 0; q < kL; ++q) {
      const int e = tid + 256 * q, r = e / kXK, k = e % kXK;
      ra[q] = (a0 + r < v && k0 + k < n) ? T[(int64_t)(a0 + r) * n + k0 + k] : 0.0;
      rb[q] = (b0 + r < v && k0 + k < n) ? Up[(int64_t)(b0 + r) * n + k0 + k] : 0.0;
    }
  };
  if (n > 0) gload(0);
  for (int k0 = 0; k0 < n; k0 += kXK) {
#pragma unroll
    for (int q = 0; q < kL; ++q) {
      const int e = tid + 256 * q, r = e / kXK, k = e % kXK;
      As[k][r] = ra[q];
      Bs[k][r] = rb[q];
    }
    __syncthreads();
    if (k0 + kXK < n) gload(k0 + kXK);
#pragma unroll
    for (int kk = 0; kk < kXK; kk += 4) {
      double av[2], bv[2];
#pragma unroll
      for (int x = 0; x < 2; ++x) av[x] = As[kk + lk][wm * 32 + x * 16 + lr];
#pragma unroll
      for (int y = 0; y < 2; ++y) bv[y] = Bs[kk + lk][wn * 32 + y * 16 + lr];
#pragma unroll
      for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y) acc[x][y] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[x], bv[y], acc[x][y], 0, 0, 0);
    }
    __syncthreads();
  }
  const double w = i == j ? 1.0 : w_off;
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int r = 0; r < 4; ++r) Cs[wm * 32 + x * 16 + lk + 4 * r][wn * 32 + y * 16 + lr] = w * acc[x][y][r];
  __syncthreads();
  const int64_t vv = (int64_t)v * v;
  double* Rij = r2 + ((int64_t)i * o + j) * vv;
  for (int e = tid; e < kXT * kXT; e += 256) {
    const int a = e / kXT, b = e % kXT;
    if (a0 + a < v && b0 + b < v) Rij[(int64_t)(a0 + a) * v + b0 + b] = Cs[a][b];
  }
  if (i != j) {
    double* Rji = r2 + ((int64_t)j * o + i) * vv;
    for (int e = tid; e < kXT * kXT; e += 256) {
      const int b = e / kXT, a = e % kXT;
      if (a0 + a < v && b0 + b < v) Rji[(int64_t)(b0 + b) * v + a0 + a] = Cs[a][b];
    }
  }
}

// x[e] /= clamp(theta + base[e])
__global__ void precond_pno_kernel(int64_t n, double theta, const double* __restrict__ base, double* __restrict__ x) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
    x[e] /= clampd(theta + base[e]);
}

// symmetrise the diagonal pair blocks of a compressed vector
__global__ void sym_diag_blocks_kernel(int ndiag, const int64_t* __restrict__ off, const int* __restrict__ nd,
                                       double* __restrict__ x) {
  const int b = blockIdx.x;  // (diagonal block b, slice blockIdx.y of its elements)
  if (b >= ndiag) return;
  const int n = nd[b];
  double* X = x + off[b];
  for (int64_t e = blockIdx.y * (int64_t)blockDim.x + threadIdx.x; e < (int64_t)n * n;
       e += (int64_t)gridDim.y * blockDim.x) {
    const int i = (int)(e / n), j = (int)(e % n);
    if (i < j) {
      const double m = 0.5 * (X[(int64_t)i * n + j] + X[(int64_t)j * n + i]);
      X[(int64_t)i * n + j] = m;
      X[(int64_t)j * n + i] = m;
    }
  }
}

}  // namespace

// Batched symmetric eigenproblems of matrices up to nmax: the one-workgroup Jacobi kernel
// while its O(n^3) HBM traffic per sweep is small (n <= kJacobiMaxN); above that the GPU
// tridiagonal solver (syev.hip; eigenvectors only of eigenvalues with |lambda| >= cut), or,
// with backend 1 or beyond kSyevMaxN, the host solver in parallel threads (Householder
// tridiagonalisation + implicit QR, csrc/eig.cpp).  Same output layout in every case.
constexpr int kJacobiMaxN = 128;

void batched_syev(hipStream_t s, int backend, int nmat, const std::vector<int>& nsz, int ld, double* A, double* Vt,
                  double* ev, int* dn, double cut) {
  int nmax = 0;
  for (int m = 0; m < nmat; ++m) nmax = std::max(nmax, nsz[m]);
  if (nmax <= kJacobiMaxN || (backend == 0 && nmax <= kSyevMaxN)) {
    PNO_HIP(hipMemcpyAsync(dn, nsz.data(), nmat * sizeof(int), hipMemcpyHostToDevice, s));
    if (nmax <= kJacobiMaxN) {
      hipLaunchKernelGGL(jacobi_kernel, dim3(nmat), dim3(256), 0, s, ld, (const int*)dn, A, Vt, ev, 60);
      PNO_HIP(hipGetLastError());
      PNO_HIP(hipStreamSynchronize(s));
    } else {
      syev_tridiag(s, nmat, dn, nmax, ld, A, Vt, ev, cut);
    }
    return;
  }
  const size_t tot = (size_t)nmat * ld * ld;
  std::vector<double> Ah(tot), Vh(tot, 0.0), eh((size_t)nmat * ld, 0.0);
  PNO_HIP(hipMemcpyAsync(Ah.data(), A, tot * sizeof(double), hipMemcpyDeviceToHost, s));
  PNO_HIP(hipStreamSynchronize(s));
  const int hw = (int)std::thread::hardware_concurrency();
  const int nthreads = std::max(1, std::min(16, hw));
  const int st = host_syev_batched(nmat, nsz.data(), ld, Ah.data(), eh.data(), Vh.data(), nthreads);
  PNO_CHECK(st == PNOEOM_OK, st, "build_sapno: symmetric eigensolver did not converge");
  PNO_HIP(hipMemcpyAsync(Vt, Vh.data(), tot * sizeof(double), hipMemcpyHostToDevice, s));
  PNO_HIP(hipMemcpyAsync(ev, eh.data(), eh.size() * sizeof(double), hipMemcpyHostToDevice, s));
  PNO_HIP(hipStreamSynchronize(s));
}

// ----------------------------------------------------------------------------- build
namespace {
// Native ladder of the pairs with n_p <= kNatSmall in one kernel: workgroup (ch, g) forms the
// partial sum over Q in [ch kNatQ, ch kNatQ + kNatQ) of Bbar^Q Rbar Bbar^Q^T for small pair g
// (tab[4 g ..]: n, Bbar offset, offset of Rbar in x, partial-block offset), FP64, without the
// Y1 intermediate.  The 256 threads form 256 / n^2 lanes of n^2 threads, one (a, b) each; lane
// l takes every (256 / n^2)-th Q: T = Bbar^Q Rbar into LDS, then S[a][b] += T[a][:] . Bbar^Q[b][:].
constexpr int kNatSmall = 16, kNatQ = 64;
__global__ __launch_bounds__(256) void native_small_kernel(int naux, const int64_t* __restrict__ tab,
                                                           const double* __restrict__ Bbar,
                                                           const double* __restrict__ x, double* __restrict__ part) {
  __shared__ double Rs[kNatSmall * kNatSmall];
  __shared__ double Bq[256];
  __shared__ double Ts[256];
  const int64_t* t = tab + 4 * (int64_t)blockIdx.y;
  const int n = (int)t[0];
  const int64_t boff = t[1], roff = t[2], poff = t[3];
  const int n2 = n * n, nl = 256 / n2;
  const int tid = threadIdx.x, lane = tid / n2, e = tid % n2, a = e / n, b = e % n;
  const bool act = lane < nl;
  const int q0 = blockIdx.x * kNatQ, q1 = min(q0 + kNatQ, naux);
  for (int i = tid; i < n2; i += 256) Rs[i] = x[roff + i];
  double acc = 0.0;
  const int steps = (q1 - q0 + nl - 1) / nl;
  // this thread's element of Bbar^Q at step st; the elements of the next kPre steps are loaded
  // while the current ones are used
  constexpr int kPre = 8;
  auto bval = [&](int st) -> double {
    const int Q = q0 + st * nl + lane;
    return act && st < steps && Q < q1 ? Bbar[boff + ((int64_t)a * naux + Q) * n + b] : 0.0;
  };
  double cur[kPre], nxt[kPre];
#pragma unroll
  for (int k = 0; k < kPre; ++k) cur[k] = bval(k);
  for (int g0 = 0; g0 < steps; g0 += kPre) {
#pragma unroll
    for (int k = 0; k < kPre; ++k) nxt[k] = bval(g0 + kPre + k);
#pragma unroll
    for (int k = 0; k < kPre; ++k) {
      if (g0 + k >= steps) break;  // (uniform)
      __syncthreads();  // Rs written; the previous step's reads of Bq and Ts done
      if (act) Bq[lane * n2 + e] = cur[k];
      __syncthreads();
      if (act) {
        double sm = 0.0;
        for (int c = 0; c < n; ++c) sm += Bq[lane * n2 + a * n + c] * Rs[c * n + b];
        Ts[lane * n2 + e] = sm;
      }
      __syncthreads();
      if (act) {
        double sm = 0.0;
        for (int d = 0; d < n; ++d) sm += Ts[lane * n2 + a * n + d] * Bq[lane * n2 + b * n + d];
        acc += sm;
      }
    }
#pragma unroll
    for (int k = 0; k < kPre; ++k) cur[k] = nxt[k];
  }
  __syncthreads();
  if (act) Ts[lane * n2 + e] = acc;
  __syncthreads();
  if (tid < n2) {
    double sm = 0.0;
    for (int l = 0; l < nl; ++l) sm += Ts[l * n2 + tid];
    part[poff + (int64_t)blockIdx.x * n2 + tid] = sm;
  }
}

// y[yoff[g] + e] += sum_ch part[poff[g] + ch n^2 + e] for e < n^2 = nn[g]^2 (one workgroup per pair g)
__global__ void sum_chunks_kernel(const int* __restrict__ nn, const int* __restrict__ nch,
                                  const int64_t* __restrict__ poff, const int64_t* __restrict__ yoff,
                                  const double* __restrict__ part, double* __restrict__ y) {
  const int g = blockIdx.x;
  const int64_t n2 = (int64_t)nn[g] * nn[g];
  const double* pp = part + poff[g];
  double* yy = y + yoff[g];
  for (int64_t e = threadIdx.x; e < n2; e += blockDim.x) {
    double acc = 0.0;
    for (int ch = 0; ch < nch[g]; ++ch) acc += pp[ch * n2 + e];
    yy[e] += acc;
  }
}

// Ladder of the small pairs in the PNO space (the reduced-cost sigma the Methods section
// points to).  W_ab^cd = sum_Q B~^Q_ac B~^Q_bd, so the projected ladder of a pair is
//   U^T [sum_cd W_abcd (U Rbar U^T)_cd] U = sum_Q Bbar^Q Rbar Bbar^Q^T,  Bbar^Q = U^T B~^Q U,
// exactly: 4 n^3 naux flop per pair instead of the v(v+1)/2 x v(v+1)/2 packed rows of the
// canonical ladder (~v^4).  Pairs with n_p up to the cut (where 128 n^3 naux = v^4: the
// grouped 64 x 64 kernel on n x n blocks, n ~ 10-50, runs at 1-3 TFLOP/s against 40-60
// for the large canonical GEMM) take this route; the others keep the canonical ladder.  Bbar_p is stored [a][Q][c] so that both products
// are plain GEMMs: Y1 = Bbar_p (rows (a,Q)) Rbar, sigma_p += Y1 (n x naux n) Bbar_p^T.
void build_native_ladder(Context& c, const std::vector<int>& pi, const std::vector<int>& pj) {
  PNOData& P = c.pno;
  hipStream_t s = c.stream;
  const int o = c.o, v = c.v, naux = c.naux, nmo = c.nmo;
  const int npair = o * (o + 1) / 2;
  const int64_t n2 = (int64_t)nmo * nmo;
  int cut = P.nat_max;
  if (cut < 0) cut = (int)std::floor(std::cbrt((double)v * v * v * v / (128.0 * naux)));
  // memory: Bbar and Y1 take 2 sum n^2 naux words; keep them within a fifth of the free HBM
  size_t fr = 0, tot = 0;
  PNO_HIP(hipMemGetInfo(&fr, &tot));
  auto words = [&](int k) {
    int64_t w = 0;
    for (int p = 0; p < npair; ++p)
      if (P.npno[p] > 0 && P.npno[p] <= k) w += (int64_t)P.npno[p] * P.npno[p] * naux;
    return w;
  };
  while (cut > 0 && 16.0 * (double)words(cut) > 0.2 * (double)fr) cut = cut * 3 / 4;
  P.nat_cut = cut;
  P.prow.assign(npair, -1);
  std::vector<int64_t> boff(npair, -1);
  int64_t bw = 0;
  int nmax = 0;
  P.nat_pairs = P.canon_pairs = 0;
  P.nat_flops = 0;
  for (int p = 0; p < npair; ++p) {
    const int n = P.npno[p];
    if (n > 0 && n <= cut) {
      boff[p] = bw;
      bw += (int64_t)n * n * naux;
      nmax = std::max(nmax, n);
      ++P.nat_pairs;
      P.nat_flops += 4.0 * (double)n * n * n * naux;
    } else if (n > 0) {
      P.prow[p] = P.canon_pairs++;
    }
  }
  P.d_prow.alloc(npair);
  PNO_HIP(hipMemcpy(P.d_prow, P.prow.data(), npair * sizeof(int), hipMemcpyHostToDevice));
  {
    std::vector<int> slot(std::max(P.canon_pairs, 1), 0);
    for (int p = 0; p < npair; ++p)
      if (P.prow[p] >= 0) slot[P.prow[p]] = pi[p] * o + pj[p];
    P.d_slot.alloc((int64_t)slot.size());
    PNO_HIP(hipMemcpy(P.d_slot, slot.data(), slot.size() * sizeof(int), hipMemcpyHostToDevice));
  }
  if (P.nat_pairs == 0) return;
  P.Bbar.alloc(bw);
  {
    bool large = false;  // Y1 (offsets of Bbar) for the pairs the fused small-pair kernel does not take
    for (int p = 0; p < npair; ++p) large = large || (boff[p] >= 0 && P.npno[p] > kNatSmall);
    if (large) P.Y1.alloc(bw);
  }
  // Bbar_p[a][Q][k] = sum_xy U_p[x][a] B~^Q[o+x][o+y] U_p[y][k]: T1 = B~^Q U for a group of
  // consecutive native pairs at once (their U columns side by side, at most 512 of them, so
  // that B~_vv is read once per group and the product is wide), then U_p^T T1 per pair
  // (the group's T1 kept within 4 GiB, but at least one pair wide)
  const int64_t kGroupN = std::max<int64_t>(nmax, std::min<int64_t>(512, (4ll << 30) / (8 * (int64_t)naux * v)));
  DBuf<double> T1, Ug;
  T1.alloc((int64_t)naux * v * kGroupN);
  Ug.alloc((int64_t)v * kGroupN);
  for (int p0 = 0; p0 < npair;) {
    std::vector<int> grp;
    int64_t ncol = 0;
    int p = p0;
    for (; p < npair; ++p) {
      if (boff[p] < 0) continue;
      if (!grp.empty() && ncol + P.npno[p] > kGroupN) break;
      grp.push_back(p);
      ncol += P.npno[p];
    }
    p0 = p;
    if (grp.empty()) continue;
    int64_t col = 0;
    for (int q : grp) {
      const int64_t n = P.npno[q];
      PNO_HIP(hipMemcpy2DAsync((double*)Ug + col, ncol * sizeof(double), P.U + P.uoff[q], n * sizeof(double),
                               n * sizeof(double), v, hipMemcpyDeviceToDevice, s));
      col += n;
    }
    GemmDesc<double> d;
    d.M = v; d.N = ncol; d.K = v; d.batch = naux;
    d.A = c.Bt + (int64_t)o * nmo + o; d.lda = nmo; d.sA = n2;
    d.B = Ug; d.ldb = ncol; d.sB = 0;
    d.C = T1; d.ldc = ncol; d.sC = (int64_t)v * ncol;
    gemm(d, s);
    col = 0;
    for (int q : grp) {
      const int n = P.npno[q];
      GemmDesc<double> e;
      e.ta = true; e.M = n; e.N = n; e.K = v; e.batch = naux;
      e.A = P.U + P.uoff[q]; e.lda = n; e.sA = 0;
      e.B = T1 + col; e.ldb = ncol; e.sB = (int64_t)v * ncol;
      e.C = P.Bbar + boff[q]; e.ldc = (int64_t)naux * n; e.sC = n;
      gemm(e, s);
      col += n;
    }
  }
  // one vector's tables (bases shifted per vector): Y1 = Bbar_p Rbar_p, then the n x n result
  // over K = naux n in chunks of about 2048 (whole Q blocks), each chunk its own partial
  // block (so that every pair spreads over several workgroups), summed by a reduction
  std::vector<GroupDesc> ga, gb;
  std::vector<int> hn, hch;
  std::vector<int64_t> hpoff, hyoff, hsmall;
  int64_t pw = 0;
  for (int p = 0; p < npair; ++p) {
    if (boff[p] < 0) continue;
    const int64_t n = P.npno[p];
    if (n <= kNatSmall) {  // fused small-pair kernel: partial blocks per kNatQ values of Q
      const int64_t nch = (naux + kNatQ - 1) / kNatQ;
      hsmall.insert(hsmall.end(), {n, boff[p], P.off[o + p], pw});
      hn.push_back((int)n);
      hch.push_back((int)nch);
      hpoff.push_back(pw);
      hyoff.push_back(P.off[o + p]);
      pw += nch * n * n;
      continue;
    }
    GroupDesc d{};
    d.M = n * naux; d.N = n; d.K = n; d.offA = boff[p]; d.lda = n; d.offB = P.off[o + p]; d.ldb = n;
    d.offC = boff[p]; d.ldc = n;
    ga.push_back(d);
    const int64_t qc = std::max<int64_t>(1, 2048 / n);
    const int64_t nch = (naux + qc - 1) / qc;
    for (int64_t ch = 0; ch < nch; ++ch) {
      const int64_t q0 = ch * qc, nq = std::min<int64_t>(qc, naux - q0);
      GroupDesc e{};
      e.M = n; e.N = n; e.K = nq * n;
      e.offA = boff[p] + q0 * n; e.lda = n * naux; e.offB = boff[p] + q0 * n; e.ldb = n * naux;
      e.offC = pw + ch * n * n; e.ldc = n;
      gb.push_back(e);
    }
    hn.push_back((int)n);
    hch.push_back((int)nch);
    hpoff.push_back(pw);
    hyoff.push_back(P.off[o + p]);
    pw += nch * n * n;
  }
  gemm_grouped_prepare(ga, false, false, P.t_na);
  gemm_grouped_prepare(gb, false, true, P.t_nb);
  P.Ypart.alloc(pw);
  const int nn = (int)hn.size();
  P.d_nn.alloc(nn); P.d_nch.alloc(nn); P.d_poff.alloc(nn); P.d_yoff.alloc(nn);
  PNO_HIP(hipMemcpy(P.d_nn, hn.data(), nn * sizeof(int), hipMemcpyHostToDevice));
  PNO_HIP(hipMemcpy(P.d_nch, hch.data(), nn * sizeof(int), hipMemcpyHostToDevice));
  PNO_HIP(hipMemcpy(P.d_poff, hpoff.data(), nn * sizeof(int64_t), hipMemcpyHostToDevice));
  PNO_HIP(hipMemcpy(P.d_yoff, hyoff.data(), nn * sizeof(int64_t), hipMemcpyHostToDevice));
  P.nsmall = (int)(hsmall.size() / 4);
  if (P.nsmall > 0) {
    P.d_small.alloc((int64_t)hsmall.size());
    PNO_HIP(hipMemcpy(P.d_small, hsmall.data(), hsmall.size() * sizeof(int64_t), hipMemcpyHostToDevice));
  }
  PNO_HIP(hipStreamSynchronize(s));
}
}  // namespace

// D[i][j] += B_ij Bt_ij^T + B_ij^T Bt_ij with Bt = 2 B - B^T per pair block, for all o^2
// pairs of the doubles amplitudes B (device [o][o][v][v]); work: o^2 v^2 doubles
void add_pair_densities(Context& c, const double* Bk, double* work, double* D) {
  hipStream_t s = c.stream;
  const int o = c.o, v = c.v;
  const int64_t vv = (int64_t)v * v, oovv = c.oovv();
  perm(s, Bk, o, o, v, v, 0, 1, 3, 2, work, -1.0, 0.0);
  axpby(s, oovv, 2.0, Bk, 1.0, work);
  gm(s, false, true, v, v, v, 1.0, Bk, v, vv, work, v, vv, 1.0, D, v, vv, (int64_t)o * o);
  gm(s, true, false, v, v, v, 1.0, Bk, v, vv, work, v, vv, 1.0, D, v, vv, (int64_t)o * o);
}

// PNOs and OSVs of pair densities (Methods: per-pair eigenvectors of the density kept when
// |occupation| >= tcut_pno; OSVs from the diagonal pairs with tcut_osv), rotated to the
// semicanonical basis of the symmetric virtual matrix Fs (device v x v); focc: occupied
// energies of the preconditioner.  D holds sums over states for all o^2 pairs, D[i][j] of
// pair (i, j) scaled by inv_n (2 inv_n off the diagonal).  Fills P except its state list,
// cuts, native ladder and `built`; returns the pair tables (pairs i <= j, row-major).
void pnos_from_density(Context& c, PNOData& P, const double* D, double inv_n, double tcut_pno, double tcut_osv,
                       const double* Fs, const std::vector<double>& focc, std::vector<int>& pi,
                       std::vector<int>& pj) {
  hipStream_t s = c.stream;
  const int o = c.o, v = c.v;
  const int64_t vv = (int64_t)v * v;
  const int npair = o * (o + 1) / 2;
  // 3. pair tables and per-pair eigenproblems
  pi.assign(npair, 0);
  pj.assign(npair, 0);
  {
    int p = 0;
    for (int i = 0; i < o; ++i)
      for (int j = i; j < o; ++j) { pi[p] = i; pj[p] = j; ++p; }
  }
  DBuf<int> dpi, dpj, dn;
  dpi.alloc(npair); dpj.alloc(npair); dn.alloc(std::max(npair, o));
  PNO_HIP(hipMemcpyAsync(dpi, pi.data(), npair * sizeof(int), hipMemcpyHostToDevice, s));
  PNO_HIP(hipMemcpyAsync(dpj, pj.data(), npair * sizeof(int), hipMemcpyHostToDevice, s));
  DBuf<double> Dp, Vt, ev;
  Dp.alloc((int64_t)npair * vv);
  Vt.alloc((int64_t)npair * vv);
  ev.alloc((int64_t)npair * v);
  hipLaunchKernelGGL(gather_pairs_kernel, dim3(gsz((int64_t)npair * vv)), dim3(256), 0, s, o, v, npair,
                     (const int*)dpi, (const int*)dpj, inv_n, D, (double*)Dp);
  PNO_HIP(hipGetLastError());
  {
    std::vector<int> nv(npair, v);
    batched_syev(s, c.eig_backend, npair, nv, v, Dp, Vt, ev, dn, std::min(tcut_pno, tcut_osv));
  }
  std::vector<double> evh((size_t)npair * v);
  PNO_HIP(hipMemcpyAsync(evh.data(), ev, evh.size() * sizeof(double), hipMemcpyDeviceToHost, s));
  PNO_HIP(hipStreamSynchronize(s));
  PNO_CHECK(std::all_of(evh.begin(), evh.end(), [](double x) { return std::isfinite(x); }), PNOEOM_ENOTCONV,
            "build_sapno: non-finite pair-density occupation");
  Dp.release();

  // 4. kept vectors: pairs with |n| >= tcut_pno, OSVs (diagonal pairs) with |n| >= tcut_osv.
  //    Blocks: 0..npair-1 pairs, npair..npair+o-1 OSVs.
  const int nblk = npair + o;
  std::vector<int> bn(nblk), bmat(nblk);
  std::vector<int> smat, srow, scol, sncol;
  std::vector<int64_t> soff;
  std::vector<int64_t> uoff(nblk + 1, 0);
  for (int b = 0; b < nblk; ++b) {
    const int mtx = b < npair ? b : [&] {
      const int i = b - npair;
      return i * o - i * (i - 1) / 2;  // diagonal pair (i, i)
    }();
    const double cut = b < npair ? tcut_pno : tcut_osv;
    std::vector<int> rows;
    for (int k = 0; k < v; ++k)
      if (std::fabs(evh[(size_t)mtx * v + k]) >= cut) rows.push_back(k);
    bn[b] = (int)rows.size();
    bmat[b] = mtx;
    uoff[b + 1] = uoff[b] + (int64_t)v * bn[b];
    for (int cidx = 0; cidx < bn[b]; ++cidx) {
      smat.push_back(mtx);
      srow.push_back(rows[cidx]);
      soff.push_back(uoff[b]);
      scol.push_back(cidx);
      sncol.push_back(bn[b]);
    }
  }
  const int64_t utot = uoff[nblk];
  int nmax = 1;
  for (int b = 0; b < nblk; ++b) nmax = std::max(nmax, bn[b]);
  DBuf<double> U0;
  U0.alloc(std::max<int64_t>(utot, 1));
  if (!smat.empty()) {
    const int nsel = (int)smat.size();
    DBuf<int> dm, dr, dc, dnc;
    DBuf<int64_t> dof;
    dm.alloc(nsel); dr.alloc(nsel); dc.alloc(nsel); dnc.alloc(nsel); dof.alloc(nsel);
    PNO_HIP(hipMemcpy(dm, smat.data(), nsel * sizeof(int), hipMemcpyHostToDevice));
    PNO_HIP(hipMemcpy(dr, srow.data(), nsel * sizeof(int), hipMemcpyHostToDevice));
    PNO_HIP(hipMemcpy(dc, scol.data(), nsel * sizeof(int), hipMemcpyHostToDevice));
    PNO_HIP(hipMemcpy(dnc, sncol.data(), nsel * sizeof(int), hipMemcpyHostToDevice));
    PNO_HIP(hipMemcpy(dof, soff.data(), nsel * sizeof(int64_t), hipMemcpyHostToDevice));
    hipLaunchKernelGGL(gather_kept_kernel, dim3(gsz((int64_t)nsel * v)), dim3(256), 0, s, v, v, nsel,
                       (const int*)dm, (const int*)dr, (const int64_t*)dof, (const int*)dc, (const int*)dnc,
                       (const double*)Vt, (double*)U0);
    PNO_HIP(hipGetLastError());
    PNO_HIP(hipStreamSynchronize(s));
  }
  Vt.release();
  ev.release();

  // 5. semicanonical rotation: eigenvectors of U0^T Fs U0
  DBuf<double> Tb, Fb, Wt, fev;
  Tb.alloc(std::max<int64_t>(utot, 1));
  Fb.alloc((int64_t)nblk * nmax * nmax);
  Wt.alloc((int64_t)nblk * nmax * nmax);
  fev.alloc((int64_t)nblk * nmax);
  fill(s, (int64_t)nblk * nmax * nmax, 0.0, Fb);
  {
    std::vector<GroupDesc> g1, g2, g3;
    for (int b = 0; b < nblk; ++b) {
      const int n = bn[b];
      if (n == 0) continue;
      GroupDesc d{};
      // Tb_b = Fs U0_b  (v x n)
      d.M = v; d.N = n; d.K = v; d.offA = 0; d.lda = v; d.offB = uoff[b]; d.ldb = n; d.offC = uoff[b]; d.ldc = n;
      g1.push_back(d);
      // Fb_b = U0_b^T Tb_b  (n x n, padded ld nmax)
      d.M = n; d.N = n; d.K = v; d.offA = uoff[b]; d.lda = n; d.offB = uoff[b]; d.ldb = n;
      d.offC = (int64_t)b * nmax * nmax; d.ldc = nmax;
      g2.push_back(d);
      // U_b = U0_b Wt_b^T  (v x n)
      d.M = v; d.N = n; d.K = n; d.offA = uoff[b]; d.lda = n; d.offB = (int64_t)b * nmax * nmax; d.ldb = nmax;
      d.offC = uoff[b]; d.ldc = n;
      g3.push_back(d);
    }
    GroupTable t1, t2, t3;
    gemm_grouped_prepare(g1, false, false, t1);
    gemm_grouped_prepare(g2, true, false, t2);
    gemm_grouped_prepare(g3, false, true, t3);
    gemm_grouped(t1, 1.0, Fs, U0, 0.0, Tb, s);
    gemm_grouped(t2, 1.0, U0, Tb, 0.0, Fb, s);
    DBuf<int> dnb;
    dnb.alloc(nblk);
    batched_syev(s, c.eig_backend, nblk, bn, nmax, Fb, Wt, fev, dnb, 0.0);
    P.U.alloc(std::max<int64_t>(utot, 1));
    gemm_grouped(t3, 1.0, U0, Wt, 0.0, P.U, s);
    PNO_HIP(hipStreamSynchronize(s));
  }
  std::vector<double> fevh((size_t)nblk * nmax);
  PNO_HIP(hipMemcpy(fevh.data(), fev, fevh.size() * sizeof(double), hipMemcpyDeviceToHost));
  for (int b = 0; b < nblk; ++b)  // (entries past bn[b] of a block are not written)
    for (int k = 0; k < bn[b]; ++k)
      PNO_CHECK(std::isfinite(fevh[(size_t)b * nmax + k]), PNOEOM_ENOTCONV,
                "build_sapno: non-finite semicanonical orbital energy");

  // 6. layout of compressed vectors: singles of i = 0..o-1, then pairs p
  P.npno.assign(bn.begin(), bn.begin() + npair);
  P.nosv.assign(bn.begin() + npair, bn.end());
  P.off.assign(o + npair + 1, 0);
  for (int i = 0; i < o; ++i) P.off[i + 1] = P.off[i] + P.nosv[i];
  for (int p = 0; p < npair; ++p) P.off[o + p + 1] = P.off[o + p] + (int64_t)P.npno[p] * P.npno[p];
  // an odd total gets one trailing zero element: rows of even length start 16-byte aligned,
  // which the Davidson's streaming inner products and updates need
  P.len = P.off[o + npair] + (P.off[o + npair] & 1);
  P.uoff = uoff;
  P.xf_flops = 0;
  for (int p = 0; p < npair; ++p)
    P.xf_flops += 2.0 * P.npno[p] * (double)v * v + 2.0 * (double)P.npno[p] * P.npno[p] * v;
  for (int i = 0; i < o; ++i) P.xf_flops += 2.0 * P.nosv[i] * (double)v;
  P.nmax = nmax;
  PNO_CHECK(P.len > 0, PNOEOM_EINVAL, "PNO build: every PNO and OSV was truncated");
  // preconditioner base: F_ii (+ F_jj) - fbar_a (- fbar_b); weights
  std::vector<double> base(P.len, 1.0);  // (the padding element: 1, so that it stays 0)
  for (int i = 0; i < o; ++i) {
    const int b = npair + i;
    for (int a = 0; a < P.nosv[i]; ++a)
      base[P.off[i] + a] = focc[i] - fevh[(size_t)b * nmax + a];
  }
  for (int p = 0; p < npair; ++p) {
    const int n = P.npno[p];
    const double e = focc[pi[p]] + focc[pj[p]];
    for (int a = 0; a < n; ++a)
      for (int b2 = 0; b2 < n; ++b2)
        base[P.off[o + p] + (int64_t)a * n + b2] = e - fevh[(size_t)p * nmax + a] - fevh[(size_t)p * nmax + b2];
  }
  P.denom_base.alloc(P.len);
  PNO_HIP(hipMemcpy(P.denom_base, base.data(), P.len * sizeof(double), hipMemcpyHostToDevice));
  // diagonal-pair block table for the singlet symmetrisation
  {
    std::vector<int64_t> doff;
    std::vector<int> dsz;
    for (int p = 0; p < npair; ++p)
      if (pi[p] == pj[p]) { doff.push_back(P.off[o + p]); dsz.push_back(P.npno[p]); }
    P.d_off.alloc(doff.size());
    P.d_n.alloc(dsz.size());
    PNO_HIP(hipMemcpy(P.d_off, doff.data(), doff.size() * sizeof(int64_t), hipMemcpyHostToDevice));
    PNO_HIP(hipMemcpy(P.d_n, dsz.data(), dsz.size() * sizeof(int), hipMemcpyHostToDevice));
  }
  // grouped-GEMM tables for compress / expand (one vector; bases shifted per vector)
  {
    std::vector<GroupDesc> cs1, cs2d, cs2o, cs3, ex1, ex3;
    int64_t toff = 0;
    P.toff.assign(npair + 1, 0);
    for (int p = 0; p < npair; ++p) {
      P.toff[p + 1] = P.toff[p] + (int64_t)v * P.npno[p];
    }
    (void)toff;
    for (int i = 0; i < o; ++i) {
      const int n = P.nosv[i];
      if (n == 0) continue;
      const int b = npair + i;
      GroupDesc d{};
      // x_i (1 x n) = r1_i (1 x v) U^i (v x n)
      d.M = 1; d.N = n; d.K = v; d.offA = (int64_t)i * v; d.lda = v; d.offB = uoff[b]; d.ldb = n;
      d.offC = P.off[i]; d.ldc = n;
      cs1.push_back(d);
      // r1_i (1 x v) = x_i (1 x n) U^i^T
      d.M = 1; d.N = v; d.K = n; d.offA = P.off[i]; d.lda = n; d.offB = uoff[b]; d.ldb = n; d.offC = (int64_t)i * v;
      d.ldc = v;
      ex1.push_back(d);
    }
    for (int p = 0; p < npair; ++p) {
      const int n = P.npno[p];
      if (n == 0) continue;
      const int64_t rof = ((int64_t)pi[p] * o + pj[p]) * vv;
      GroupDesc d{};
      // T_p = R^{ij} U_p   (v x n)
      d.M = v; d.N = n; d.K = v; d.offA = rof; d.lda = v; d.offB = uoff[p]; d.ldb = n; d.offC = P.toff[p]; d.ldc = n;
      cs3.push_back(d);
      // x_p = w U_p^T T_p  (n x n)
      d.M = n; d.N = n; d.K = v; d.offA = uoff[p]; d.lda = n; d.offB = P.toff[p]; d.ldb = n; d.offC = P.off[o + p];
      d.ldc = n;
      (pi[p] == pj[p] ? cs2d : cs2o).push_back(d);
      // T_p = U_p X_p  (v x n)
      d.M = v; d.N = n; d.K = n; d.offA = uoff[p]; d.lda = n; d.offB = P.off[o + p]; d.ldb = n; d.offC = P.toff[p];
      d.ldc = n;
      ex3.push_back(d);
      // R^{ij} = T_p U_p^T / w (v x v, and its transpose for ji): expand_pairs_kernel
    }
    gemm_grouped_prepare(cs1, false, false, P.t_c1);
    gemm_grouped_prepare(cs3, false, false, P.t_c3);
    gemm_grouped_prepare(cs2d, true, false, P.t_c2d);
    gemm_grouped_prepare(cs2o, true, false, P.t_c2o);
    gemm_grouped_prepare(ex1, false, true, P.t_e1);
    gemm_grouped_prepare(ex3, false, false, P.t_e3);
    P.Tw.alloc(std::max<int64_t>(P.toff[npair], 1));
    std::vector<int64_t> xp(5 * (size_t)npair);
    for (int p = 0; p < npair; ++p) {
      xp[5 * p] = pi[p]; xp[5 * p + 1] = pj[p]; xp[5 * p + 2] = P.npno[p];
      xp[5 * p + 3] = P.toff[p]; xp[5 * p + 4] = uoff[p];
    }
    P.d_xpair.alloc(std::max<int64_t>(5 * npair, 1));
    PNO_HIP(hipMemcpy(P.d_xpair, xp.data(), xp.size() * sizeof(int64_t), hipMemcpyHostToDevice));
  }
}

void build_sapno(Context& c, int nstates, double tcut_pno, double tcut_osv) {
  PNO_CHECK(c.have_df, PNOEOM_ESTATE, "build_sapno before build_df");
  PNO_CHECK(nstates >= 1 && nstates <= c.ov(), PNOEOM_EINVAL, "build_sapno: bad nstates");
  hipStream_t s = c.stream;
  PNOData& P = c.pno;
  c.drop_graphs();
  P.reset();
  const int o = c.o, v = c.v, naux = c.naux, nmo = c.nmo;
  const int64_t n2 = (int64_t)nmo * nmo, ov = c.ov(), oovv = c.oovv(), vv = (int64_t)v * v;
  const int npair = o * (o + 1) / 2;
  // states whose densities are averaged: the lowest nstates, or the list set by
  // pnoeom_set_pno_states (one state: the state-specific PNOs of that state)
  std::vector<int> avg = P.states;
  if (avg.empty())
    for (int k = 0; k < nstates; ++k) avg.push_back(k);
  const int ncis = *std::max_element(avg.begin(), avg.end()) + 1;
  PNO_CHECK(ncis <= c.ov(), PNOEOM_EINVAL, "build_sapno: state index beyond the CIS space");
  P.nstates = (int)avg.size();
  P.tcut_pno = tcut_pno;
  P.tcut_osv = tcut_osv;

  // 1. CIS roots
  std::vector<double> w(ncis);
  DBuf<double> bvec;
  bvec.alloc((int64_t)ncis * ov);
  cis_roots(c, ncis, w.data(), bvec);

  // 2. averaged pair densities D[i][j] (all pairs, unscaled sum over states)
  DBuf<double> D, Bk, Bt2, Kt, Bp, XT, BvoT0;
  D.alloc(oovv);
  Bk.alloc(oovv);
  Bt2.alloc(oovv);
  Kt.alloc(oovv);
  Bp.alloc((int64_t)naux * v * o);
  XT.alloc(ov * naux);
  BvoT0.alloc(ov * naux);
  fill(s, oovv, 0.0, D);
  {
    Perm4 p;  // BvoT0[(j,b)][Q] = B[Q][o+b][j]
    p.d[0] = o; p.d[1] = v; p.d[2] = naux; p.d[3] = 1;
    p.is[0] = 1; p.is[1] = nmo; p.is[2] = n2; p.is[3] = 0;
    p.os[0] = (int64_t)v * naux; p.os[1] = naux; p.os[2] = 1; p.os[3] = 0;
    permute4(s, p, 1.0, c.B + (int64_t)o * nmo, 0.0, BvoT0);
  }
  for (int k : avg) {
    const double* b = bvec + (int64_t)k * ov;
    // B'_vo[Q][a][i] = -sum_l b_l^a B[Q][l][i] + sum_c B[Q][o+a][o+c] b_i^c
    gm(s, true, false, v, o, o, -1.0, b, v, 0, c.B, nmo, n2, 0.0, Bp, o, (int64_t)v * o, naux);
    gm(s, false, true, v, o, v, 1.0, c.B + (int64_t)o * nmo + o, nmo, n2, b, v, 0, 1.0, Bp, o, (int64_t)v * o, naux);
    perm(s, Bp, naux, v, o, 1, 2, 1, 0, 3, XT);  // XT[(i,a)][Q]
    // K[(i,a),(j,b)] = sum_Q B'_ai B_bj + B_ai B'_bj  ->  [i][j][a][b]
    gm(s, false, true, ov, ov, naux, 1.0, XT, naux, 0, BvoT0, naux, 0, 0.0, Bt2, ov, 0, 1);
    gm(s, false, true, ov, ov, naux, 1.0, BvoT0, naux, 0, XT, naux, 0, 1.0, Bt2, ov, 0, 1);
    perm(s, Bt2, o, v, o, v, 0, 2, 1, 3, Kt);
    hipLaunchKernelGGL(cisd_div_kernel, dim3(gsz(oovv)), dim3(256), 0, s, o, v, (const double*)c.eps, w[k],
                       (const double*)Kt, (double*)Bk);
    PNO_HIP(hipGetLastError());
    add_pair_densities(c, Bk, Bt2, D);
  }
  Bk.release(); Bt2.release(); Kt.release(); Bp.release(); XT.release(); BvoT0.release();

  // 3.-6. PNOs / OSVs, semicanonical in the symmetric part of the virtual block of the
  //       one-particle part of H-bar, occupied energies from its occupied block
  std::vector<int> pi, pj;
  {
    DBuf<double> Fs;
    Fs.alloc(vv);
    perm(s, c.Fvv, v, v, 1, 1, 1, 0, 2, 3, Fs, 0.5, 0.0);
    axpby(s, vv, 0.5, c.Fvv, 1.0, Fs);
    std::vector<double> Fooh((size_t)o * o), focc(o);
    PNO_HIP(hipMemcpy(Fooh.data(), c.Foo, Fooh.size() * sizeof(double), hipMemcpyDeviceToHost));
    for (int i = 0; i < o; ++i) focc[i] = Fooh[(size_t)i * o + i];
    pnos_from_density(c, P, D, 1.0 / (double)avg.size(), tcut_pno, tcut_osv, Fs, focc, pi, pj);
  }
  D.release();
  build_native_ladder(c, pi, pj);
  P.built = true;
}

// Ground-state PNOs / OSVs (Methods: pair densities D_(0) of the guess amplitudes, the same
// eigenvector truncation), semicanonical in the Fock matrix diag(eps) with occupied
// energies eps_i: the basis of the ground-state PNO-CCSD simulation.  Kept in c.gs, which
// build_df leaves alone.
void build_gs_pnos(Context& c, const double* t2, double tcut_pno, double tcut_osv) {
  hipStream_t s = c.stream;
  const int o = c.o, v = c.v, nmo = c.nmo;
  const int64_t vv = (int64_t)v * v, oovv = c.oovv();
  PNOData& P = c.gs;
  P.reset();
  {
    DBuf<double> D, work;
    D.alloc(oovv);
    work.alloc(oovv);
    fill(s, oovv, 0.0, D);
    add_pair_densities(c, t2, work, D);
    work.release();
    std::vector<double> eh(nmo), Fh((size_t)vv, 0.0), focc(o);
    PNO_HIP(hipMemcpyAsync(eh.data(), c.eps, nmo * sizeof(double), hipMemcpyDeviceToHost, s));
    PNO_HIP(hipStreamSynchronize(s));
    for (int a = 0; a < v; ++a) Fh[(size_t)a * v + a] = eh[o + a];
    for (int i = 0; i < o; ++i) focc[i] = eh[i];
    DBuf<double> Fs;
    Fs.alloc(vv);
    PNO_HIP(hipMemcpy(Fs, Fh.data(), vv * sizeof(double), hipMemcpyHostToDevice));
    std::vector<int> pi, pj;
    pnos_from_density(c, P, D, 1.0, tcut_pno, tcut_osv, Fs, focc, pi, pj);
  }
  P.nstates = 0;
  P.tcut_pno = tcut_pno;
  P.tcut_osv = tcut_osv;
  P.built = true;
}

// ----------------------------------------------------------------------------- transforms
void pno_compress(Context& c, int nvec, const double* r1, const double* r2, double* x) {
  pno_compress(c, c.pno, nvec, r1, r2, x);
}

void pno_compress(Context& c, PNOData& P, int nvec, const double* r1, const double* r2, double* x) {
  PNO_CHECK(P.built, PNOEOM_ESTATE, "PNO compress before the PNOs are built");
  hipStream_t s = c.stream;
  const double sq2 = std::sqrt(2.0);
  hipEvent_t ev = c.region_begin(1, s);
  for (int q = 0; q < nvec; ++q) {
    const double* a1 = r1 + (int64_t)q * c.ov();
    const double* a2 = r2 + (int64_t)q * c.oovv();
    double* y = x + (int64_t)q * P.len;
    gemm_grouped(P.t_c1, 1.0, a1, P.U, 0.0, y, s);
    gemm_grouped(P.t_c3, 1.0, a2, P.U, 0.0, P.Tw, s);
    gemm_grouped(P.t_c2d, 1.0, P.U, P.Tw, 0.0, y, s);
    gemm_grouped(P.t_c2o, sq2, P.U, P.Tw, 0.0, y, s);
    const int64_t end = P.off.back();
    if (P.len > end) fill(s, P.len - end, 0.0, y + end);  // padding
  }
  c.region_end(ev, 1, s, 4 * nvec, nvec * P.xf_flops,
               8.0 * nvec * ((double)c.ov() + (double)c.oovv() + (double)P.len + (double)P.U.n));
}

void pno_expand(Context& c, int nvec, const double* x, double* r1, double* r2) {
  pno_expand(c, c.pno, nvec, x, r1, r2);
}

void pno_expand(Context& c, PNOData& P, int nvec, const double* x, double* r1, double* r2) {
  PNO_CHECK(P.built, PNOEOM_ESTATE, "PNO expand before the PNOs are built");
  hipStream_t s = c.stream;
  const double isq2 = 1.0 / std::sqrt(2.0);
  hipEvent_t ev = c.region_begin(1, s);
  for (int q = 0; q < nvec; ++q) {
    double* b1 = r1 + (int64_t)q * c.ov();
    double* b2 = r2 + (int64_t)q * c.oovv();
    const double* y = x + (int64_t)q * P.len;
    fill(s, c.ov(), 0.0, b1);
    gemm_grouped(P.t_e1, 1.0, y, P.U, 0.0, b1, s);
    gemm_grouped(P.t_e3, 1.0, P.U, y, 0.0, P.Tw, s);
    const int npair = c.o * (c.o + 1) / 2;
    const int nt = (c.v + kXT - 1) / kXT;
    PNO_CHECK(npair <= 65535, PNOEOM_EINVAL, "pno_expand: too many pairs for one launch");
    hipLaunchKernelGGL(expand_pairs_kernel, dim3((unsigned)(nt * nt), (unsigned)npair), dim3(256), 0, s, c.o, c.v,
                       (const int64_t*)P.d_xpair, (const double*)P.Tw, (const double*)P.U, isq2, b2);
    PNO_HIP(hipGetLastError());
  }
  c.region_end(ev, 1, s, 4 * nvec, nvec * P.xf_flops,
               8.0 * nvec * ((double)c.ov() + (double)c.oovv() + (double)P.len + (double)P.U.n));
}

void project_pno(Context& c, double* x) { project_pno(c, c.pno, x); }

void project_pno(Context& c, PNOData& P, double* x) {
  const int nd = (int)P.d_n.n;
  if (nd == 0) return;
  hipLaunchKernelGGL(sym_diag_blocks_kernel, dim3(nd, 32), dim3(256), 0, c.stream, nd, (const int64_t*)P.d_off,
                     (const int*)P.d_n, x);
  PNO_HIP(hipGetLastError());
}

void precond_pno(Context& c, double* x, double theta) { precond_pno(c, c.pno, x, theta); }

void precond_pno(Context& c, PNOData& P, double* x, double theta) {
  hipLaunchKernelGGL(precond_pno_kernel, dim3(gsz(P.len)), dim3(256), 0, c.stream, P.len, theta,
                     (const double*)P.denom_base, x);
  PNO_HIP(hipGetLastError());
  project_pno(c, P, x);
}

void sigma_pno(Context& c, int nvec, const double* x, double* y, int precision) {
  PNOData& P = c.pno;
  PNO_CHECK(P.built, PNOEOM_ESTATE, "PNO sigma before build_sapno");
  if (nvec <= 0) return;
  auto grow = [](DBuf<double>& b, int64_t n) {
    if ((int64_t)b.n < n) b.alloc(n);
  };
  // chunks whose canonical expansions, ladder operands and work arrays fit in HBM
  const int nb = sigma_chunk(c, nvec, precision, true);
  grow(P.r1, (int64_t)nb * c.ov());
  grow(P.r2, (int64_t)nb * c.oovv());
  grow(P.s1, (int64_t)nb * c.ov());
  grow(P.s2, (int64_t)nb * c.oovv());
  // canonical sigma with the ladder restricted to the pairs that keep it
  struct Restrict {
    Context& c;
    Restrict(Context& cc, const int* prow, const int* slot, int64_t nsub) : c(cc) {
      c.lad_prow = prow;
      c.lad_slot = slot;
      c.lad_nsub = nsub;
    }
    ~Restrict() {
      c.lad_prow = nullptr;
      c.lad_slot = nullptr;
      c.lad_nsub = -1;
    }
  };
  for (int q0 = 0; q0 < nvec; q0 += nb) {
    const int n = std::min(nb, nvec - q0);
    pno_expand(c, n, x + (int64_t)q0 * P.len, P.r1, P.r2);
    {
      Restrict r(c, P.nat_pairs > 0 ? (const int*)P.d_prow : nullptr, P.nat_pairs > 0 ? (const int*)P.d_slot : nullptr,
                 P.nat_pairs > 0 ? P.canon_pairs : -1);
      sigma_block(c, n, P.r1, P.r2, P.s1, P.s2, c.ov(), c.oovv(), precision);
    }
    pno_compress(c, n, P.s1, P.s2, y + (int64_t)q0 * P.len);
  }
  // the native pairs' ladder, added in the PNO space (FP64: the fused small-pair kernel for
  // n_p <= 16, grouped MFMA GEMMs for the others)
  if (P.nat_pairs > 0) {
    hipEvent_t ev = c.region_begin(4, c.stream);
    PNO_CHECK(P.nsmall <= 65535, PNOEOM_EINVAL, "native ladder: too many pairs for one launch");
    for (int q = 0; q < nvec; ++q) {
      if (P.nsmall > 0)
        hipLaunchKernelGGL(native_small_kernel, dim3((unsigned)((c.naux + kNatQ - 1) / kNatQ), (unsigned)P.nsmall),
                           dim3(256), 0, c.stream, c.naux, (const int64_t*)P.d_small, (const double*)P.Bbar,
                           (const double*)(x + (int64_t)q * P.len), (double*)P.Ypart);
      gemm_grouped(P.t_na, 1.0, P.Bbar, x + (int64_t)q * P.len, 0.0, P.Y1, c.stream);
      gemm_grouped(P.t_nb, 1.0, P.Y1, P.Bbar, 0.0, P.Ypart, c.stream);
      hipLaunchKernelGGL(sum_chunks_kernel, dim3((unsigned)P.nat_pairs), dim3(256), 0, c.stream,
                         (const int*)P.d_nn, (const int*)P.d_nch, (const int64_t*)P.d_poff,
                         (const int64_t*)P.d_yoff, (const double*)P.Ypart, y + (int64_t)q * P.len);
      PNO_HIP(hipGetLastError());
    }
    c.region_end(ev, 4, c.stream, 3 * nvec, nvec * P.nat_flops, 8.0 * nvec * 3.0 * (double)P.Bbar.n);
  }
  for (int q = 0; q < nvec; ++q) project_pno(c, y + (int64_t)q * P.len);
}

}  // namespace pnoeom
