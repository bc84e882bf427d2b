// Closed-shell EOM-CCSD sigma = <mu|[H-bar, R]|0> on the GPU.
//
// H-bar = exp(-T) H exp(T) (Methods).  T1 is folded into the DF factors by the
// similarity dressing B~ = (1 - t)^T B (1 + t^T), which leaves a doubles-only
// coupled-cluster polynomial in T2 with the dressed Hamiltonian.  Since R commutes
// with T, sigma is the derivative of the projected CC equations along R:
//   * R1 enters through the one-index transformation B' = -r^T B~ + B~ r^T of the
//     dressed factors (and of the dressed core operator);
//   * R2 enters linearly and through the two bilinear T2.T2 terms.
// Every term is a pair of a "T-side" intermediate (built once per T in build_df)
// applied to R, or an "R-side" intermediate applied to T; all of them are MFMA
// GEMMs on ov x ov, o^2 x v^2 or v^2 x v^2 matrices plus layout permutations.
// The particle-particle ladder sum_cd W_ab^cd R_ij^cd uses the dressed ladder
// intermediate W_ab^cd = (ac|bd)~, which contains the first three terms and the
// T1.T1 term of the paper's W_ab^cd; its T2 G_ij^cd part is applied as the
// bilinear hole-ladder term X_klij = sum_cd (kc|ld) R_ij^cd.
#include <mutex>

#include "context.h"

namespace pnoeom {
namespace {

void gm(hipStream_t s, bool ta, bool tb, int64_t M, int64_t N, int64_t K, double alpha, const double* A,
        int64_t lda, const double* B, int64_t ldb, double beta, double* C, int64_t ldc) {
  GemmDesc<double> d;
  d.ta = ta; d.tb = tb; d.M = M; d.N = N; d.K = K; d.alpha = alpha; d.beta = beta;
  d.A = A; d.lda = lda; d.B = B; d.ldb = ldb; d.C = C; d.ldc = ldc;
  gemm(d, s);
}

void gmb(hipStream_t s, bool ta, bool tb, int64_t M, int64_t N, int64_t K, double alpha, const double* A,
         int64_t lda, int64_t sA, const double* B, int64_t ldb, int64_t sB, double beta, double* C,
         int64_t ldc, int64_t sC, int64_t batch, bool reduce = false) {
  GemmDesc<double> d;
  d.ta = ta; d.tb = tb; d.M = M; d.N = N; d.K = K; d.alpha = alpha; d.beta = beta;
  d.A = A; d.lda = lda; d.sA = sA; d.B = B; d.ldb = ldb; d.sB = sB; d.C = C; d.ldc = ldc; d.sC = sC;
  d.batch = batch; d.reduce = reduce;
  gemm(d, s);
}

// contiguous out[d0][d1][d2][d3] = alpha * in[i0*is0 + ...] + beta * out
void ext(hipStream_t s, int64_t d0, int64_t d1, int64_t d2, int64_t d3, int64_t is0, int64_t is1, int64_t is2,
         int64_t is3, const double* in, double* out, double alpha = 1.0, double beta = 0.0) {
  Perm4 p;
  p.d[0] = d0; p.d[1] = d1; p.d[2] = d2; p.d[3] = d3;
  p.is[0] = is0; p.is[1] = is1; p.is[2] = is2; p.is[3] = is3;
  p.os[3] = 1; p.os[2] = d3; p.os[1] = d2 * d3; p.os[0] = d1 * d2 * d3;
  permute4(s, p, alpha, in, beta, out);
}

void perm(hipStream_t s, const double* in, int64_t a, int64_t b, int64_t c, int64_t d, int p0, int p1, int p2,
          int p3, double* out, double alpha = 1.0, double beta = 0.0) {
  const int64_t dims[4] = {a, b, c, d};
  const int pp[4] = {p0, p1, p2, p3};
  permute_c(s, dims, pp, alpha, in, beta, out);
}

// d[q] = sum_{k < o} X[q sq + k ld + k]: the occupied-block trace of each fitting function's matrix
__global__ void trace_rows_kernel(int naux, int64_t ld, int64_t sq, int o, const double* __restrict__ X,
                                  double* __restrict__ d) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= naux) return;
  const double* b = X + (int64_t)q * sq;
  double acc = 0.0;
  for (int k = 0; k < o; ++k) acc += b[(int64_t)k * ld + k];
  d[q] = acc;
}

__global__ void trace_occ_kernel(int naux, int nmo, int o, const double* __restrict__ B, double* __restrict__ d) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= naux) return;
  const double* b = B + (int64_t)q * nmo * nmo;
  double acc = 0.0;
  for (int k = 0; k < o; ++k) acc += b[(int64_t)k * nmo + k];
  d[q] = acc;
}

__global__ void add_diag_kernel(int n, const double* __restrict__ e, double* __restrict__ h) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p < n) h[(int64_t)p * n + p] += e[p];
}

__global__ void mp2_div_kernel(int o, int v, const double* __restrict__ eps, double* __restrict__ t) {
  const int64_t n = (int64_t)o * o * v * v;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
    int64_t r = e;
    const int b = (int)(r % v); r /= v;
    const int a = (int)(r % v); r /= v;
    const int j = (int)(r % o); r /= o;
    const int i = (int)r;
    t[e] /= (eps[i] + eps[j] - eps[o + a] - eps[o + b]);
  }
}

__global__ void symmetrize_kernel(int o, int v, double* __restrict__ r2) {
  const int64_t n = (int64_t)o * o * v * v;
  const int64_t V = v, O = o;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
    int64_t r = e;
    const int64_t b = r % V; r /= V;
    const int64_t a = r % V; r /= V;
    const int64_t j = r % O; r /= O;
    const int64_t i = r;
    const int64_t p = ((j * O + i) * V + b) * V + a;
    if (p > e) {
      const double m = 0.5 * (r2[e] + r2[p]);
      r2[e] = m;
      r2[p] = m;
    }
  }
}

constexpr int kAsmTile = 32;  // (a, b) tile edge of the R2 layout and sigma2 assembly kernels

__host__ __device__ __forceinline__ int64_t tri_idx(int64_t c, int64_t d, int64_t v) {  // c <= d
  return c * v - c * (c - 1) / 2 + (d - c);
}
__host__ __device__ __forceinline__ int64_t stri_idx(int64_t c, int64_t d, int64_t v) {  // c < d
  return c * (v - 1) - c * (c - 1) / 2 + (d - c - 1);
}
__device__ __forceinline__ int64_t pair_idx(int64_t i, int64_t j, int64_t o) {  // i <= j
  return i * o - i * (i - 1) / 2 + (j - i);
}

__global__ void zero_u16_kernel(int64_t n, uint16_t* __restrict__ x) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
    x[e] = 0;
}

// storage conversions of the packed ladder operands: FP64, FP32, or bfloat16 bits
// (round to nearest even through FP32)
__device__ __forceinline__ uint16_t bf16_bits(double x) {
  uint32_t u = __float_as_uint((float)x);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40u);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
template <typename T>
__device__ __forceinline__ T cvt_out(double x) {
  return (T)x;
}
template <>
__device__ __forceinline__ uint16_t cvt_out<uint16_t>(double x) {
  return bf16_bits(x);
}

// dst[q][c][r] = bf16(src[q][r][c]) for r < R, zero for R <= r < ld (rows of ld values), c < C:
// a transpose through 32 x 32 LDS tiles, reads along c and writes along r
__global__ __launch_bounds__(256) void bf16_transpose_kernel(int64_t R, int64_t C, const double* __restrict__ src,
                                                             int64_t sbatch, uint16_t* __restrict__ dst, int64_t ld,
                                                             int64_t dbatch) {
  __shared__ double t[32][33];
  const int64_t c0 = (int64_t)blockIdx.x * 32, r0 = (int64_t)blockIdx.y * 32;
  const double* sq = src + (int64_t)blockIdx.z * sbatch;
  uint16_t* dq = dst + (int64_t)blockIdx.z * dbatch;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8
  for (int yy = ty; yy < 32; yy += 8) {
    const int64_t r = r0 + yy, c = c0 + tx;
    t[yy][tx] = (r < R && c < C) ? sq[r * C + c] : 0.0;
  }
  __syncthreads();
  for (int yy = ty; yy < 32; yy += 8) {
    const int64_t c = c0 + yy, r = r0 + tx;
    if (c < C && r < ld) dq[c * ld + r] = bf16_bits(t[tx][yy]);
  }
}

// out[b][c] = bf16(F[b][c]) for c != b (zero on the diagonal and beyond n, rows of ld values),
// d[b] = F[b][b]: a square matrix split into its exact diagonal and a bfloat16 remainder
__global__ void offdiag_rows_bf16_kernel(int64_t n, const double* __restrict__ F, uint16_t* __restrict__ out,
                                         int64_t ld, double* __restrict__ d) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n * ld; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t b = e / ld, c = e % ld;
    out[e] = bf16_bits(c < n && c != b ? F[b * n + c] : 0.0);
    if (c == b) d[b] = F[b * n + b];
  }
}

// acc[e] += R[e] (d[b] - fd[j]) for e = (((q o + i) o + j) v + a) v + b: the diagonal parts of
// R Fvv^T and of -Foo^T R added to the FP32 sum of the Fock-type products (the products
// themselves in FP64, rounded once)
__global__ void zp_finish_kernel(int64_t n, int64_t o, int64_t v, float* __restrict__ acc,
                                 const double* __restrict__ R, const double* __restrict__ d,
                                 const double* __restrict__ fd) {
  const int64_t vv = v * v;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
    acc[e] = (float)((double)acc[e] + R[e] * (d[e % v] - fd[(e / vv) % o]));
}

// bfloat16 rows (ld columns, zero beyond o^2) of Wh[(ij)][(kl)] - delta_ik Foo[l][j] (l != j)
// - delta_jl Foo[k][i] (k != i): the off-diagonal part of the -Foo^T R Fock-type term and of its
// (ij, ab) <-> (ji, ba) partner, carried by the hole ladder (R_kj^ab = R_jk^ba); fd = diag(Foo)
__global__ void wh_foo_rows_bf16_kernel(int64_t o, const double* __restrict__ Wh, const double* __restrict__ Foo,
                                        uint16_t* __restrict__ out, int64_t ld, double* __restrict__ fd) {
  const int64_t oo = o * o;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < oo * ld; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = e / ld, cl = e % ld;
    double val = 0.0;
    if (cl < oo) {
      const int64_t i = r / o, j = r % o, k = cl / o, l = cl % o;
      val = Wh[r * oo + cl];
      if (i == k && l != j) val -= Foo[l * o + j];
      if (j == l && k != i) val -= Foo[k * o + i];
    }
    out[e] = bf16_bits(val);
    if (e < o) fd[e] = Foo[e * o + e];
  }
}

// row p of a pair-compacted array <- row (i o + j) of the full one, for the pairs p = (i <= j)
// in row-major order (i, then j >= i); one workgroup per destination row (nvec x o(o+1)/2
// rows: grid.y = vector, grid.x = pair), FP64 source rows of K values converted to bfloat16
// rows of ld (zero beyond K), or bfloat16 rows copied (src16)
__device__ __forceinline__ void pair_of(int64_t p, int64_t o, int64_t& i, int64_t& j) {
  i = 0;
  while (p >= o - i) {
    p -= o - i;
    ++i;
  }
  j = i + p;
}
__global__ void pair_rows_gather_kernel(int o, int64_t K, const double* __restrict__ src,
                                        const uint16_t* __restrict__ src16, int64_t ld, uint16_t* __restrict__ dst) {
  const int64_t O = o, np = O * (O + 1) / 2, p = blockIdx.x, q = blockIdx.y;
  int64_t i, j;
  pair_of(p, O, i, j);
  const int64_t srow = (q * O + i) * O + j, drow = q * np + p;
  for (int64_t c = threadIdx.x; c < ld; c += blockDim.x) {
    if (src16)
      dst[drow * ld + c] = src16[srow * ld + c];
    else
      dst[drow * ld + c] = c < K ? bf16_bits(src[srow * K + c]) : (uint16_t)0;
  }
}

// out[q][a][(p, c)] = bf16(U[q][p][a][c]) for pairs p < npair (U: [nb][npair][v][v]), rows of
// ld values, zero beyond npair v: the left operand of Ftv = -sum_(p,c) U[p][a][c] Gq[(p,c)][b]
__global__ void pair_rows_bf16_kernel(int64_t nb, int64_t npair, int64_t v, const double* __restrict__ U,
                                      uint16_t* __restrict__ out, int64_t ld) {
  const int64_t total = nb * v * ld;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t k = e % ld, r = e / ld;  // r = (q, a)
    const int64_t q = r / v, a = r % v;
    double x = 0.0;
    if (k < npair * v) {
      const int64_t p = k / v, c = k % v;
      x = U[((q * npair + p) * v + a) * v + c];
    }
    out[e] = bf16_bits(x);
  }
}

// bfloat16 operand rows: row m of out (row stride ldo) holds `passes` blocks of ldk values;
// with x = scale src[m sm + k sk] (0 for k >= K; scale a power of two), hi = bf16(x) and
// lo = bf16(x - hi), a left operand (right = 0) takes [hi | hi | lo] and a right operand
// [hi | lo | hi], so that the three passes of one product sum to hi hi + hi lo + lo hi; one
// pass takes hi alone
__global__ void bf16_split_kernel(int64_t M, int64_t K, const double* __restrict__ src, int64_t sm, int64_t sk,
                                  uint16_t* __restrict__ out, int64_t ldk, int64_t ldo, int passes, int right,
                                  double scale) {
  const int64_t total = M * ldk, row = ldo;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t m = e / ldk, k = e % ldk;
    const double x = k < K ? scale * src[m * sm + k * sk] : 0.0;
    const uint16_t hi = bf16_bits(x);
    uint16_t* o = out + m * row + k;
    o[0] = hi;
    if (passes == 3) {
      const uint16_t lo = bf16_bits(x - (double)__uint_as_float((uint32_t)hi << 16));
      o[ldk] = right ? lo : hi;
      o[2 * ldk] = right ? hi : lo;
    }
  }
}

unsigned grid1(int64_t n) {
  int64_t b = (n + 255) / 256;
  if (b > 65536) b = 65536;
  if (b < 1) b = 1;
  return (unsigned)b;
}

// host side of bf16_split_kernel (ldo: row stride of out, at least passes x ldk)
void bf16_rows(hipStream_t s, int64_t M, int64_t K, const double* src, int64_t sm, int64_t sk, uint16_t* out,
               int64_t ldk, int64_t ldo, int passes = 1, int right = 0, double scale = 1.0) {
  PNO_CHECK(ldo >= passes * ldk && K <= ldk, PNOEOM_EINVAL, "bf16_rows: row layout");
  hipLaunchKernelGGL(bf16_split_kernel, dim3(grid1(M * ldk)), dim3(256), 0, s, M, K, src, sm, sk, out, ldk, ldo,
                     passes, right, scale);
  PNO_HIP(hipGetLastError());
}

// W+[(a<=b),(c<=d)] = W_abcd + W_abdc (c<d), W_abcc (c=d);  W-[(a<b),(c<d)] = W_abcd - W_abdc,
// from a slab tmp[a-a0][c][b][d] = W_abcd of rows a in [a0, a0+na); row strides ldp, ldm
template <typename OutT>
__global__ void ladder_wpm_kernel(int v, int a0, int na, const double* __restrict__ tmp, OutT* __restrict__ Wp,
                                  int64_t ldp, OutT* __restrict__ Wm, int64_t ldm) {
  const int64_t V = v, vp = V * (V + 1) / 2, vm = V * (V - 1) / 2;
  const int64_t total = (int64_t)na * V * V * V;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    int64_t r = e;
    const int64_t d = r % V; r /= V;
    const int64_t c = r % V; r /= V;
    const int64_t b = r % V; r /= V;
    const int64_t al = r, a = a0 + al;
    if (b < a || d < c) continue;
    const double w1 = tmp[((al * V + c) * V + b) * V + d];
    const double w2 = tmp[((al * V + d) * V + b) * V + c];
    Wp[tri_idx(a, b, V) * ldp + tri_idx(c, d, V)] = cvt_out<OutT>(c < d ? w1 + w2 : w1);
    if (a < b && c < d) Wm[stri_idx(a, b, V) * ldm + stri_idx(c, d, V)] = cvt_out<OutT>(w1 - w2);
  }
}

// S[(q,p)][(c<=d)] = (R^cd + R^dc)/2 (c<d), R^cc ;  A[(q,p)][(c<d)] = (R^cd - R^dc)/2  for pairs p = (i<=j);
// row strides ldS, ldA.  With prow, pair p goes to slot prow[p] of nrow slots per vector (none if < 0)
template <typename OutT>
__global__ void ladder_pack_kernel(int o, int v, int nvec, const double* __restrict__ r2, int64_t stride,
                                   OutT* __restrict__ S, int64_t ldS, OutT* __restrict__ A, int64_t ldA,
                                   const int* __restrict__ prow, int64_t nrow) {
  const int64_t O = o, V = v, vp = V * (V + 1) / 2, vm = V * (V - 1) / 2;
  const int64_t total = (int64_t)nvec * O * O * V * V;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    int64_t r = e;
    const int64_t d = r % V; r /= V;
    const int64_t c = r % V; r /= V;
    const int64_t j = r % O; r /= O;
    const int64_t i = r % O; r /= O;
    const int64_t q = r;
    if (j < i || d < c) continue;
    const int64_t slot = prow ? (int64_t)prow[pair_idx(i, j, O)] : pair_idx(i, j, O);
    if (slot < 0) continue;
    const double* R = r2 + q * stride + (i * O + j) * V * V;
    const double x = R[c * V + d], y = R[d * V + c];
    const int64_t row = q * nrow + slot;
    S[row * ldS + tri_idx(c, d, V)] = cvt_out<OutT>(c < d ? 0.5 * (x + y) : x);
    if (c < d) A[row * ldA + stri_idx(c, d, V)] = cvt_out<OutT>(0.5 * (x - y));
  }
}

// the same packing driven by the list of slots (slot_ij: i o + j of the pair of each of the nrow
// slots): only the R blocks of the listed pairs are read
template <typename OutT>
__global__ void ladder_pack_slots_kernel(int o, int v, int nvec, const double* __restrict__ r2, int64_t stride,
                                         OutT* __restrict__ S, int64_t ldS, OutT* __restrict__ A, int64_t ldA,
                                         const int* __restrict__ slot_ij, int64_t nrow) {
  const int64_t O = o, V = v, VV = V * V;
  const int64_t total = (int64_t)nvec * nrow * VV;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    int64_t r = e;
    const int64_t d = r % V; r /= V;
    const int64_t c = r % V; r /= V;
    const int64_t slot = r % nrow;
    const int64_t q = r / nrow;
    if (d < c) continue;
    const int64_t ij = slot_ij[slot], i = ij / O, j = ij % O;
    const double* R = r2 + q * stride + (i * O + j) * VV;
    const double x = R[c * V + d], y = R[d * V + c];
    const int64_t row = q * nrow + slot;
    S[row * ldS + tri_idx(c, d, V)] = cvt_out<OutT>(c < d ? 0.5 * (x + y) : x);
    if (c < d) A[row * ldA + stri_idx(c, d, V)] = cvt_out<OutT>(0.5 * (x - y));
  }
}

// out[q][i][j][a][b] = sigma_ij^ab of the ladder from sigma+ (a<=b) and sigma- (a<b) of pair min(i,j), max(i,j)
// (rows as in ladder_pack_kernel; zero for a pair without a slot)
template <typename InT>
__global__ void ladder_unpack_kernel(int o, int v, int nvec, const InT* __restrict__ SP, const InT* __restrict__ SM,
                                     double* __restrict__ out, int64_t stride, const int* __restrict__ prow,
                                     int64_t nrow) {
  const int64_t O = o, V = v, vp = V * (V + 1) / 2, vm = V * (V - 1) / 2;
  const int64_t total = (int64_t)nvec * O * O * V * V;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    int64_t r = e;
    int64_t b = r % V; r /= V;
    int64_t a = r % V; r /= V;
    int64_t j = r % O; r /= O;
    int64_t i = r % O; r /= O;
    const int64_t q = r;
    if (i > j) {  // sigma_ij^ab = sigma_ji^ba
      int64_t t = i; i = j; j = t;
      t = a; a = b; b = t;
    }
    const int64_t slot = prow ? (int64_t)prow[pair_idx(i, j, O)] : pair_idx(i, j, O);
    if (slot < 0) {
      out[q * stride + (e % (O * O * V * V))] = 0.0;
      continue;
    }
    const int64_t row = q * nrow + slot;
    double val;
    if (a == b) val = (double)SP[row * vp + tri_idx(a, a, V)];
    else if (a < b) val = (double)SP[row * vp + tri_idx(a, b, V)] + (double)SM[row * vm + stri_idx(a, b, V)];
    else val = (double)SP[row * vp + tri_idx(b, a, V)] - (double)SM[row * vm + stri_idx(b, a, V)];
    out[q * stride + (e % (O * O * V * V))] = val;
  }
}

// out[q][p][a][b] += sigma_ij^ab of the ladder for the nrow pairs p = (i <= j) listed in slot_ij
// (i o + j per slot; rows of sigma+ / sigma- as in ladder_pack_kernel; out holds the pairs
// i <= j in row-major order, the fused mode's direct block), written along b
__global__ void ladder_unpack_add_kernel(int o, int v, int nvec, int64_t nrow, const float* __restrict__ SP,
                                         const float* __restrict__ SM, const int* __restrict__ slot_ij,
                                         float* __restrict__ out) {
  const int64_t O = o, V = v, VV = V * V, vp = V * (V + 1) / 2, vm = V * (V - 1) / 2;
  const int64_t total = (int64_t)nvec * nrow * VV;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    int64_t r = e;
    const int64_t b = r % V; r /= V;
    const int64_t a = r % V; r /= V;
    const int64_t slot = r % nrow;
    const int64_t q = r / nrow;
    const int64_t ij = slot_ij[slot], i = ij / O, j = ij % O;
    const int64_t row = q * nrow + slot;
    float val;
    if (a == b) val = SP[row * vp + tri_idx(a, a, V)];
    else if (a < b) val = SP[row * vp + tri_idx(a, b, V)] + SM[row * vm + stri_idx(a, b, V)];
    else val = SP[row * vp + tri_idx(b, a, V)] - SM[row * vm + stri_idx(b, a, V)];
    out[(q * (O * (O + 1) / 2) + pair_idx(i, j, O)) * VV + a * V + b] += val;
  }
}

// x~ = (1 - t)^T x (1 + t^T) for nb stacked nmo x nmo matrices; work has the same size as x
void dress(Context& c, const double* x, double* out, double* work, int64_t nb) {
  hipStream_t s = c.stream;
  const int o = c.o, v = c.v, nmo = c.nmo;
  const int64_t n2 = (int64_t)nmo * nmo;
  PNO_HIP(hipMemcpyAsync(work, x, nb * n2 * sizeof(double), hipMemcpyDeviceToDevice, s));
  // work[:, 0:o] += x[:, o:] t1^T
  gmb(s, false, true, nmo, o, v, 1.0, x + o, nmo, n2, c.t1, v, 0, 1.0, work, nmo, n2, nb);
  PNO_HIP(hipMemcpyAsync(out, work, nb * n2 * sizeof(double), hipMemcpyDeviceToDevice, s));
  // out[o:, :] -= t1^T work[0:o, :]
  gmb(s, true, false, v, nmo, o, -1.0, c.t1, v, 0, work, nmo, n2, 1.0, out + (int64_t)o * nmo, nmo, n2, nb);
}

// f = h + 2 J - K for the pairs (L, R) given (J, K summed over the listed pairs)
void coulomb_exchange(Context& c, const double* L, const double* R, const double* dR, double* J, double* K,
                      double beta) {
  hipStream_t s = c.stream;
  const int64_t n2 = (int64_t)c.nmo * c.nmo;
  // J = dR^T L_flat   (M = 1, N = n2, K = naux)
  gm(s, false, false, 1, n2, c.naux, 1.0, dR, c.naux, L, n2, beta, J, n2);
  // K = sum_Q L_Q[:, 0:o] R_Q[0:o, :]
  gmb(s, false, false, c.nmo, c.nmo, c.o, 1.0, L, c.nmo, n2, R, c.nmo, n2, beta, K, c.nmo, 0, c.naux, true);
}

}  // namespace

void symmetrize_r2(hipStream_t s, int o, int v, double* r2) {
  const int64_t n = (int64_t)o * o * v * v;
  if (n == 0) return;
  hipLaunchKernelGGL(symmetrize_kernel, dim3(grid1(n)), dim3(256), 0, s, o, v, r2);
  PNO_HIP(hipGetLastError());
}

void build_df(Context& c, const double* Bin, const double* epsin, const double* t1in, const double* t2in,
              int precision) {
  hipStream_t s = c.stream;
  const int o = c.o, v = c.v, nmo = c.nmo, naux = c.naux;
  const int64_t n2 = (int64_t)nmo * nmo, ov = c.ov(), oo = (int64_t)o * o, vv = (int64_t)v * v;
  const int64_t oovv = c.oovv();
  c.have_df = false;
  c.have_lad = false;
  c.precision = precision;
  // workspaces and bases of the previous intermediates are dropped first, so that the
  // new ones (e.g. a second copy of W+/- in another precision) have the memory
  c.drop_graphs();
  if (!c.keep_build_tmp) c.sw.release();  // (the CCSD iteration keeps its FP64 sigma workspaces)
  c.pno.reset();
  for (DBuf<float>* b : {&c.DX2f, &c.DXTTf, &c.Whf, &c.g2f, &c.T32, &c.BovTf, &c.BYUf, &c.YUf, &c.Foof,
                         &c.Wvo2f, &c.Zrf})
    b->release();
  for (DBuf<uint16_t>* b : {&c.Whb, &c.Whbs, &c.g2b, &c.TTb, &c.BovQb, &c.BYUb, &c.YUb, &c.Yrb, &c.DXb, &c.DX2b, &c.Gqb,
                            &c.Tvb, &c.Fvob})
    b->release();
  c.Fvvd.release();
  c.Food.release();
  c.bf_rest = false;
  c.ring_y = false;
  c.Yr.release();
  c.Zr.release();

  c.B.alloc((int64_t)naux * n2);
  c.eps.alloc(nmo);
  c.t1.alloc(ov);
  PNO_HIP(hipMemcpyAsync(c.B, Bin, (int64_t)naux * n2 * sizeof(double), hipMemcpyDeviceToDevice, s));
  PNO_HIP(hipMemcpyAsync(c.eps, epsin, nmo * sizeof(double), hipMemcpyDeviceToDevice, s));
  if (t1in)
    PNO_HIP(hipMemcpyAsync(c.t1, t1in, ov * sizeof(double), hipMemcpyDeviceToDevice, s));
  else
    fill(s, ov, 0.0, c.t1);

  // ---------------------------------------------------------------- dressing
  c.Bt.alloc((int64_t)naux * n2);
  dress(c, c.B, c.Bt, c.build_tmp(0, (int64_t)naux * n2), naux);

  // core operator h = diag(eps) - (2 J - K) from the bare factors; dressed h~ and f~
  c.dt.alloc(naux);
  c.dtmp.alloc(naux);
  c.J.alloc(n2);
  c.K.alloc(n2);
  c.h.alloc(n2);
  c.hd.alloc(n2);
  c.fd.alloc(n2);
  hipLaunchKernelGGL(trace_occ_kernel, dim3((naux + 255) / 256), dim3(256), 0, s, naux, nmo, o,
                     (const double*)c.B, (double*)c.dtmp);
  coulomb_exchange(c, c.B, c.B, c.dtmp, c.J, c.K, 0.0);
  axpby(s, n2, -2.0, c.J, 0.0, c.h);
  axpby(s, n2, 1.0, c.K, 1.0, c.h);
  hipLaunchKernelGGL(add_diag_kernel, dim3((nmo + 255) / 256), dim3(256), 0, s, nmo, (const double*)c.eps,
                     (double*)c.h);
  dress(c, c.h, c.hd, c.build_tmp(1, n2), 1);
  hipLaunchKernelGGL(trace_occ_kernel, dim3((naux + 255) / 256), dim3(256), 0, s, naux, nmo, o,
                     (const double*)c.Bt, (double*)c.dt);
  coulomb_exchange(c, c.Bt, c.Bt, c.dt, c.J, c.K, 0.0);
  PNO_HIP(hipMemcpyAsync(c.fd, c.hd, n2 * sizeof(double), hipMemcpyDeviceToDevice, s));
  axpby(s, n2, 2.0, c.J, 1.0, c.fd);
  axpby(s, n2, -1.0, c.K, 1.0, c.fd);

  // ---------------------------------------------------------------- transposed DF blocks [(p,q)][Q]
  c.BovT.alloc(ov * naux);
  c.BvoT.alloc(ov * naux);
  c.BooT.alloc(oo * naux);
  c.BvvT.alloc(vv * naux);
  c.Bvv2.alloc(vv * naux);
  ext(s, o, v, naux, 1, nmo, 1, n2, 0, c.Bt + o, c.BovT);
  ext(s, o, v, naux, 1, 1, nmo, n2, 0, c.Bt + (int64_t)o * nmo, c.BvoT);
  ext(s, o, o, naux, 1, nmo, 1, n2, 0, c.Bt, c.BooT);
  ext(s, v, v, naux, 1, nmo, 1, n2, 0, c.Bt + (int64_t)o * nmo + o, c.BvvT);
  ext(s, v, naux, v, 1, 1, n2, nmo, 0, c.Bt + (int64_t)o * nmo + o, c.Bvv2);

  // ---------------------------------------------------------------- (kc|ld), amplitudes
  // B~_ov = B_ov, so (ia|jb) of the bare and dressed Hamiltonians coincide.
  c.G.alloc(ov * ov);
  gm(s, false, true, ov, ov, naux, 1.0, c.BovT, naux, c.BovT, naux, 0.0, c.G, ov);
  c.T.alloc(oovv);
  if (t2in) {
    PNO_HIP(hipMemcpyAsync(c.T, t2in, oovv * sizeof(double), hipMemcpyDeviceToDevice, s));
  } else {
    perm(s, c.G, o, v, o, v, 0, 2, 1, 3, c.T);
    hipLaunchKernelGGL(mp2_div_kernel, dim3(grid1(oovv)), dim3(256), 0, s, o, v, (const double*)c.eps,
                       (double*)c.T);
    PNO_HIP(hipGetLastError());
  }
  c.U.alloc(oovv);
  perm(s, c.T, o, o, v, v, 0, 1, 3, 2, c.U, -1.0, 0.0);
  axpby(s, oovv, 2.0, c.T, 1.0, c.U);
  c.Tia.alloc(oovv);
  c.Tsia.alloc(oovv);
  c.UiaT.alloc(oovv);
  perm(s, c.T, o, o, v, v, 0, 2, 1, 3, c.Tia);
  perm(s, c.T, o, o, v, v, 0, 3, 1, 2, c.Tsia);
  PNO_HIP(hipMemcpyAsync(c.UiaT, c.Tia, oovv * sizeof(double), hipMemcpyDeviceToDevice, s));
  axpby(s, oovv, -1.0, c.Tsia, 2.0, c.UiaT);

  c.GX.alloc(oovv);
  c.g2.alloc(oovv);
  c.Gq.alloc(oovv);
  perm(s, c.G, o, v, o, v, 0, 3, 2, 1, c.GX);
  perm(s, c.G, o, v, o, v, 0, 2, 1, 3, c.g2);
  perm(s, c.G, o, v, o, v, 0, 2, 3, 1, c.Gq);

  // ---------------------------------------------------------------- dressed integral blocks
  c.OVVO.alloc(oovv);
  gm(s, false, true, ov, ov, naux, 1.0, c.BovT, naux, c.BvoT, naux, 0.0, c.OVVO, ov);
  c.OOVVx.alloc(oovv);
  {
    double* tmp = c.build_tmp(1, oovv);
    gm(s, false, true, oo, vv, naux, 1.0, c.BooT, naux, c.BvvT, naux, 0.0, tmp, vv);
    perm(s, tmp, o, o, v, v, 0, 3, 1, 2, c.OOVVx);
  }
  c.Wh.alloc(oo * oo);
  {
    double* tmp = c.build_tmp(1, oo * oo);
    gm(s, false, true, oo, oo, naux, 1.0, c.BooT, naux, c.BooT, naux, 0.0, tmp, oo);
    perm(s, tmp, o, o, o, o, 1, 3, 0, 2, c.Wh);
    gm(s, false, true, oo, oo, vv, 1.0, c.T, vv, c.g2, vv, 1.0, c.Wh, oo);
  }
  c.OOOVp.alloc(oo * ov);
  {
    double* tmp = c.build_tmp(1, oo * ov);
    gm(s, false, true, oo, ov, naux, 1.0, c.BooT, naux, c.BovT, naux, 0.0, tmp, ov);
    perm(s, tmp, o, o, o, v, 1, 0, 2, 3, c.OOOVp);
  }

  // Fock-like T intermediates
  c.Fqvv.alloc(vv);
  c.Fqoo.alloc(oo);
  c.Fvv.alloc(vv);
  c.Foo.alloc(oo);
  c.fd_ov.alloc(ov);
  {
    double* Ub = c.build_tmp(1, oovv);
    perm(s, c.U, o, o, v, v, 2, 0, 1, 3, Ub);
    gm(s, false, false, v, v, oo * v, -1.0, Ub, oo * v, c.Gq, v, 0.0, c.Fqvv, v);
  }
  gm(s, false, true, o, o, ov * v, 1.0, c.g2, ov * v, c.U, ov * v, 0.0, c.Fqoo, o);
  ext(s, v, v, 1, 1, nmo, 1, 0, 0, c.fd + (int64_t)o * nmo + o, c.Fvv);
  axpby(s, vv, 1.0, c.Fqvv, 1.0, c.Fvv);
  ext(s, o, o, 1, 1, nmo, 1, 0, 0, c.fd, c.Foo);
  axpby(s, oo, 1.0, c.Fqoo, 1.0, c.Foo);
  ext(s, o, v, 1, 1, nmo, 1, 0, 0, c.fd + o, c.fd_ov);

  // ring intermediates as [(k,c),(j,b)]: D = (kc|bj)~ + Dq(T), X = (kj|bc)~ + Xq(T), where the
  // exchange parts -1/2 GX T carry a second -1/2 GX T: the bilinear T-side ring terms
  // T (GX R) of sigma are folded into them (see sigma_rest_block), hence GX T in full
  c.Dr.alloc(oovv);
  c.Xr.alloc(oovv);
  c.DX2.alloc(oovv);
  PNO_HIP(hipMemcpyAsync(c.Dr, c.OVVO, oovv * sizeof(double), hipMemcpyDeviceToDevice, s));
  gm(s, false, true, ov, ov, ov, 0.5, c.G, ov, c.UiaT, ov, 1.0, c.Dr, ov);
  gm(s, false, true, ov, ov, ov, -1.0, c.GX, ov, c.Tia, ov, 1.0, c.Dr, ov);
  PNO_HIP(hipMemcpyAsync(c.Xr, c.OOVVx, oovv * sizeof(double), hipMemcpyDeviceToDevice, s));
  gm(s, false, true, ov, ov, ov, -1.0, c.GX, ov, c.Tsia, ov, 1.0, c.Xr, ov);
  PNO_HIP(hipMemcpyAsync(c.DX2, c.Xr, oovv * sizeof(double), hipMemcpyDeviceToDevice, s));
  axpby(s, oovv, 2.0, c.Dr, -1.0, c.DX2);
  // the right operand of the fused ring product: [Dr | Xr] stacked on [Tia | Tsia], rows of 2 ov
  c.DXTT.alloc(4 * oovv);
  {
    const size_t row = (size_t)ov * sizeof(double), pitch = 2 * row;
    double* tt = c.DXTT + 2 * oovv;
    PNO_HIP(hipMemcpy2DAsync(c.DXTT, pitch, c.Dr, row, row, ov, hipMemcpyDeviceToDevice, s));
    PNO_HIP(hipMemcpy2DAsync(c.DXTT + ov, pitch, c.Xr, row, row, ov, hipMemcpyDeviceToDevice, s));
    PNO_HIP(hipMemcpy2DAsync(tt, pitch, c.Tia, row, row, ov, hipMemcpyDeviceToDevice, s));
    PNO_HIP(hipMemcpy2DAsync(tt + ov, pitch, c.Tsia, row, row, ov, hipMemcpyDeviceToDevice, s));
  }
  // YU[Q][(k,c)] = sum_(j,b) B_jb^Q (2 T - T^s)[(j,b),(k,c)]: the Coulomb (DF) part of the
  // R-side ring intermediate contracted with T ahead of time
  {
    double* U2 = c.build_tmp(1, oovv);
    PNO_HIP(hipMemcpyAsync(U2, c.Tsia, oovv * sizeof(double), hipMemcpyDeviceToDevice, s));
    axpby(s, oovv, 2.0, c.Tia, -1.0, U2);
    c.YU.alloc((int64_t)naux * ov);
    gm(s, true, false, naux, ov, ov, 1.0, c.BovT, naux, U2, ov, 0.0, c.YU, ov);
    // B'_vo enters the ring terms through B'_vo (B~_vo^T + YU): one factor for both
    c.BYU.alloc((int64_t)naux * ov);
    perm(s, c.BvoT, ov, naux, 1, 1, 1, 0, 2, 3, c.BYU);
    axpby(s, (int64_t)naux * ov, 1.0, c.YU, 1.0, c.BYU);
    PNO_HIP(hipStreamSynchronize(s));
  }

  // R1-driven three-body ring terms.  The one-index transformed factors give
  // (ij|ab)' = sum_c r_j^c (ic|ab)~ - sum_l r_l^a (ij|lb)~, so the products of E_X = (ij|ab)'
  // with T_ia and T^s_ia are r1 times the T-only intermediates Yr (v^2 x 2 ov) and Zr
  // (o^2 x 2 ov): 4 o^2 v^3 + 4 o^3 v^2 flop per vector instead of 4 (ov)^3 (and no E_X).
  // Built when Yr and Zr take at most a third of the free memory (or when asked for).
  {
    size_t fr = 0, tot = 0;
    PNO_HIP(hipMemGetInfo(&fr, &tot));
    double need = 8.0 * 2.0 * (double)ov * ((double)vv + (double)oo);
    if (precision == PNOEOM_BF16) need += 2.0 * 2.0 * (double)ov * v * bf16_ld(v);  // + its bfloat16 copy
    c.ring_y = c.ring_mode == 2 || (c.ring_mode == 0 && need <= (double)fr / 3.0);
  }
  if (c.ring_y) {
    const double* TT = c.DXTT + 2 * oovv;  // [Tia | Tsia], rows of 2 ov
    const int64_t ov2 = 2 * ov;
    c.Yr.alloc(vv * ov2);
    c.Zr.alloc(oo * ov2);
    {
      // (ij|lb)~ as [(i,j)][(l,b)] -> [(j,l)][(i,b)] -> Zr
      double* t1 = c.build_tmp(1, oo * ov);
      double* t2 = c.build_tmp(2, oo * ov);
      gm(s, false, true, oo, ov, naux, 1.0, c.BooT, naux, c.BovT, naux, 0.0, t1, ov);
      perm(s, t1, o, o, o, v, 1, 2, 0, 3, t2);
      gm(s, false, false, oo, ov2, ov, 1.0, t2, ov, TT, ov2, 0.0, c.Zr, ov2);
    }
    {
      // slabs of a: (ic|ab)~ as [(a,b)][(i,c)] -> [(a,c)][(i,b)] -> rows (a,c) of Yr
      int64_t na = v;
      const int64_t budget = (int64_t)1 << 28;  // doubles per temporary
      while (na > 1 && na * v * ov > budget) na = (na + 1) / 2;
      double* t1 = c.build_tmp(1, na * v * ov);
      double* t2 = c.build_tmp(2, na * v * ov);
      for (int64_t a0 = 0; a0 < v; a0 += na) {
        const int64_t nab = std::min<int64_t>(na, v - a0);
        gm(s, false, true, nab * v, ov, naux, 1.0, c.BvvT + a0 * v * naux, naux, c.BovT, naux, 0.0, t1, ov);
        perm(s, t1, nab, v, o, v, 0, 3, 2, 1, t2);
        gm(s, false, false, nab * v, ov2, ov, 1.0, t2, ov, TT, ov2, 0.0, c.Yr + a0 * v * ov2, ov2);
      }
    }
    // only the [Dr | Xr] rows of DXTT are used from here on
    DBuf<double> top;
    top.alloc(2 * oovv);
    PNO_HIP(hipMemcpyAsync(top, c.DXTT, 2 * oovv * sizeof(double), hipMemcpyDeviceToDevice, s));
    PNO_HIP(hipStreamSynchronize(s));
    std::swap(c.DXTT.p, top.p);
    std::swap(c.DXTT.n, top.n);
  }

  // Wvo_kbij = sum_cd (kc|bd)~ T_ij^cd stored as [(i,j,b)][k]; built in slabs of b
  c.Wvo2.alloc(oo * v * o);
  {
    int64_t nb = v;
    const int64_t budget = (int64_t)1 << 28;  // doubles per temporary
    while (nb > 1 && (int64_t)o * nb * vv > budget) nb = (nb + 1) / 2;
    double* t1b = c.build_tmp(1, ov * nb * v);
    double* t2b = c.build_tmp(2, ov * nb * v);
    double* t3b = c.build_tmp(3, oo * o * nb);
    for (int64_t b0 = 0; b0 < v; b0 += nb) {
      const int64_t nbb = std::min<int64_t>(nb, v - b0);
      // OVVV[(k,c),(b,d)] for b in slab
      gm(s, false, true, ov, nbb * v, naux, 1.0, c.BovT, naux, c.BvvT + b0 * v * naux, naux, 0.0, t1b, nbb * v);
      perm(s, t1b, o, v, nbb, v, 0, 2, 1, 3, t2b);   // [(k,b),(c,d)]
      gm(s, false, true, oo, o * nbb, vv, 1.0, c.T, vv, t2b, vv, 0.0, t3b, o * nbb);  // [(i,j),(k,b)]
      Perm4 p;
      p.d[0] = oo; p.d[1] = nbb; p.d[2] = o; p.d[3] = 1;
      p.is[0] = o * nbb; p.is[1] = 1; p.is[2] = nbb; p.is[3] = 0;
      p.os[0] = (int64_t)v * o; p.os[1] = o; p.os[2] = 1; p.os[3] = 0;
      permute4(s, p, 1.0, t3b, 0.0, c.Wvo2 + b0 * o);
    }
  }

  // packed ladder matrices W+ / W- built from slabs W_abcd = (ac|bd)~ of rows a, cached for
  // every sigma; or, when they do not fit (or streaming is asked for), rebuilt per sigma
  const int64_t lad_vp = (int64_t)v * (v + 1) / 2, lad_vm = std::max<int64_t>((int64_t)v * (v - 1) / 2, 1);
  c.Wp.release(); c.Wm.release(); c.Wpf.release(); c.Wmf.release(); c.Wpb.release(); c.Wmb.release();
  c.ldpb = bf16_ld(lad_vp);
  c.ldmb = bf16_ld(lad_vm);
  bool stream_w = c.lad_mode == 2;
  if (c.lad_mode == 0) {
    double need = 8.0 * ((double)lad_vp * lad_vp + (double)lad_vm * lad_vm);
    if (precision == PNOEOM_FP32) need *= 1.5;
    if (precision == PNOEOM_BF16) need += 2.0 * ((double)lad_vp * c.ldpb + (double)lad_vm * c.ldmb);
    size_t fr = 0, tot = 0;
    PNO_HIP(hipMemGetInfo(&fr, &tot));
    stream_w = need > 0.6 * (double)fr;
  }
  if (stream_w) {
    prepare_streamed_ladder(c, precision, ladder_budget());
  } else {
    c.lad_streamed = false;
    c.BvvTf.release(); c.BvvTb.release(); c.lad_tmp.release(); c.lad_wp.release(); c.lad_wm.release();
  }
  if (!stream_w) {
    const int64_t vp = (int64_t)v * (v + 1) / 2, vm = (int64_t)v * (v - 1) / 2;
    const bool f32w = precision == PNOEOM_FP32;
    const bool bfw = precision == PNOEOM_BF16;
    c.Wp.alloc(vp * vp);
    c.Wm.alloc(std::max<int64_t>(vm * vm, 1));
    if (f32w) { c.Wpf.alloc(vp * vp); c.Wmf.alloc(std::max<int64_t>(vm * vm, 1)); }
    // bfloat16 copies with rows padded to a multiple of 64 columns (zeros past the end)
    if (bfw) {
      c.Wpb.alloc(vp * c.ldpb);
      c.Wmb.alloc(std::max<int64_t>(vm, 1) * c.ldmb);
      hipLaunchKernelGGL(zero_u16_kernel, dim3(grid1(vp * c.ldpb)), dim3(256), 0, s, vp * c.ldpb, (uint16_t*)c.Wpb);
      hipLaunchKernelGGL(zero_u16_kernel, dim3(grid1(std::max<int64_t>(vm, 1) * c.ldmb)), dim3(256), 0, s,
                         std::max<int64_t>(vm, 1) * c.ldmb, (uint16_t*)c.Wmb);
      PNO_HIP(hipGetLastError());
    }
    int64_t na = v;
    const int64_t budget = (int64_t)1 << 28;
    while (na > 1 && na * v * vv > budget) na = (na + 1) / 2;
    double* tmp = c.build_tmp(0, na * v * vv);
    for (int64_t a0 = 0; a0 < v; a0 += na) {
      const int64_t nab = std::min<int64_t>(na, v - a0);
      gm(s, false, true, nab * v, vv, naux, 1.0, c.BvvT + a0 * v * naux, naux, c.BvvT, naux, 0.0, tmp, vv);
      const int64_t tot = nab * v * vv;
      hipLaunchKernelGGL((ladder_wpm_kernel<double>), dim3(grid1(tot)), dim3(256), 0, s, v, (int)a0, (int)nab,
                         (const double*)tmp, (double*)c.Wp, vp, (double*)c.Wm, vm);
      if (f32w)
        hipLaunchKernelGGL((ladder_wpm_kernel<float>), dim3(grid1(tot)), dim3(256), 0, s, v, (int)a0, (int)nab,
                           (const double*)tmp, (float*)c.Wpf, vp, (float*)c.Wmf, vm);
      if (bfw)
        hipLaunchKernelGGL((ladder_wpm_kernel<uint16_t>), dim3(grid1(tot)), dim3(256), 0, s, v, (int)a0, (int)nab,
                           (const double*)tmp, (uint16_t*)c.Wpb, c.ldpb, (uint16_t*)c.Wmb, c.ldmb);
      PNO_HIP(hipGetLastError());
    }
    PNO_HIP(hipStreamSynchronize(s));
  }
  // BF16: the hole ladder, X_klij, M1 and the DF ring terms run on bfloat16 MFMA when their
  // staging in sigma fits (o <= v and o v naux <= o^2 v^2), else on FP32 like in FP32 mode
  c.bf_rest = precision == PNOEOM_BF16 && c.bf16_scope == 1 && oo * oo <= oovv && ov * naux <= oovv;
  if (precision == PNOEOM_FP32 || (precision == PNOEOM_BF16 && !c.ring_y)) {  // FP32 ring operands
    c.DX2f.alloc(oovv);
    const int64_t ndx = c.ring_y ? 2 * oovv : 4 * oovv;
    c.DXTTf.alloc(ndx);
    to_float(s, oovv, c.DX2, c.DX2f);
    to_float(s, ndx, c.DXTT, c.DXTTf);
  }
  if (precision == PNOEOM_FP32 || (precision == PNOEOM_BF16 && !c.bf_rest)) {  // FP32 operands of the rest
    c.Whf.alloc(oo * oo);
    c.g2f.alloc(oovv);
    c.T32.alloc(oovv);
    c.BovTf.alloc(ov * naux);
    to_float(s, oo * oo, c.Wh, c.Whf);
    to_float(s, oovv, c.g2, c.g2f);
    to_float(s, oovv, c.T, c.T32);
    to_float(s, ov * naux, c.BovT, c.BovTf);
    c.BYUf.alloc((int64_t)naux * ov);
    c.YUf.alloc((int64_t)naux * ov);
    to_float(s, (int64_t)naux * ov, c.BYU, c.BYUf);
    to_float(s, (int64_t)naux * ov, c.YU, c.YUf);
  }
  if (c.bf_rest) {
    c.ldoo = bf16_ld(oo);
    c.ldvv = bf16_ld(vv);
    c.ldov = bf16_ld(ov);
    c.ldq = bf16_ld(naux);
    c.ldv = bf16_ld(v);
    c.Whb.alloc(oo * c.ldoo);
    c.g2b.alloc(oo * c.ldvv);
    c.TTb.alloc(vv * c.ldoo);
    c.BovQb.alloc(naux * c.ldov);
    c.BYUb.alloc(ov * c.ldq);
    c.YUb.alloc(ov * c.ldq);
    c.Food.alloc(o);
    hipLaunchKernelGGL(wh_foo_rows_bf16_kernel, dim3(grid1(oo * c.ldoo)), dim3(256), 0, s, (int64_t)o,
                       (const double*)c.Wh, (const double*)c.Foo, (uint16_t*)c.Whb, c.ldoo, (double*)c.Food);
    c.Whbs.alloc((int64_t)o * (o + 1) / 2 * c.ldoo);
    hipLaunchKernelGGL(pair_rows_gather_kernel, dim3((unsigned)(o * (o + 1) / 2), 1), dim3(256), 0, s, o, (int64_t)0,
                       (const double*)nullptr, (const uint16_t*)c.Whb, c.ldoo, (uint16_t*)c.Whbs);
    PNO_HIP(hipGetLastError());
    bf16_rows(s, oo, vv, c.g2, vv, 1, c.g2b, c.ldvv, c.ldvv);
    auto tr = [&](int64_t R, int64_t C, const double* src, int64_t sb, uint16_t* dst, int64_t ld, int64_t db,
                  int64_t nbat) {
      hipLaunchKernelGGL(bf16_transpose_kernel, dim3((unsigned)((C + 31) / 32), (unsigned)((ld + 31) / 32), (unsigned)nbat),
                         dim3(256), 0, s, R, C, src, sb, dst, ld, db);
    };
    tr(oo, vv, c.T, 0, c.TTb, c.ldoo, 0, 1);        // T [(kl)][(ab)] -> [(ab)][(kl)]
    tr(ov, naux, c.BovT, 0, c.BovQb, c.ldov, 0, 1);  // B~_ov [(jb)][Q] -> [Q][(jb)]
    tr(naux, ov, c.BYU, 0, c.BYUb, c.ldq, 0, 1);    // BYU [Q][(kc)] -> [(kc)][Q]
    tr(naux, ov, c.YU, 0, c.YUb, c.ldq, 0, 1);
    c.ldg = bf16_ld(oo * v);
    c.Gqb.alloc(v * c.ldg);
    tr(oo * v, v, c.Gq, 0, c.Gqb, c.ldg, 0, 1);  // Gq [(k,l,d)][b] -> [b][(k,l,d)]
    c.Tvb.alloc(oo * v * c.ldv);
    bf16_rows(s, oo * v, v, c.T, v, 1, c.Tvb, c.ldv, c.ldv);
    c.Fvvd.alloc(v);
    c.Fvob.alloc(v * c.ldv);
    hipLaunchKernelGGL(offdiag_rows_bf16_kernel, dim3(grid1(v * c.ldv)), dim3(256), 0, s, (int64_t)v, (const double*)c.Fvv,
                       (uint16_t*)c.Fvob, c.ldv, (double*)c.Fvvd);
    PNO_HIP(hipGetLastError());
    if (c.ring_y) {  // Yr[(a,c)][n] -> Yrb[(a,n)][c], one transpose per a
      const int64_t ov2 = 2 * ov;
      c.Yrb.alloc((int64_t)v * ov2 * c.ldv);
      tr(v, ov2, c.Yr, (int64_t)v * ov2, c.Yrb, c.ldv, ov2 * c.ldv, v);
      c.Zrf.alloc(oo * ov2);
      to_float(s, oo * ov2, c.Zr, c.Zrf);
    }
    // FP32 operands of the Fock-type and Wvo products (R Fvv^T, T Ftv^T, Foo R, Fto T, r1 Wvo)
    c.Foof.alloc(oo);
    c.Wvo2f.alloc(oo * v * o);
    c.T32.alloc(oovv);
    to_float(s, oo, c.Foo, c.Foof);
    to_float(s, oo * v * o, c.Wvo2, c.Wvo2f);
    to_float(s, oovv, c.T, c.T32);
    PNO_HIP(hipGetLastError());
  }
  c.DXb.release();
  c.DX2b.release();
  c.RBb.release();
  c.kfold = 0;
  if (precision == PNOEOM_BF16 && c.ring_y) {  // bfloat16 right operands of the ring products
    const int64_t ov2 = 2 * ov;
    c.ldr = bf16_ld(ov);
    const int64_t kr = c.ring_passes * c.ldr;
    c.DXb.alloc(ov2 * kr);
    c.DX2b.alloc(ov * kr);
    bf16_rows(s, ov2, ov, c.DXTT, 1, ov2, c.DXb, c.ldr, kr, c.ring_passes, 1);
    bf16_rows(s, ov, ov, c.DX2, 1, ov, c.DX2b, c.ldr, kr, c.ring_passes, 1);
    if (c.bf_rest && c.ring_passes == 1) {
      // right operand of the fused product (see sigma_rest_block): row n = [Dr^T | DX2^T | BYU^T |
      // YU^T] (column n of Dr, DX2, BYU and YU), rows of kfold = 2 ldr + 2 ldq values
      c.kfold = 2 * c.ldr + 2 * c.ldq;
      c.RBb.alloc(ov * c.kfold);
      bf16_rows(s, ov, ov, c.DXTT, 1, ov2, c.RBb, c.ldr, c.kfold);
      bf16_rows(s, ov, ov, c.DX2, 1, ov, c.RBb + c.ldr, c.ldr, c.kfold);
      bf16_rows(s, ov, naux, c.BYU, 1, ov, c.RBb + 2 * c.ldr, c.ldq, c.kfold);
      bf16_rows(s, ov, naux, c.YU, 1, ov, c.RBb + 2 * c.ldr + c.ldq, c.ldq, c.kfold);
    }
  }
  PNO_HIP(hipStreamSynchronize(s));
  // kept only stacked (DXTT) from here on
  c.Dr.release(); c.Xr.release(); c.Tia.release(); c.Tsia.release();
  if (!c.keep_build_tmp)
    for (DBuf<double>& b : c.btmp) b.release();
  c.have_df = true;
  c.have_lad = true;
}

namespace {
template <typename T>
void grow(DBuf<T>& b, int64_t n) {
  if ((int64_t)b.n < n) b.alloc(std::max<int64_t>(n, 1));
}

// floats of FP32 staging (fa) the bfloat16 left operands of the BF16 ring products take
// (nb ov rows of ring_passes x ldr bfloat16 values); 0 when the ring is not run in BF16
int64_t bf16_ring_floats(const Context& c, int precision, int64_t nb) {
  if (precision != PNOEOM_BF16 || !c.ring_y || !c.DXb.p) return 0;
  if (c.RBb.p) return 0;  // the fused product's left operand has its own buffer (RAb)
  return nb * c.ov() * c.ring_passes * c.ldr;  // two left operands of nb ov rows
}

// BF16 scope 1, one pass: the ring products fused with the DF ring terms, their left operand
// rows written by r2_layouts_kernel (R^s, R_ia) and the R1 part (B'_vo, M1) into RAb, and
// neither R_ia nor R^s kept in FP64
bool ring_fold(const Context& c, int precision) {
  return precision == PNOEOM_BF16 && c.bf_rest && c.ring_y && c.RBb.p && c.DXb.p && c.ring_passes == 1;
}

// bfloat16 values of fa staging that the other BF16 products of sigma_rest take for nb vectors
// (0 when they run in another precision): R2^T rows (hole ladder), then R2 rows (X_klij), then
// Xh rows; U(R)_ia rows (M1); B'_vo, M1 and R1 rows (DF and R1 ring terms); U(R) rows (Ftv);
// the operands of the Fock-type products
int64_t bf16_rest_values(const Context& c, int precision, int64_t nb) {
  if (precision != PNOEOM_BF16 || !c.bf_rest) return 0;
  const int64_t oo = (int64_t)c.o * c.o, vv = (int64_t)c.v * c.v, ov = c.ov();
  const int64_t hole = std::max({vv * c.ldoo, oo * c.ldvv, oo * c.ldoo});
  const int64_t df = 2 * ov * c.ldq + (c.Yrb.p ? (int64_t)c.o * c.ldv : 0);
  // Fock-type block: Fto and R1 in FP32, then R2 and Ftv rows in bfloat16
  const int64_t fock = 2 * (oo + ov + 4) + (oo + 1) * c.v * c.ldv;
  return nb * std::max({hole, ov * c.ldov, df, (int64_t)c.v * c.ldg, fock});
}

// device memory of the per-vector work arrays of sigma_rest (bytes per vector)
int64_t rest_bytes_per_vector(const Context& c, int precision, bool r2c) {
  const bool f32 = precision != PNOEOM_FP64;
  const bool fold = ring_fold(c, precision);
  const int64_t ov = c.ov(), oo = (int64_t)c.o * c.o, vv = (int64_t)c.v * c.v, oovv = c.oovv();
  // 9 o^2 v^2 arrays (Ria, UiaR, UR, ZZ x 2, RE x 2, Zp, OOVVp), 7 when the E_X products go
  // through Yr / Zr (RE holds R^s only, no OOVVp), 1 (UR) with the fused BF16 ring product (no
  // Ria, no RE: their bfloat16 rows go to RAb; no UiaR: its bfloat16 rows go to fa; no ZZ, no
  // Zp: the ring block and the Fock-type sum stay FP32), + R2c for strided input
  const int64_t narr = (c.ring_y ? (fold ? 1 : 7) : 9) + (r2c ? 1 : 0);
  int64_t nd = narr * oovv + (ov + oo + (c.ring_y ? 0 : vv)) * (int64_t)c.naux + ov * c.naux + 2 * oo * oo + ov + vv +
               oo + vv + oo +
               (c.ring_y ? ov + (int64_t)c.nmo * c.o * c.naux : 0);  // (+ the vector's columns of Bc)
  int64_t bytes = nd * (int64_t)sizeof(double);
  if (fold)  // RAb, fz, Sdf (pairs i <= j), S1p
    bytes += ov * c.kfold * (int64_t)sizeof(uint16_t) +
             (oovv + (int64_t)c.o * (c.o + 1) / 2 * vv) * (int64_t)sizeof(float) +
             ov * c.o * ((c.v + kAsmTile - 1) / kAsmTile) * (int64_t)sizeof(double);
  if (f32)  // fa and fc (two oovv each; fa larger when it stages the BF16 operands)
    bytes += (2 * oovv + std::max({2 * oovv, bf16_ring_floats(c, PNOEOM_BF16, 1) + 1,
                                   (bf16_rest_values(c, PNOEOM_BF16, 1) + (fold ? c.v * c.ldg + 8 : 0)) / 2 + 1})) *
             (int64_t)sizeof(float);
  return bytes;
}

}  // namespace

// device bytes per trial vector of one sigma chunk: the rest's work arrays, the
// ladder's packed operands / results and unpacked output, and (PNO space) the
// canonical expansion of the vector and of its sigma
int64_t sigma_bytes_per_vector(const Context& c, int precision, bool pno) {
  const int64_t npair = (int64_t)c.o * (c.o + 1) / 2, vp = (int64_t)c.v * (c.v + 1) / 2;
  const int64_t vm = std::max<int64_t>((int64_t)c.v * (c.v - 1) / 2, 1);
  // (the PNO path expands its vectors with the singles and doubles apart: no R2c)
  int64_t b = rest_bytes_per_vector(c, precision, !pno) +
              (ring_fold(c, precision) ? 0 : c.oovv() * (int64_t)sizeof(double));  // + LadAll
  const int64_t in_elt = precision == PNOEOM_FP64 ? 8 : precision == PNOEOM_FP32 ? 4 : 2;
  const int64_t out_elt = precision == PNOEOM_FP64 ? 8 : 4;
  const int64_t kp = precision == PNOEOM_BF16 ? c.ldpb + c.ldmb : vp + vm;
  b += npair * (kp * in_elt + (vp + vm) * out_elt);
  if (pno) b += 2 * c.vlen() * (int64_t)sizeof(double);
  return b;
}

// bytes currently held by the sigma workspaces (reused by the next chunk)
int64_t sigma_held_bytes(const Context& c) {
  const SigmaWork& w = c.sw;
  int64_t b = 0;
  for (const DBuf<double>* x : {&w.Bp, &w.Bc, &w.hp, &w.Jp, &w.Kp, &w.fp, &w.dp, &w.fp_ov, &w.fp_vv, &w.fp_oo, &w.BvopT,
                                &w.BoopT, &w.BvvpT, &w.R2c, &w.Ria, &w.UiaR, &w.S1p, &w.UR, &w.ZZ,
                                &w.RE, &w.Zp, &w.Xh, &w.O4p, &w.OOVVp, &w.M1, &w.R1c, &w.Ftv, &w.Fto,
                                &w.LadAll, &w.Sp, &w.Am, &w.SigP, &w.SigM, &c.pno.r1, &c.pno.r2, &c.pno.s1,
                                &c.pno.s2})
    b += (int64_t)x->n * 8;
  for (const DBuf<float>* x : {&w.Spf, &w.Amf, &w.SigPf, &w.SigMf, &w.fa, &w.fc, &w.fz, &w.Sdf}) b += (int64_t)x->n * 4;
  b += (int64_t)(w.Spb.n + w.Amb.n + w.RAb.n) * 2;
  return b;
}

// device bytes sigma chunks leave to the caller: 3% of the device, at least 2 GiB (split-K
// partials, graphs and the caller's own tensors)
int64_t sigma_headroom(int64_t total) { return std::max<int64_t>(2ll << 30, total * 3 / 100); }

// vectors per sigma chunk: as many as fit in the free device memory plus what the
// workspaces already hold, less the headroom.  While a graph is captured the decision of
// the eager run is reused.
int sigma_chunk(Context& c, int nvec, int precision, bool pno) {
  if (c.fixed_chunk > 0) return std::max(1, std::min(c.fixed_chunk, nvec));
  if (c.sw_precision >= 0 && c.sw_precision != precision) {
    // another precision's workspaces keep the sizes of its chunk (arrays only grow), which the
    // count below would take as free for this precision's arrays: release them (and the graphs
    // that refer to them), so that the chunk is sized against what is really free
    c.drop_graphs();
    c.sw.release();
    for (DBuf<double>* b : {&c.pno.r1, &c.pno.r2, &c.pno.s1, &c.pno.s2}) b->release();
  }
  c.sw_precision = precision;
  const int64_t per = sigma_bytes_per_vector(c, precision, pno);
  size_t freeb = 0, totalb = 0;
  PNO_HIP(hipMemGetInfo(&freeb, &totalb));
  const int64_t avail = (int64_t)freeb + sigma_held_bytes(c) - sigma_headroom((int64_t)totalb);
  const int64_t nb = avail > 0 ? avail / per : 0;
  c.last_chunk = (int)std::max<int64_t>(1, std::min<int64_t>(nb, nvec));
  return c.last_chunk;
}

namespace {
// The chunk size counts what the workspaces hold as free, so an array a call of this
// precision does not use is released before anything is grown
void trim_sigma_work(Context& c, int precision, bool need_r2c) {
  SigmaWork& w = c.sw;
  if (precision == PNOEOM_FP64) {
    w.fa.release();
    w.fc.release();
  }
  if (ring_fold(c, precision)) {  // (the fused BF16 ring mode keeps the ring block and the
                                  // Fock-type sum in FP32 (fc, fz): no FP64 ZZ, Ria or RE)
    w.Ria.release();
    w.RE.release();
    w.ZZ.release();
    w.LadAll.release();
    w.Zp.release();
    w.UiaR.release();
  } else {
    w.RAb.release();
    w.fz.release();
    w.Sdf.release();
    w.S1p.release();
  }
  if (!need_r2c) w.R2c.release();
}

void alloc_sigma_work(Context& c, int precision, int nb, bool need_r2c) {
  SigmaWork& w = c.sw;
  const int64_t n2 = (int64_t)c.nmo * c.nmo, ov = c.ov(), oo = (int64_t)c.o * c.o, vv = (int64_t)c.v * c.v;
  const int64_t oovv = c.oovv(), B = nb;
  const bool fold = ring_fold(c, precision);
  trim_sigma_work(c, precision, need_r2c);
  // scratch of the R1 one-index transformation (Bc: all vectors of the chunk)
  if (c.ring_y)
    grow(w.Bc, B * c.naux * c.nmo * c.o);
  else
    grow(w.Bp, (int64_t)c.naux * n2);
  grow(w.hp, n2); grow(w.Jp, n2); grow(w.Kp, n2); grow(w.fp, n2); grow(w.dp, c.naux);
  // per-vector arrays, [nb][...]
  grow(w.fp_ov, B * ov); grow(w.fp_vv, B * vv); grow(w.fp_oo, B * oo);
  grow(w.BvopT, B * ov * c.naux); grow(w.BoopT, B * oo * c.naux);
  if (!c.ring_y) grow(w.BvvpT, B * vv * c.naux);
  if (need_r2c) grow(w.R2c, B * oovv);
  grow(w.UR, B * oovv);
  if (fold)  // (U(R)_ia only as bfloat16 rows in fa, sigma1's term as partial sums)
    grow(w.S1p, B * ov * c.o * ((c.v + kAsmTile - 1) / kAsmTile));
  else
    grow(w.UiaR, B * oovv);
  if (fold) {
    grow(w.RAb, B * c.ov() * c.kfold);
    grow(w.fz, B * oovv);
    grow(w.Sdf, B * (int64_t)c.o * (c.o + 1) / 2 * vv);
  } else {
    grow(w.Ria, B * oovv);
    grow(w.RE, (c.ring_y ? 1 : 2) * B * oovv);
    grow(w.ZZ, 2 * B * oovv);
  }
  if (!fold) grow(w.Zp, B * oovv);  // (the FP64 sum of the Fock-type products)
  if (c.ring_y)
    grow(w.R1c, B * ov);
  else
    grow(w.OOVVp, B * oovv);
  grow(w.Xh, B * oo * oo); grow(w.O4p, B * oo * oo); grow(w.M1, B * ov * c.naux);
  grow(w.Ftv, B * vv); grow(w.Fto, B * oo);
  if (precision != PNOEOM_FP64) {
    grow(w.fa, std::max({2 * B * oovv, bf16_ring_floats(c, precision, nb),
                         (bf16_rest_values(c, precision, nb) + (fold ? B * c.v * c.ldg + 8 : 0) + 1) / 2}));
    grow(w.fc, 2 * B * oovv);
  }
}

// batched C_q = alpha op(A_q) op(B_q) + beta C_q with FP32 operands and accumulation,
// C in FP64 with C_q contiguous (ldc = N, sC = M N); fc is FP32 staging of nb M N
void gmbf(hipStream_t s, bool ta, bool tb, int64_t M, int64_t N, int64_t K, double alpha, const float* A, int64_t lda,
          int64_t sA, const float* B, int64_t ldb, int64_t sB, double beta, double* C, int64_t nb, float* fc) {
  GemmDesc<float> d;
  d.ta = ta; d.tb = tb; d.M = M; d.N = N; d.K = K; d.alpha = (float)alpha; d.beta = 0.f;
  d.A = A; d.lda = lda; d.sA = sA; d.B = B; d.ldb = ldb; d.sB = sB; d.C = fc; d.ldc = N; d.sC = M * N;
  d.batch = nb;
  gemm(d, s);
  to_double(s, nb * M * N, fc, C, beta);
}
}  // namespace

namespace {
// s2[q] = Sd[q] + Z(i,j,a,b) + Z(j,i,b,a) for nb vectors, with
// Z(i,j,a,b) = Zp[i][j][a][b] + Ziajb[i][a][j][b] + Z3[j][a][i][b]
// where Ziajb and Z3 of vector q are the two halves of the rows of ZZ[q] ([(i,a)][2 ov]).
// Three of the six reads run along a for fixed b (Zp[j][i][b][:] and the (j,b) / (i,b) rows
// of ZZ), the other three along b: one workgroup takes a 32 x 32 (a, b)
// tile of one pair (i, j) of one vector, sums the a-contiguous terms into LDS with lanes
// along a, and adds them transposed to the b-contiguous terms read and written with lanes
// along b, so that every global access is a contiguous 256-byte row segment.  Zp and ZZ are
// FP64, or FP32 (BF16 mode: the FP32 accumulators of the bfloat16 products, read as they are)
template <typename TS, typename TZ>
__global__ __launch_bounds__(256) void assemble_s2_tiled_kernel(int o, int v, const TS* __restrict__ Sd,
                                                                const TZ* __restrict__ Zp,
                                                                const TZ* __restrict__ ZZ,
                                                                double* __restrict__ s2, int64_t stride2) {
  __shared__ double tile[kAsmTile][kAsmTile + 1];
  const int64_t V = v, O = o, n = O * O * V * V, ov = O * V, ov2 = 2 * ov;
  const int ntb = (v + kAsmTile - 1) / kAsmTile;
  const int a0 = (int)(blockIdx.x / ntb) * kAsmTile, b0 = (int)(blockIdx.x % ntb) * kAsmTile;
  const int64_t i = blockIdx.y / o, j = blockIdx.y % o, q = blockIdx.z;
  const int tx = threadIdx.x % kAsmTile, ty = threadIdx.x / kAsmTile;  // 32 x 8
  const TZ* zp = Zp + q * n;
  const TZ* zz = ZZ + q * 2 * n;
  // terms contiguous along a: tile[b][a]
  for (int bb = ty; bb < kAsmTile; bb += 256 / kAsmTile) {
    const int64_t a = a0 + tx, b = b0 + bb;
    if (a < V && b < V)
      tile[bb][tx] = (double)zp[((j * O + i) * V + b) * V + a] + (double)zz[(j * V + b) * ov2 + i * V + a] +
                     (double)zz[(i * V + b) * ov2 + ov + j * V + a];
  }
  __syncthreads();
  // terms contiguous along b, plus the tile transposed
  for (int aa = ty; aa < kAsmTile; aa += 256 / kAsmTile) {
    const int64_t a = a0 + aa, b = b0 + tx;
    if (a < V && b < V) {
      const int64_t e = ((i * O + j) * V + a) * V + b;
      s2[q * stride2 + e] = (double)Sd[q * n + e] + (double)zp[e] + (double)zz[(i * V + a) * ov2 + j * V + b] +
                            (double)zz[(j * V + a) * ov2 + ov + i * V + b] + tile[tx][aa];
    }
  }
}

// Fused BF16 mode: sigma2 has the pair symmetry s_ji^ba = s_ij^ab, and so has each block that
// enters it, so one workgroup per 32 x 32 (a, b) tile of a pair i <= j of vector q forms
//   s_ij^ab = Sd_ij^ab + D(i,j,a,b) + D(j,i,b,a) + R_ij^ab (Fvv_aa + Fvv_bb - Foo_ii - Foo_jj),
//   D(i,j,a,b) = Zp_ij^ab + Z[(i,a)][(j,b)] + Z'[(j,a)][(i,b)]
// from the FP32 direct (pairs i <= j in row-major order), Fock-type and ring blocks (Z | Z' the
// two halves of the ring rows) and
// the orbital-energy terms (dv, doo: diagonals of Fvv and Foo) in FP64, and writes it to (i, j)
// and, transposed through LDS, to (j, i): every element of the blocks is read once (Sd at
// (i, j) only).  The D(j,i,b,a) terms are read along a into LDS, the rest along b.
__global__ __launch_bounds__(256) void assemble_s2_sym_kernel(int o, int v, const float* __restrict__ Sd,
                                                              const float* __restrict__ Zp,
                                                              const float* __restrict__ ZZ,
                                                              const double* __restrict__ R2,
                                                              const double* __restrict__ dv,
                                                              const double* __restrict__ doo,
                                                              double* __restrict__ s2, int64_t stride2) {
  __shared__ double tile[kAsmTile][kAsmTile + 1];
  const int64_t V = v, O = o, n = O * O * V * V, ov = O * V, ov2 = 2 * ov;
  const int ntb = (v + kAsmTile - 1) / kAsmTile;
  const int a0 = (int)(blockIdx.x / ntb) * kAsmTile, b0 = (int)(blockIdx.x % ntb) * kAsmTile;
  int64_t p = blockIdx.y, i = 0;  // pair p (i <= j, row-major) -> (i, j)
  while (p >= O - i) {
    p -= O - i;
    ++i;
  }
  const int64_t j = i + p, q = blockIdx.z;
  const int tx = threadIdx.x % kAsmTile, ty = threadIdx.x / kAsmTile;  // 32 x 8
  const float* zp = Zp + q * n;
  const float* zz = ZZ + q * 2 * n;
  // D(j,i,b,a), contiguous along a: tile[b][a]
  for (int bb = ty; bb < kAsmTile; bb += 256 / kAsmTile) {
    const int64_t a = a0 + tx, b = b0 + bb;
    if (a < V && b < V)
      tile[bb][tx] = (double)zp[((j * O + i) * V + b) * V + a] + (double)zz[(j * V + b) * ov2 + i * V + a] +
                     (double)zz[(i * V + b) * ov2 + ov + j * V + a];
  }
  __syncthreads();
  double val[kAsmTile / 8];
  const double fij = doo[i] + doo[j];
#pragma unroll
  for (int k = 0; k < kAsmTile / 8; ++k) {
    const int aa = ty + 8 * k;
    const int64_t a = a0 + aa, b = b0 + tx;
    val[k] = 0.0;
    if (a < V && b < V) {
      const int64_t e = ((i * O + j) * V + a) * V + b;
      val[k] = (double)Sd[(q * (O * (O + 1) / 2) + blockIdx.y) * V * V + a * V + b] + (double)zp[e] + (double)zz[(i * V + a) * ov2 + j * V + b] +
               (double)zz[(j * V + a) * ov2 + ov + i * V + b] + tile[tx][aa] +
               R2[q * n + e] * (dv[a] + dv[b] - fij);
      s2[q * stride2 + e] = val[k];
    }
  }
  if (i == j) return;  // (uniform) the mirror tile writes the mirror elements of a diagonal pair
  __syncthreads();     // the reads of the tile are done
#pragma unroll
  for (int k = 0; k < kAsmTile / 8; ++k) tile[ty + 8 * k][tx] = val[k];  // tile[a][b]
  __syncthreads();
  // s_ji^ba = s_ij^ab, rows b of pair (j, i) along a
  for (int bb = ty; bb < kAsmTile; bb += 256 / kAsmTile) {
    const int64_t a = a0 + tx, b = b0 + bb;
    if (a < V && b < V) s2[q * stride2 + ((j * O + i) * V + b) * V + a] = tile[tx][bb];
  }
}

// The layouts of R2 that the rest of sigma reads, in one pass over R2 (one workgroup per
// 32 x 32 (a, b) tile of a pair (i, j) of a vector, the tile and its mirror (b, a) in LDS):
//   Ria[(q,i,a)][(j,b)] = R_ij^ab,   UiaR[(q,i,a)][(j,b)] = UR[q][i][j][a][b] = 2 R_ij^ab - R_ij^ba,
//   R^s[(q,i,b)][(j,a)] = R_ij^ab (rows of ldre in RE)
// every store runs along a row segment of 32 consecutive values (R^s through the LDS transpose)
//   (fused BF16 ring product: -R^s and R_ia instead as bfloat16 into the rows of RAb, the
//    first two blocks of ldr values of rows of ldra, and no FP64 Ria / RE; U(R)_ia as bfloat16
//    rows of ldu (UiaRb, the M1 operand) instead of FP64, and sigma1's U(R)_ia f'_ov term as
//    partial sums over the b of a tile, s1p[(q,i,a)][(j, b tile)] = sum_b U(R)_ia,jb f'_jb; and
//    U(R) also as the bfloat16 rows [(q,a)][(i,j,b)] of ldg values of the Ftv product, URb)
__global__ __launch_bounds__(256) void r2_layouts_kernel(int o, int v, const double* __restrict__ R2,
                                                         double* __restrict__ Ria, double* __restrict__ UiaR,
                                                         double* __restrict__ UR,
                                                         double* __restrict__ RE, int64_t ldre,
                                                         uint16_t* __restrict__ RAb, int64_t ldra, int64_t ldr,
                                                         uint16_t* __restrict__ UiaRb, int64_t ldu,
                                                         const double* __restrict__ fdov, double* __restrict__ s1p,
                                                         uint16_t* __restrict__ URb, int64_t ldg) {
  __shared__ double t[kAsmTile][kAsmTile + 1];  // t[a - a0][b - b0] = R_ij^ab
  __shared__ double u[kAsmTile][kAsmTile + 1];  // u[b - b0][a - a0] = R_ij^ba
  const int64_t V = v, O = o, vv = V * V, n = O * O * vv;
  const int ntb = (v + kAsmTile - 1) / kAsmTile;
  const int a0 = (int)(blockIdx.x / ntb) * kAsmTile, b0 = (int)(blockIdx.x % ntb) * kAsmTile;
  const int64_t i = blockIdx.y / o, j = blockIdx.y % o, q = blockIdx.z;
  const int64_t base = q * n + (i * O + j) * vv;
  const double* R = R2 + base;
  const int tx = threadIdx.x % kAsmTile, ty = threadIdx.x / kAsmTile;  // 32 x 8
  for (int r = ty; r < kAsmTile; r += 256 / kAsmTile) {
    const int64_t a = a0 + r, b = b0 + tx;
    t[r][tx] = (a < V && b < V) ? R[a * V + b] : 0.0;
    const int64_t b2 = b0 + r, a2 = a0 + tx;
    u[r][tx] = (b2 < V && a2 < V) ? R[b2 * V + a2] : 0.0;
  }
  __syncthreads();
  for (int r = ty; r < kAsmTile; r += 256 / kAsmTile) {
    const int64_t a = a0 + r, b = b0 + tx;
    double part = 0.0;
    if (a < V && b < V) {
      const double x = t[r][tx], y = u[tx][r];
      const int64_t e = base + a * V + b;
      const int64_t f = q * n + ((i * V + a) * O + j) * V + b;
      if (RAb)
        RAb[((q * O + i) * V + a) * ldra + ldr + j * V + b] = bf16_bits(x);
      else
        Ria[f] = x;
      const double uia = 2.0 * x - y;
      if (UiaRb)
        UiaRb[((q * O + i) * V + a) * ldu + j * V + b] = bf16_bits(uia);
      else
        UiaR[f] = uia;
      UR[e] = uia;
      if (URb) URb[(q * V + a) * ldg + (i * O + j) * V + b] = bf16_bits(uia);
      if (s1p) part = uia * fdov[j * V + b];
    }
    if (s1p) {  // (uniform) sum over the 32 lanes of this row (one half of a wave)
      for (int m = 16; m >= 1; m >>= 1) part += __shfl_xor(part, m, 32);
      if (tx == 0 && a < V) s1p[((q * O + i) * V + a) * (O * ntb) + j * ntb + b0 / kAsmTile] = part;
    }
  }
  for (int r = ty; r < kAsmTile; r += 256 / kAsmTile) {
    const int64_t b = b0 + r, a = a0 + tx;
    if (a < V && b < V) {
      if (RAb)
        RAb[((q * O + i) * V + b) * ldra + j * V + a] = bf16_bits(-t[tx][r]);
      else
        RE[((q * O + i) * V + b) * ldre + j * V + a] = t[tx][r];
    }
  }
}

// s1[q][r] += sum_m part[(q ov + r) nm + m] for r < ov (the partial sums of r2_layouts_kernel,
// in order)
__global__ void s1_partials_kernel(int64_t nb, int64_t ov, int64_t nm, const double* __restrict__ part,
                                   double* __restrict__ s1, int64_t stride1) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < nb * ov; e += (int64_t)gridDim.x * blockDim.x) {
    double acc = 0.0;
    for (int64_t m = 0; m < nm; ++m) acc += part[e * nm + m];
    s1[(e / ov) * stride1 + e % ov] += acc;
  }
}

// out[r ld + c] = 0 for rows r < rows and columns c0 <= c < c1 (padding of bfloat16 rows)
__global__ void zero_cols_kernel(int64_t rows, int64_t ld, int64_t c0, int64_t c1, uint16_t* __restrict__ out) {
  const int64_t w = c1 - c0, total = rows * w;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x)
    out[(e / w) * ld + c0 + e % w] = 0;
}

// every sigma term except the particle ladder, for nb vectors at once; the caller
// has written the ladder of vector q into Sd + q * oovv (in the fused BF16 ring mode Sd is
// null: the packed ladder results of the chunk are added into the FP32 direct block Sdf
// here).  Contractions whose one
// operand is a fixed intermediate run as one batched GEMM over the vectors.
void sigma_rest_block(Context& c, int nb, const double* r1, int64_t stride1, const double* r2, int64_t stride2,
                      double* s1, double* s2, int precision, double* Sd) {
  PNO_CHECK(Sd || ring_fold(c, precision), PNOEOM_EINVAL, "sigma: no ladder block");
  SigmaWork& w = c.sw;
  hipStream_t s = c.stream;
  const int o = c.o, v = c.v, nmo = c.nmo, naux = c.naux;
  const int64_t n2 = (int64_t)nmo * nmo, ov = c.ov(), oo = (int64_t)o * o, vv = (int64_t)v * v;
  const int64_t oovv = c.oovv(), oon = oo * naux, ovn = ov * naux, vvn = vv * naux, o4 = oo * oo;
  const int64_t npair = (int64_t)o * (o + 1) / 2;
  const bool f32 = precision != PNOEOM_FP64;  // FP32 or BF16: FP32 contractions here
  alloc_sigma_work(c, precision, nb, stride2 != oovv);

  // ---------------------------------------------------------------- R1: one-index transformed factors, per vector
  // B'^Q = -r^T B~^Q (virtual rows) + B~^Q r^T (occupied columns) has a zero occupied-virtual
  // block, and with the T-only ring intermediates only its occupied columns are read: the
  // oo and vo blocks Bc[Q][p][i] = B'^Q_{p,i} (nmo x o), the Coulomb part through the one-index
  // transformation of D = sum_Q dt_Q B~^Q (c.J) and the exchange part from Bc (without them the
  // whole B' is formed for its vv block)
  // Bc holds all vectors of the block, [Q][p][(q, i)] (row stride nbo): the product over the
  // virtual columns is one GEMM over all rows (Q, p) of B~ and, with uniformly strided r1 rows,
  // over all vectors at once (B~'s vo block read once)
  const int64_t ldc1 = (int64_t)nb * o, sc = (int64_t)nmo * ldc1;
  if (c.ring_y) {
    if (stride1 == ov)
      gm(s, false, true, (int64_t)naux * nmo, ldc1, v, 1.0, c.Bt + o, nmo, r1, v, 0.0, w.Bc, ldc1);
    else
      for (int q = 0; q < nb; ++q)
        gm(s, false, true, (int64_t)naux * nmo, o, v, 1.0, c.Bt + o, nmo, r1 + q * stride1, v, 0.0, w.Bc + q * o, ldc1);
  }
  for (int q = 0; q < nb && c.ring_y; ++q) {
    const double* r1q = r1 + q * stride1;
    double* bcq = w.Bc + q * o;  // this vector's columns of Bc
    gmb(s, true, false, v, o, o, -1.0, r1q, v, 0, c.Bt, nmo, n2, 1.0, bcq + (int64_t)o * ldc1, ldc1, sc, naux);
    fill(s, n2, 0.0, w.hp);
    gm(s, true, false, v, nmo, o, -1.0, r1q, v, c.hd, nmo, 1.0, w.hp + (int64_t)o * nmo, nmo);
    gm(s, false, true, nmo, o, v, 1.0, c.hd + o, nmo, r1q, v, 1.0, w.hp, nmo);
    hipLaunchKernelGGL(trace_rows_kernel, dim3((naux + 255) / 256), dim3(256), 0, s, naux, ldc1, sc, o,
                       (const double*)bcq, (double*)w.dp);
    // J' = sum_Q dp_Q B~^Q + (one-index transformed D);  K' = sum_Q Bc^Q B~^Q[occ, :] + B~^Q[:, occ] Bc^Q[occ, :]
    gm(s, false, false, 1, n2, naux, 1.0, w.dp, naux, c.Bt, n2, 0.0, w.Jp, n2);
    gm(s, true, false, v, nmo, o, -1.0, r1q, v, c.J, nmo, 1.0, w.Jp + (int64_t)o * nmo, nmo);
    gm(s, false, true, nmo, o, v, 1.0, c.J + o, nmo, r1q, v, 1.0, w.Jp, nmo);
    gmb(s, false, false, nmo, nmo, o, 1.0, bcq, ldc1, sc, c.Bt, nmo, n2, 0.0, w.Kp, nmo, 0, naux, true);
    gmb(s, false, false, nmo, o, o, 1.0, c.Bt, nmo, n2, bcq, ldc1, sc, 1.0, w.Kp, nmo, 0, naux, true);
    PNO_HIP(hipMemcpyAsync(w.fp, w.hp, n2 * sizeof(double), hipMemcpyDeviceToDevice, s));
    axpby(s, n2, 2.0, w.Jp, 1.0, w.fp);
    axpby(s, n2, -1.0, w.Kp, 1.0, w.fp);
    ext(s, o, v, 1, 1, nmo, 1, 0, 0, w.fp + o, w.fp_ov + q * ov);
    ext(s, v, v, 1, 1, nmo, 1, 0, 0, w.fp + (int64_t)o * nmo + o, w.fp_vv + q * vv);
    ext(s, o, o, 1, 1, nmo, 1, 0, 0, w.fp, w.fp_oo + q * oo);
    ext(s, o, v, naux, 1, 1, ldc1, sc, 0, bcq + (int64_t)o * ldc1, w.BvopT + q * ovn);  // [(i,a)][Q] = B'^Q_{o+a,i}
    ext(s, o, o, naux, 1, ldc1, 1, sc, 0, bcq, w.BoopT + q * oon);                      // [(j,i)][Q] = B'^Q_{j,i}
    ext(s, o, v, 1, 1, 1, nmo, 0, 0, w.fp + (int64_t)o * nmo, s1 + q * stride1);  // f'_ai
  }
  for (int q = 0; q < nb && !c.ring_y; ++q) {
    const double* r1q = r1 + q * stride1;
    fill(s, (int64_t)naux * n2, 0.0, w.Bp);
    gmb(s, true, false, v, nmo, o, -1.0, r1q, v, 0, c.Bt, nmo, n2, 1.0, w.Bp + (int64_t)o * nmo, nmo, n2, naux);
    gmb(s, false, true, nmo, o, v, 1.0, c.Bt + o, nmo, n2, r1q, v, 0, 1.0, w.Bp, nmo, n2, naux);
    fill(s, n2, 0.0, w.hp);
    gm(s, true, false, v, nmo, o, -1.0, r1q, v, c.hd, nmo, 1.0, w.hp + (int64_t)o * nmo, nmo);
    gm(s, false, true, nmo, o, v, 1.0, c.hd + o, nmo, r1q, v, 1.0, w.hp, nmo);
    hipLaunchKernelGGL(trace_occ_kernel, dim3((naux + 255) / 256), dim3(256), 0, s, naux, nmo, o,
                       (const double*)w.Bp, (double*)w.dp);
    // J' = dt^T Bp + dp^T Bt ; K' = sum_Q Bp_Q[:,occ] Bt_Q[occ,:] + Bt_Q[:,occ] Bp_Q[occ,:]
    gm(s, false, false, 1, n2, naux, 1.0, c.dt, naux, w.Bp, n2, 0.0, w.Jp, n2);
    gm(s, false, false, 1, n2, naux, 1.0, w.dp, naux, c.Bt, n2, 1.0, w.Jp, n2);
    gmb(s, false, false, nmo, nmo, o, 1.0, w.Bp, nmo, n2, c.Bt, nmo, n2, 0.0, w.Kp, nmo, 0, naux, true);
    gmb(s, false, false, nmo, nmo, o, 1.0, c.Bt, nmo, n2, w.Bp, nmo, n2, 1.0, w.Kp, nmo, 0, naux, true);
    PNO_HIP(hipMemcpyAsync(w.fp, w.hp, n2 * sizeof(double), hipMemcpyDeviceToDevice, s));
    axpby(s, n2, 2.0, w.Jp, 1.0, w.fp);
    axpby(s, n2, -1.0, w.Kp, 1.0, w.fp);
    ext(s, o, v, 1, 1, nmo, 1, 0, 0, w.fp + o, w.fp_ov + q * ov);
    ext(s, v, v, 1, 1, nmo, 1, 0, 0, w.fp + (int64_t)o * nmo + o, w.fp_vv + q * vv);
    ext(s, o, o, 1, 1, nmo, 1, 0, 0, w.fp, w.fp_oo + q * oo);
    ext(s, o, v, naux, 1, 1, nmo, n2, 0, w.Bp + (int64_t)o * nmo, w.BvopT + q * ovn);
    ext(s, o, o, naux, 1, nmo, 1, n2, 0, w.Bp, w.BoopT + q * oon);
    ext(s, v, v, naux, 1, nmo, 1, n2, 0, w.Bp + (int64_t)o * nmo + o, w.BvvpT + q * vvn);
    ext(s, o, v, 1, 1, 1, nmo, 0, 0, w.fp + (int64_t)o * nmo, s1 + q * stride1);  // f'_ai
  }

  // ---------------------------------------------------------------- R2 layouts, [nb][...]
  const double* R2 = r2;
  if (stride2 != oovv) {
    Perm4 p;
    p.d[0] = nb; p.d[1] = 1; p.d[2] = 1; p.d[3] = oovv;
    p.is[0] = stride2; p.is[1] = 0; p.is[2] = 0; p.is[3] = 1;
    p.os[0] = oovv; p.os[1] = 0; p.os[2] = 0; p.os[3] = 1;
    permute4(s, p, 1.0, r2, 0.0, w.R2c);
    R2 = w.R2c;
  }
  const int64_t nbo = (int64_t)nb * o;
  const int64_t ov2 = 2 * ov;
  const int64_t ldre = c.ring_y ? ov : ov2;  // RE rows: [R^s] or [R^s | E_X]
  // Ria, R^s (left half of the rows of RE), UiaR = 2 R_ia - R^s and UR in one pass over R2
  const bool fold = ring_fold(c, precision);
  // (fused mode: the bfloat16 rows of U(R) for the Ftv product, written by the layout pass at
  // the end of fa, beyond every staging used before the Ftv product)
  uint16_t* urb = nullptr;
  if (fold && c.Gqb.p) {
    const int64_t need = (int64_t)nb * v * c.ldg, cap = 2 * (int64_t)w.fa.n;
    PNO_CHECK(cap >= need + bf16_rest_values(c, precision, nb), PNOEOM_EINVAL, "sigma: BF16 staging too small");
    urb = reinterpret_cast<uint16_t*>((float*)w.fa) + ((cap - need) & ~(int64_t)7);
  }
  {
    const unsigned ntb = (unsigned)((v + kAsmTile - 1) / kAsmTile);
    PNO_CHECK((int64_t)o * o <= 65535 && nb <= 65535, PNOEOM_EINVAL, "sigma: too many pairs or vectors per block");
    uint16_t* rab = fold ? (uint16_t*)w.RAb : nullptr;
    // (fused mode: U(R)_ia as the bfloat16 rows of the M1 product in fa, and sigma1's
    // U(R)_ia f'_ov term as partial sums, no FP64 U(R)_ia)
    uint16_t* ub = fold ? reinterpret_cast<uint16_t*>((float*)w.fa) : nullptr;
    hipLaunchKernelGGL(r2_layouts_kernel, dim3(ntb * ntb, (unsigned)(o * o), (unsigned)nb), dim3(256), 0, s, o, v,
                       R2, (double*)w.Ria, (double*)w.UiaR, (double*)w.UR, (double*)w.RE, ldre, rab, c.kfold,
                       c.ldr, ub, c.ldov, (const double*)c.fd_ov, fold ? (double*)w.S1p : (double*)nullptr, urb,
                       c.ldg);
    PNO_HIP(hipGetLastError());
    if (fold && c.ldov > ov)
      hipLaunchKernelGGL(zero_cols_kernel, dim3(grid1((int64_t)nb * ov * (c.ldov - ov))), dim3(256), 0, s,
                         (int64_t)nb * ov, c.ldov, ov, c.ldov, ub);
    if (urb && c.ldg > oo * v)  // (padding of the Ftv operand rows: zeros, as the product reads them)
      hipLaunchKernelGGL(zero_cols_kernel, dim3(grid1((int64_t)nb * v * (c.ldg - oo * v))), dim3(256), 0, s,
                         (int64_t)nb * v, c.ldg, oo * v, c.ldg, urb);
    if (fold)
      hipLaunchKernelGGL(s1_partials_kernel, dim3(grid1((int64_t)nb * ov)), dim3(256), 0, s, (int64_t)nb, ov,
                         (int64_t)o * ntb, (const double*)w.S1p, s1, stride1);
    PNO_HIP(hipGetLastError());
    if (fold && c.ldr > ov) {  // padding of the -R^s and R_ia blocks of the rows
      const int64_t rows = (int64_t)nb * ov;
      hipLaunchKernelGGL(zero_cols_kernel, dim3(grid1(rows * (c.ldr - ov))), dim3(256), 0, s, rows, c.kfold, ov, c.ldr,
                         rab);
      hipLaunchKernelGGL(zero_cols_kernel, dim3(grid1(rows * (c.ldr - ov))), dim3(256), 0, s, rows, c.kfold,
                         c.ldr + ov, 2 * c.ldr, rab);
      PNO_HIP(hipGetLastError());
    }
  }

  // ---------------------------------------------------------------- sigma1
  // (s1[q] += U_ia fp_ov[q] for all vectors in one product, U_ia read once)
  gm(s, false, true, nb, ov, ov, 1.0, w.fp_ov, ov, c.UiaT, ov, 1.0, s1, stride1);
  gmb(s, true, false, o, v, o, -1.0, c.Fqoo, o, 0, r1, v, stride1, 1.0, s1, v, stride1, nb);
  gmb(s, false, true, o, v, v, 1.0, r1, v, stride1, c.Fqvv, v, 0, 1.0, s1, v, stride1, nb);
  if (!fold)  // (the fused mode summed it in the layout pass)
    gmb(s, false, false, ov, 1, ov, 1.0, w.UiaR, ov, oovv, c.fd_ov, 1, 0, 1.0, s1, 1, stride1, nb);
  // (FP32 / BF16: the products with a T-only right factor below run on FP32 MFMA, their
  // per-vector left operands staged in FP32 in fa; the staging holds 2 nb o^2 v^2 floats in
  // each of fa and fc: M1 stages nb o v naux floats in fc, R2 and Xh take nb (o^2 v^2 + o^4)
  // in fa and Xh's product nb o^4 in fc, so o <= v is needed besides o v naux <= 2 o^2 v^2)
  // (BF16 with the bfloat16 operands built: these products and those of the hole ladder,
  // X_klij and the DF and R1 ring terms run on bfloat16 MFMA with FP32 accumulation, the
  // per-vector operands converted into bfloat16 rows staged in fa, the FP32 results in fc)
  const bool bfr = precision == PNOEOM_BF16 && c.bf_rest;
  const bool f32x = !bfr && f32 && ovn <= 2 * oovv && o4 <= oovv;
  uint16_t* hb = reinterpret_cast<uint16_t*>((float*)w.fa);
  // rows m < M of K values, src[m sm + k], as bfloat16 rows of ld values (zero beyond K)
  auto rows_bf16 = [&](int64_t Mr, int64_t Kr, const double* src, int64_t sm, uint16_t* out, int64_t ld) {
    bf16_rows(s, Mr, Kr, src, sm, 1, out, ld, ld);
  };
  // C = alpha A B^T + beta C with A [Mg][ld], B [Ng][ld] bfloat16 rows, C FP32 rows of ldc
  auto bgemm = [&](int64_t Mg, int64_t Ng, int64_t ld, float alpha, const uint16_t* A, const uint16_t* Bm,
                   float beta, float* C, int64_t ldc) {
    GemmBf16Desc d;
    d.M = Mg; d.N = Ng; d.K = ld; d.alpha = alpha; d.beta = beta; d.A = A; d.lda = ld; d.B = Bm; d.ldb = ld;
    d.C = C; d.ldc = ldc;
    gemm_bf16(d, s);
  };
  if (bfr) {
    // M1[(q,i,a)][Q] = sum_(jb) U(R)_ia[(q,i,a)][(jb)] B~_ov[(jb)][Q], all vectors in one product
    if (!fold) rows_bf16(nb * ov, ov, w.UiaR, ov, hb, c.ldov);  // (the fused mode's layout pass wrote them)
    bgemm(nb * ov, naux, c.ldov, 1.f, hb, c.BovQb, 0.f, w.fc, naux);
    to_double(s, nb * ovn, w.fc, w.M1, 0.0);
  } else if (f32x) {
    to_float(s, nb * oovv, w.UiaR, w.fa);
    gmbf(s, false, false, ov, naux, ov, 1.0, w.fa, ov, oovv, c.BovTf, naux, 0, 0.0, w.M1, nb, w.fc);
  } else {
    gmb(s, false, false, ov, naux, ov, 1.0, w.UiaR, ov, oovv, c.BovT, naux, 0, 0.0, w.M1, naux, ovn, nb);
  }
  if (stride1 == ov)  // rows (q, i) of M1 and of s1 uniformly strided: one product, Bvv2 read once
    gm(s, false, false, (int64_t)nb * o, v, (int64_t)v * naux, 1.0, w.M1, (int64_t)v * naux, c.Bvv2, v, 1.0, s1, v);
  else
    gmb(s, false, false, o, v, (int64_t)v * naux, 1.0, w.M1, (int64_t)v * naux, ovn, c.Bvv2, v, 0, 1.0, s1, v,
        stride1, nb);
  // s1[q][i][a] -= sum_(k,l,c) OOOV'[i][(k,l,c)] U(R)[q][k][l][a][c]: per vector one product per
  // pair (k, l) (K = c), summed over the pairs into s1 (U(R) read in place, no a <-> b copy)
  for (int q = 0; q < nb; ++q)
    gmb(s, false, true, o, v, v, -1.0, c.OOOVp, oo * v, v, w.UR + q * oovv, v, vv, 1.0, s1 + q * stride1, v, 0, oo,
        true);

  // ---------------------------------------------------------------- sigma2, direct (not P-symmetrised)
  float* R2f = w.fa;             // FP32 staging of R2, then of Xh after it
  float* Xhf = w.fa + nb * oovv;
  if (bfr) {
    // hole ladder Sd[q] += Wh R2[q] (R2[q]^T as bfloat16 rows [(ab)][(kl)]), FP32 into fc[q]
    hipLaunchKernelGGL(bf16_transpose_kernel, dim3((unsigned)((vv + 31) / 32), (unsigned)((c.ldoo + 31) / 32), (unsigned)nb),
                       dim3(256), 0, s, oo, vv, R2, oovv, hb, c.ldoo, vv * c.ldoo);
    PNO_HIP(hipGetLastError());
    // (the fused mode keeps this direct block in FP32, Sdf, for the pairs i <= j only (the
    // assembly reads no other): rows of Whbs, the ladder added into it below)
    float* dblk = fold ? (float*)w.Sdf : (float*)w.fc;
    const int64_t nrw = fold ? npair : oo;  // rows (pairs) of the direct block per vector
    for (int q = 0; q < nb; ++q)
      bgemm(nrw, vv, c.ldoo, 1.f, fold ? (const uint16_t*)c.Whbs : (const uint16_t*)c.Whb, hb + q * vv * c.ldoo, 0.f,
            dblk + q * nrw * vv, vv);
    // Xh[(q,i,j)][(kl)] = sum_(ab) R2[(q,i,j)][(ab)] g2[(kl)][(ab)], into fc after the ladder block
    rows_bf16(nb * oo, vv, R2, vv, hb, c.ldvv);
    bgemm(nb * oo, oo, c.ldvv, 1.f, hb, c.g2b, 0.f, w.fc + nb * oovv, oo);
    to_double(s, nb * o4, w.fc + nb * oovv, w.Xh, 0.0);
  } else if (f32x) {
    to_float(s, nb * oovv, R2, R2f);
    gmbf(s, false, false, oo, vv, oo, 1.0, c.Whf, oo, 0, R2f, vv, oovv, 1.0, Sd, nb, w.fc);
    gmbf(s, false, true, oo, oo, vv, 1.0, R2f, vv, oovv, c.g2f, vv, 0, 0.0, w.Xh, nb, w.fc);
  } else {
    gmb(s, false, false, oo, vv, oo, 1.0, c.Wh, oo, 0, R2, vv, oovv, 1.0, Sd, vv, oovv, nb);
    gmb(s, false, true, oo, oo, vv, 1.0, R2, vv, oovv, c.g2, vv, 0, 0.0, w.Xh, oo, o4, nb);
  }
  gmb(s, false, true, oo, oo, naux, 1.0, w.BoopT, naux, oon, c.BooT, naux, 0, 0.0, w.O4p, oo, o4, nb);
  gmb(s, false, true, oo, oo, naux, 1.0, c.BooT, naux, 0, w.BoopT, naux, oon, 1.0, w.O4p, oo, o4, nb);
  {
    const int64_t dims[4] = {o, o, o, o};
    const int pp[4] = {1, 3, 0, 2};
    permute_c(s, dims, pp, 1.0, w.O4p, 1.0, w.Xh, nb);
  }
  if (bfr) {
    // Sd[q] += Xh[q] T, all vectors in one product onto the ladder block in fc (the fused
    // mode: the rows (q, i <= j) onto Sdf)
    float* dblk = fold ? (float*)w.Sdf : (float*)w.fc;
    if (fold) {
      hipLaunchKernelGGL(pair_rows_gather_kernel, dim3((unsigned)npair, (unsigned)nb), dim3(256), 0, s, o, oo,
                         (const double*)w.Xh, (const uint16_t*)nullptr, c.ldoo, hb);
      PNO_HIP(hipGetLastError());
    } else {
      rows_bf16(nb * oo, oo, w.Xh, oo, hb, c.ldoo);
    }
    bgemm(nb * (fold ? npair : oo), vv, c.ldoo, 1.f, hb, c.TTb, 1.f, dblk, vv);
    if (fold) {
      // + the particle ladder of the pairs that keep the canonical ladder (packed results
      // of this chunk in SigPf / SigMf)
      const int64_t nrow = c.lad_nsub >= 0 ? c.lad_nsub : (int64_t)o * (o + 1) / 2;
      const int* slot = c.lad_nsub >= 0 ? c.lad_slot : (const int*)c.slot_all;
      PNO_CHECK(slot != nullptr, PNOEOM_ESTATE, "sigma: no pair table of the ladder slots");
      if (nrow > 0) {
        hipLaunchKernelGGL(ladder_unpack_add_kernel, dim3(grid1((int64_t)nb * nrow * vv)), dim3(256), 0, s, o, v,
                           nb, nrow, (const float*)w.SigPf, (const float*)w.SigMf, slot, dblk);
        PNO_HIP(hipGetLastError());
      }
    } else {
      to_double(s, nb * oovv, w.fc, Sd, 1.0);
    }
  } else if (f32x) {
    to_float(s, nb * o4, w.Xh, Xhf);
    gmbf(s, false, false, oo, vv, oo, 1.0, Xhf, oo, o4, c.T32, vv, 0, 1.0, Sd, nb, w.fc);
  } else {
    gmb(s, false, false, oo, vv, oo, 1.0, w.Xh, oo, o4, c.T, vv, 0, 1.0, Sd, vv, oovv, nb);
  }

  // ---------------------------------------------------------------- ring terms in [(i,a),(j,b)] form
  // Ziajb and Z3 enter sigma2 only as Z + Z^T (assembly below), so any term may be
  // added transposed.  With R_ia, R^s_ia, T_ia, T^s_ia and GX symmetric, the T-side
  // products T (2 D(R) - X(R)) - T^s D(R) and -T^s X(R), where D(R) = E_D - 1/2 GX R,
  // X(R) = E_X - 1/2 GX R^s, become R-side products with the T-only intermediates
  // (whose GX T parts are doubled in build_df) plus
  //   E_D^T (2T - T^s) = (1/2 M1 + B'_vo) YU   (DF rank naux)
  //   -E_X^T T, -E_X^T T^s                       (E_X = (ij|ab)' in ring order)
  // so that five (ov x ov x ov) products per vector remain.
  if (!c.ring_y) {
    gmb(s, false, true, oo, vv, naux, 1.0, w.BoopT, naux, oon, c.BvvT, naux, 0, 0.0, w.OOVVp, vv, oovv, nb);
    gmb(s, false, true, oo, vv, naux, 1.0, c.BooT, naux, 0, w.BvvpT, naux, vvn, 1.0, w.OOVVp, vv, oovv, nb);
    // E_X[(j,a),(i,b)] = (ij|ab)' = OOVVp[i][j][a][b] into the right half of the rows of RE
    Perm4 p;
    p.d[0] = o; p.d[1] = v; p.d[2] = o; p.d[3] = v;
    p.is[0] = vv; p.is[1] = v; p.is[2] = (int64_t)o * vv; p.is[3] = 1;
    p.os[0] = (int64_t)v * ov2; p.os[1] = ov2; p.os[2] = v; p.os[3] = 1;
    p.nb = nb; p.ibs = oovv; p.obs = 2 * oovv;
    permute4(s, p, 1.0, w.OOVVp, 0.0, w.RE + ov);
  }
  // The per-vector operands are stacked ([nb][ov][...] is nb*ov rows), so each product
  // with a fixed right operand is one tall GEMM.  R^s [Dr | Xr] + E_X [Tia | Tsia] is one
  // product with K = 2 ov: [R^s | E_X] (rows of RE) times [Dr | Xr] stacked on [Tia | Tsia]
  // (DXTT), filling both halves of the rows of ZZ = [Ziajb | Z3]; R_ia DX2 adds into the
  // Ziajb half.
  // With Yr / Zr the first product is R^s [Dr | Xr] alone (K = ov) and the E_X parts follow it.
  const int64_t M = (int64_t)nb * ov;
  const int64_t K1 = c.ring_y ? ov : ov2;
  // ==== ring product launches: begin
  const bool bf_ring = precision == PNOEOM_BF16 && c.ring_y && c.DXb.p;
  // BF16 scope 1, one pass: the DF-factorised ring terms join the ring products.  The left
  // half of ZZ's rows is one product with K = 2 ov + 2 naux, [-R^s | R_ia | B'_vo | M1 / 2]
  // times [Dr ; DX2 ; BYU ; YU], the right half -R^s Xr (the first ldr values of the same rows):
  // no partial result is written and read back
  uint16_t* ab1 = nullptr;
  uint16_t* ab2 = nullptr;
  const int64_t kr = c.ring_passes * c.ldr;
  if (fold) {
    // -R^s and R_ia are in RAb already (r2_layouts_kernel); the R1 part joins them
    ab1 = w.RAb;
    bf16_rows(s, M, naux, w.BvopT, naux, 1, ab1 + 2 * c.ldr, c.ldq, c.kfold);
    bf16_rows(s, M, naux, w.M1, naux, 1, ab1 + 2 * c.ldr + c.ldq, c.ldq, c.kfold, 1, 0, 0.5);
  } else if (bf_ring) {
    // the left operands R^s and R_ia as bfloat16 rows of ring_passes x ldr values, staged in fa
    ab1 = reinterpret_cast<uint16_t*>((float*)w.fa);
    ab2 = ab1 + M * kr;
    bf16_rows(s, M, ov, w.RE, ldre, 1, ab1, c.ldr, kr, c.ring_passes, 0);
    bf16_rows(s, M, ov, w.Ria, ov, 1, ab2, c.ldr, kr, c.ring_passes, 0);
  }
  hipEvent_t ring_ev = c.region_begin(3, s);
  if (fold) {
    GemmBf16Desc d;
    d.M = M; d.N = ov; d.K = c.kfold; d.alpha = 1.f; d.beta = 0.f; d.A = ab1; d.lda = c.kfold; d.B = c.RBb;
    d.ldb = c.kfold; d.C = w.fc; d.ldc = ov2; d.tag = 3;
    gemm_bf16(d, s);
    d.K = c.ldr; d.B = c.DXb + ov * kr; d.ldb = kr; d.C = w.fc + ov;
    gemm_bf16(d, s);
  } else if (bf_ring) {
    // bfloat16 MFMA with FP32 accumulation: -R^s [Dr | Xr], then + R_ia DX2 into the left half
    GemmBf16Desc d;
    d.M = M; d.N = ov2; d.K = kr; d.alpha = -1.f; d.beta = 0.f; d.A = ab1; d.lda = kr; d.B = c.DXb; d.ldb = kr;
    d.C = w.fc; d.ldc = ov2; d.tag = 3;
    gemm_bf16(d, s);
    d.N = ov; d.alpha = 1.f; d.beta = 1.f; d.A = ab2; d.B = c.DX2b;
    gemm_bf16(d, s);
  } else if (f32) {
    float* fa = w.fa;
    float* fc = w.fc;
    const int64_t nt = nb * oovv;
    GemmDesc<float> d;
    d.M = M; d.N = ov2; d.K = K1; d.alpha = -1.f; d.beta = 0.f; d.lda = ldre; d.ldb = ov2; d.C = fc; d.ldc = ov2;
    d.tag = 3;
    to_float(s, (c.ring_y ? 1 : 2) * nt, w.RE, fa);
    d.A = fa; d.B = c.DXTTf;
    gemm(d, s);
    to_float(s, nt, w.Ria, fa);
    d.N = ov; d.K = ov; d.alpha = 1.f; d.beta = 1.f; d.A = fa; d.lda = ov; d.B = c.DX2f; d.ldb = ov;
    gemm(d, s);
  } else {
    GemmDesc<double> d;
    d.M = M; d.N = ov2; d.K = K1; d.alpha = -1.0; d.beta = 0.0; d.lda = ldre; d.ldb = ov2; d.C = w.ZZ; d.ldc = ov2;
    d.tag = 3;
    d.A = w.RE; d.B = c.DXTT;
    gemm(d, s);
    d.N = ov; d.K = ov; d.alpha = 1.0; d.beta = 1.0; d.A = w.Ria; d.lda = ov; d.B = c.DX2; d.ldb = ov;
    gemm(d, s);
  }
  c.region_end(ring_ev, 3, s, 2,
               2.0 * (double)M * ov2 * K1 + 2.0 * (double)M * ov * ov + (fold ? 4.0 * (double)M * ov * naux : 0.0),
               8.0 * ((double)M * K1 + (double)K1 * ov2 + 5.0 * M * ov + (double)oovv));
  // ==== ring product launches: end
  // the DF-factorised parts of the ring terms, into the Ziajb half: (B'_vo BYU + 1/2 M1 YU), in
  // FP32 on top of the FP32 ring result when the contractions are FP32 / BF16 (then one
  // conversion of the whole ring block to FP64), else in FP64 below
  const bool df32 = f32 && c.BYUf.p && 2 * ovn <= (int64_t)w.fa.n / std::max(nb, 1);
  const bool ybf = bfr && c.ring_y && c.Yrb.p;  // R1 ring term through Yr on bfloat16 MFMA
  const bool zf32 = ybf && c.Zrf.p;             // and the one through Zr on FP32 MFMA
  // the fused mode has no FP64 ZZ: every term of the ring block and of Zp goes through FP32
  PNO_CHECK(!fold || (zf32 && c.Gqb.p && c.Fvob.p && c.Wvo2f.p && c.T32.p), PNOEOM_ESTATE,
            "sigma: BF16 operands of the fused mode missing");
  if (ybf) {
    // R1c: the block's R1 compacted as [(q,j)][c]
    Perm4 p;
    p.d[0] = nb; p.d[1] = 1; p.d[2] = 1; p.d[3] = ov;
    p.is[0] = stride1; p.is[1] = 0; p.is[2] = 0; p.is[3] = 1;
    p.os[0] = ov; p.os[1] = 0; p.os[2] = 0; p.os[3] = 1;
    permute4(s, p, 1.0, r1, 0.0, w.R1c);
  }
  if (bfr) {
    // B'_vo BYU + 1/2 M1 YU on top of the FP32 ring block (rows (q,i,a) of 2 ov in fc), unless
    // the ring products took them
    uint16_t* bv = hb;
    uint16_t* bm = hb + nb * ov * c.ldq;
    if (!fold) {
      rows_bf16(nb * ov, naux, w.BvopT, naux, bv, c.ldq);
      rows_bf16(nb * ov, naux, w.M1, naux, bm, c.ldq);
      bgemm(nb * ov, ov, c.ldq, 1.f, bv, c.BYUb, 1.f, w.fc, ov2);
      bgemm(nb * ov, ov, c.ldq, 0.5f, bm, c.YUb, 1.f, w.fc, ov2);
    }
    if (ybf) {
      uint16_t* br = bm + nb * ov * c.ldq;
      // -sum_c R1[q][j][c] Yr[(a,c)][n] for all (q,j) x (a,n) at once: the rows (q,j,a) of the
      // ring block are the rows (q,j) of a [nb o][v 2 ov] matrix
      rows_bf16(nb * o, v, w.R1c, v, br, c.ldv);
      bgemm(nb * o, v * ov2, c.ldv, -1.f, br, c.Yrb, 1.f, w.fc, v * ov2);
    }
    if (zf32) {
      // + sum_l R1[q][l][a] Zr[(j,l)][n] in FP32 on the ring block: per vector one product per j
      float* r1f = w.fa;
      to_float(s, nb * ov, w.R1c, r1f);
      for (int q = 0; q < nb; ++q) {
        GemmDesc<float> d;
        d.ta = true; d.M = v; d.N = ov2; d.K = o; d.alpha = 1.f; d.beta = 1.f;
        d.A = r1f + q * ov; d.lda = v; d.sA = 0; d.B = c.Zrf; d.ldb = ov2; d.sB = (int64_t)o * ov2;
        d.C = w.fc + (int64_t)q * ov * ov2; d.ldc = ov2; d.sC = v * ov2; d.batch = o;
        gemm(d, s);
      }
    }
    // (the fused mode keeps the ring block in FP32 for the assembly)
    if (!fold) to_double(s, 2 * (int64_t)nb * oovv, w.fc, w.ZZ, 0.0);
  } else if (f32) {
    if (df32) {
      float* fa = w.fa;
      to_float(s, nb * ovn, w.BvopT, fa);
      to_float(s, nb * ovn, w.M1, fa + nb * ovn);
      GemmDesc<float> d;
      d.M = ov; d.N = ov; d.K = naux; d.alpha = 1.f; d.beta = 1.f; d.A = fa; d.lda = naux; d.sA = ovn;
      d.B = c.BYUf; d.ldb = ov; d.sB = 0; d.C = w.fc; d.ldc = ov2; d.sC = 2 * oovv; d.batch = nb;
      gemm(d, s);
      d.alpha = 0.5f; d.A = fa + nb * ovn; d.B = c.YUf;
      gemm(d, s);
    }
    to_double(s, 2 * (int64_t)nb * oovv, w.fc, w.ZZ, 0.0);
  }
  if (!df32 && !bfr) {
    gmb(s, false, false, ov, ov, naux, 1.0, w.BvopT, naux, ovn, c.BYU, ov, 0, 1.0, w.ZZ, ov2, 2 * oovv, nb);
    gmb(s, false, false, ov, ov, naux, 0.5, w.M1, naux, ovn, c.YU, ov, 0, 1.0, w.ZZ, ov2, 2 * oovv, nb);
  }
  if (c.ring_y) {
    // E_X [T_ia | T^s_ia] = sum_c r_j^c Yr[(a,c)] - sum_l r_l^a Zr[(j,l)], with the sign of the
    // fused product: ZZ[(q,j,a)] -= sum_c R1[q][j][c] Yr[(a,c)], += sum_l R1[q][l][a] Zr[(j,l)]
    if (!ybf) {
      Perm4 p;  // R1 of the block compacted to [(q,j)][c]
      p.d[0] = nb; p.d[1] = 1; p.d[2] = 1; p.d[3] = ov;
      p.is[0] = stride1; p.is[1] = 0; p.is[2] = 0; p.is[3] = 1;
      p.os[0] = ov; p.os[1] = 0; p.os[2] = 0; p.os[3] = 1;
      permute4(s, p, 1.0, r1, 0.0, w.R1c);
      // one product per a over all vectors: [(q,j)] x [c] times Yr[(a,c)] into rows (q,j,a)
      gmb(s, false, false, (int64_t)nb * o, ov2, v, -1.0, w.R1c, v, 0, c.Yr, ov2, v * ov2, 1.0, w.ZZ, v * ov2,
          ov2, v);
    }
    // per vector, one product per j: R1[q]^T (v x o) times Zr[(j,l)] (o x 2 ov) into rows (q,j,a)
    if (!zf32)
      for (int q = 0; q < nb; ++q)
        gmb(s, true, false, v, ov2, o, 1.0, w.R1c + q * ov, v, 0, c.Zr, ov2, (int64_t)o * ov2, 1.0,
            w.ZZ + (int64_t)q * ov * ov2, ov2, v * ov2, o);
  }

  // ---------------------------------------------------------------- Fock-type terms in [i][j][a][b]
  // Ftv[q][a][b] = -sum_(i,j) sum_c U(R)[q][i][j][a][c] Gq[(i,j,c)][b]: per vector one product
  // summed over the o^2 pair blocks (v x v times v x v), rows of U(R) read in place
  if (bfr && c.Gqb.p) {
    // BF16 scope 1: one bfloat16 product per vector, U(R) rows as [a][(k,l,d)] staged in fa
    // (written by the layout pass in the fused mode)
    uint16_t* ub = urb ? urb : reinterpret_cast<uint16_t*>((float*)w.fa);
    if (!urb) {
      hipLaunchKernelGGL(pair_rows_bf16_kernel, dim3(grid1(nb * v * c.ldg)), dim3(256), 0, s, (int64_t)nb, oo,
                         (int64_t)v, (const double*)w.UR, ub, c.ldg);
      PNO_HIP(hipGetLastError());
    }
    float* ftv32 = fold ? (float*)w.fz : (float*)w.fc;  // (fc holds the FP32 ring block in the fused mode)
    for (int q = 0; q < nb; ++q)
      bgemm(v, v, c.ldg, -1.f, ub + q * v * c.ldg, c.Gqb, 0.f, ftv32 + q * vv, v);
    to_double(s, nb * vv, ftv32, w.Ftv, 0.0);
  } else {
    for (int q = 0; q < nb; ++q)
      gmb(s, false, false, v, v, v, -1.0, w.UR + q * oovv, v, vv, c.Gq, v, vv, 0.0, w.Ftv + q * vv, v, 0, oo,
          true);
  }
  axpby(s, nb * vv, 1.0, w.fp_vv, 1.0, w.Ftv);
  // Fto[q][k][j] = sum_x g2[k][x] U(R)[q][j][x]: one product over the rows (q, j) of U(R) into
  // [q][j][k] (in O4p, free by now), then transposed per vector
  gm(s, false, true, nbo, o, ov * v, 1.0, w.UR, ov * v, c.g2, ov * v, 0.0, w.O4p, o);
  ext(s, nb, o, o, 1, oo, 1, o, 0, w.O4p, w.Fto);
  axpby(s, nb * oo, 1.0, w.fp_oo, 1.0, w.Fto);
  // Zp[q][i][j][a][b] = sum_c R_ij^ac Fvv[b][c] - sum_k Foo[k][j] R_ik^ab + sum_c T_ij^ac Ftv[b][c]
  //                   - sum_k Fto[k][j] T_ik^ab - sum_k r_k^a Wvo2[(i,j,b)][k]
  // (the last one is -P[ sum_k r_k^a Wvo_kbij ] before the P symmetrisation of the assembly)
  if (bfr && c.Fvob.p && c.Wvo2f.p && c.T32.p) {
    // BF16 scope 1: R (Fvv - diag)^T and T Ftv^T on bfloat16 MFMA, the products with K = o
    // (Fto T, r1 Wvo2) on FP32 MFMA, all into one FP32 sum (operands staged in fa); the
    // diagonal parts of R Fvv^T and of -Foo^T R are added exactly by zp_finish_kernel (by the
    // assembly in the fused mode), the off-diagonal part of -Foo^T R rides with the hole
    // ladder (Whb)
    float* fof = w.fa;
    float* r1f = fof + nb * oo;
    const int64_t boff = (nb * (oo + ov) + 3) / 4 * 4;  // floats: bfloat16 rows 16-byte aligned
    uint16_t* r2b = reinterpret_cast<uint16_t*>((float*)w.fa + boff);
    uint16_t* ftb = r2b + nb * oo * v * c.ldv;
    to_float(s, nb * oo, w.Fto, fof);
    for (int q = 0; q < nb; ++q) to_float(s, ov, r1 + q * stride1, r1f + q * ov);
    rows_bf16(nb * oo * v, v, R2, v, r2b, c.ldv);
    rows_bf16(nb * v, v, w.Ftv, v, ftb, c.ldv);
    // (FP32 sum in fz in the fused mode, where it goes to the assembly as it is; else in fc)
    float* zf = fold ? (float*)w.fz : (float*)w.fc;
    bgemm(nb * oo * v, v, c.ldv, 1.f, r2b, c.Fvob, 0.f, zf, v);
    for (int q = 0; q < nb; ++q) bgemm(oo * v, v, c.ldv, 1.f, c.Tvb, ftb + q * v * c.ldv, 1.f, zf + q * oovv, v);
    // (- Foo^T R: its off-diagonal part went with the hole ladder (Whb), its diagonal part is
    // added exactly below)
    for (int q = 0; q < nb; ++q) {
      GemmDesc<float> f;  // - Fto[q]^T T, batched over i
      f.ta = true; f.M = o; f.N = vv; f.K = o; f.alpha = -1.f; f.beta = 1.f; f.A = fof + q * oo; f.lda = o;
      f.sA = 0; f.B = c.T32; f.ldb = vv; f.sB = o * vv; f.C = zf + q * oovv; f.ldc = vv; f.sC = o * vv;
      f.batch = o;
      gemm(f, s);
      GemmDesc<float> g;  // - r1[q]^T Wvo2_ij^T, batched over the pairs
      g.ta = true; g.tb = true; g.M = v; g.N = v; g.K = o; g.alpha = -1.f; g.beta = 1.f; g.A = r1f + q * ov;
      g.lda = v; g.sA = 0; g.B = c.Wvo2f; g.ldb = o; g.sB = (int64_t)v * o; g.C = zf + q * oovv; g.ldc = v;
      g.sC = vv; g.batch = oo;
      gemm(g, s);
    }
    // (the fused mode's assembly adds the orbital-energy terms itself)
    if (!fold) {
      hipLaunchKernelGGL(zp_finish_kernel, dim3(grid1(nb * oovv)), dim3(256), 0, s, nb * oovv, (int64_t)o,
                         (int64_t)v, zf, R2, (const double*)c.Fvvd, (const double*)c.Food);
      PNO_HIP(hipGetLastError());
      to_double(s, nb * oovv, zf, w.Zp, 0.0);
    }
  } else {
    gm(s, false, true, (int64_t)nb * oo * v, v, v, 1.0, R2, v, c.Fvv, v, 0.0, w.Zp, v);
    gmb(s, false, true, oo * v, v, v, 1.0, c.T, v, 0, w.Ftv, v, vv, 1.0, w.Zp, v, oovv, nb);
    gmb(s, true, false, o, vv, o, -1.0, c.Foo, o, 0, R2, vv, o * vv, 1.0, w.Zp, vv, o * vv, nbo);
    for (int q = 0; q < nb; ++q)
      gmb(s, true, false, o, vv, o, -1.0, w.Fto + q * oo, o, 0, c.T, vv, o * vv, 1.0, w.Zp + q * oovv, vv, o * vv,
          o);
    for (int q = 0; q < nb; ++q)
      gmb(s, true, true, v, v, o, -1.0, r1 + q * stride1, v, 0, c.Wvo2, o, (int64_t)v * o, 1.0, w.Zp + q * oovv, v,
          vv, oo);
  }

  {
    const unsigned ntb = (unsigned)((v + kAsmTile - 1) / kAsmTile);
    PNO_CHECK((int64_t)o * o <= 65535 && nb <= 65535, PNOEOM_EINVAL, "sigma: too many pairs or vectors per block");
    if (fold)
      hipLaunchKernelGGL(assemble_s2_sym_kernel, dim3(ntb * ntb, (unsigned)(o * (o + 1) / 2), (unsigned)nb), dim3(256),
                         0, s, o, v, (const float*)w.Sdf, (const float*)w.fz, (const float*)w.fc, R2,
                         (const double*)c.Fvvd, (const double*)c.Food, s2, stride2);
    else
      hipLaunchKernelGGL((assemble_s2_tiled_kernel<double, double>), dim3(ntb * ntb, (unsigned)(o * o), (unsigned)nb),
                         dim3(256), 0, s, o, v, (const double*)Sd, (const double*)w.Zp, (const double*)w.ZZ, s2,
                         stride2);
    PNO_HIP(hipGetLastError());
  }
}
}  // namespace

namespace {
// the ladder can run in this precision: FP64 always; FP32 / BF16 only in the precision of the build
void ladder_check(const Context& c, int precision) {
  PNO_CHECK(precision == PNOEOM_FP64 || precision == PNOEOM_FP32 || precision == PNOEOM_BF16, PNOEOM_EINVAL,
            "ladder: precision must be FP64, FP32 or BF16");
  const bool f32 = precision == PNOEOM_FP32, bf = precision == PNOEOM_BF16;
  const bool ok = c.lad_streamed ? (f32 ? c.BvvTf.p != nullptr : bf ? c.BvvTb.p != nullptr : c.BvvT.p != nullptr)
                                 : (f32 ? c.Wpf.p != nullptr : bf ? c.Wpb.p != nullptr : c.Wp.p != nullptr);
  PNO_CHECK(ok, PNOEOM_EINVAL, "ladder: the contraction precision must match the one given to build_df");
}

// sigma+/- of `rows` packed rows of the work arrays (Sp/Am, Spf/Amf or Spb/Amb -> SigP/SigM or
// SigPf/SigMf): the cached W+/- in one GEMM each, or the streamed slabs
void ladder_contract(Context& c, int precision, int64_t rows) {
  SigmaWork& w = c.sw;
  hipStream_t s = c.stream;
  const int64_t v = c.v, vp = v * (v + 1) / 2, vm = v * (v - 1) / 2;
  const bool f32 = precision == PNOEOM_FP32, bf = precision == PNOEOM_BF16;
  if (c.lad_streamed) {
    if (f32)
      ladder_streamed(c, precision, rows, w.Spf, vp, w.Amf, vm, w.SigPf, w.SigMf);
    else if (bf)
      ladder_streamed(c, precision, rows, w.Spb, c.ldpb, w.Amb, c.ldmb, w.SigPf, w.SigMf);
    else
      ladder_streamed(c, precision, rows, w.Sp, vp, w.Am, vm, w.SigP, w.SigM);
    return;
  }
  hipEvent_t lad0 = nullptr, lad1 = nullptr;
  if (c.timing) {
    lad0 = c.next_event();
    lad1 = c.next_event();
    c.ev_prec.push_back(precision);
    PNO_HIP(hipEventRecord(lad0, s));
  }
  if (f32) {
    GemmDesc<float> d;
    d.tb = true; d.M = rows; d.N = vp; d.K = vp; d.tag = 1;
    d.A = w.Spf; d.lda = vp; d.B = c.Wpf; d.ldb = vp; d.C = w.SigPf; d.ldc = vp;
    gemm(d, s);
    d.N = vm; d.K = vm; d.A = w.Amf; d.lda = vm; d.B = c.Wmf; d.ldb = vm; d.C = w.SigMf; d.ldc = vm;
    gemm(d, s);
  } else if (bf) {
    GemmBf16Desc d;
    d.M = rows; d.N = vp; d.K = c.ldpb; d.tag = 1;
    d.A = w.Spb; d.lda = c.ldpb; d.B = c.Wpb; d.ldb = c.ldpb; d.C = w.SigPf; d.ldc = vp;
    gemm_bf16(d, s);
    d.N = vm; d.K = c.ldmb; d.A = w.Amb; d.lda = c.ldmb; d.B = c.Wmb; d.ldb = c.ldmb; d.C = w.SigMf; d.ldc = vm;
    gemm_bf16(d, s);
  } else {
    GemmDesc<double> d;
    d.tb = true; d.M = rows; d.N = vp; d.K = vp; d.tag = 1;
    d.A = w.Sp; d.lda = vp; d.B = c.Wp; d.ldb = vp; d.C = w.SigP; d.ldc = vp;
    gemm(d, s);
    d.N = vm; d.K = vm; d.A = w.Am; d.lda = vm; d.B = c.Wm; d.ldb = vm; d.C = w.SigM; d.ldc = vm;
    gemm(d, s);
  }
  if (c.timing) {
    PNO_HIP(hipEventRecord(lad1, s));
    const double fl = 2.0 * (double)rows * ((double)vp * vp + (double)vm * vm);
    const int nl = vm > 0 ? 2 : 1;
    c.ladder_flops += fl;
    c.ladder_kernel_launches += nl;
    c.ladder_flops_p[precision] += fl;
    c.ladder_launches_p[precision] += nl;
  }
}

// packs nvec vectors (pairs of o occupied) into the ladder work arrays of a precision; with
// prow, only the pairs with a slot (nrow slots per vector), else all o(o+1)/2 pairs
void ladder_pack(Context& c, int precision, int o, int nvec, const double* r2, int64_t stride2,
                 const int* prow = nullptr, int64_t nrow = -1, const int* slot = nullptr) {
  SigmaWork& w = c.sw;
  hipStream_t s = c.stream;
  const int64_t v = c.v, vp = v * (v + 1) / 2, vm = v * (v - 1) / 2, vm1 = std::max<int64_t>(vm, 1);
  if (!prow) nrow = (int64_t)o * (o + 1) / 2;
  const int64_t rows = std::max<int64_t>((int64_t)nvec * nrow, 1);
  const int64_t tot = (int64_t)nvec * o * o * v * v;
  const bool f32 = precision == PNOEOM_FP32, bf = precision == PNOEOM_BF16;
  // (the other precisions' operands are released: the chunk size counts them as free)
  if (!f32) {
    w.Spf.release();
    w.Amf.release();
  }
  if (!bf) {
    w.Spb.release();
    w.Amb.release();
  }
  if (f32 || bf) {
    w.Sp.release();
    w.Am.release();
    w.SigP.release();
    w.SigM.release();
    grow(w.SigPf, rows * vp); grow(w.SigMf, rows * vm1);
  } else {
    w.SigPf.release();
    w.SigMf.release();
    grow(w.SigP, rows * vp); grow(w.SigM, rows * vm1);
  }
  if (f32) {
    grow(w.Spf, rows * vp); grow(w.Amf, rows * vm1);
    hipLaunchKernelGGL((ladder_pack_kernel<float>), dim3(grid1(tot)), dim3(256), 0, s, o, (int)v, nvec, r2, stride2,
                       (float*)w.Spf, vp, (float*)w.Amf, vm, prow, nrow);
  } else if (bf) {
    // padded rows; the padding columns are zeroed once per allocation and never written
    if ((int64_t)w.Spb.n < rows * c.ldpb || (int64_t)w.Amb.n < rows * c.ldmb) {
      w.Spb.alloc(rows * c.ldpb);
      w.Amb.alloc(rows * c.ldmb);
      hipLaunchKernelGGL(zero_u16_kernel, dim3(grid1((int64_t)w.Spb.n)), dim3(256), 0, s, (int64_t)w.Spb.n,
                         (uint16_t*)w.Spb);
      hipLaunchKernelGGL(zero_u16_kernel, dim3(grid1((int64_t)w.Amb.n)), dim3(256), 0, s, (int64_t)w.Amb.n,
                         (uint16_t*)w.Amb);
      PNO_HIP(hipGetLastError());
    }
    if (slot)  // (only the listed pairs' blocks of R are read)
      hipLaunchKernelGGL((ladder_pack_slots_kernel<uint16_t>), dim3(grid1((int64_t)nvec * nrow * v * v)), dim3(256), 0,
                         s, o, (int)v, nvec, r2, stride2, (uint16_t*)w.Spb, c.ldpb, (uint16_t*)w.Amb, c.ldmb, slot,
                         nrow);
    else
      hipLaunchKernelGGL((ladder_pack_kernel<uint16_t>), dim3(grid1(tot)), dim3(256), 0, s, o, (int)v, nvec, r2,
                         stride2, (uint16_t*)w.Spb, c.ldpb, (uint16_t*)w.Amb, c.ldmb, prow, nrow);
  } else {
    grow(w.Sp, rows * vp); grow(w.Am, rows * vm1);
    hipLaunchKernelGGL((ladder_pack_kernel<double>), dim3(grid1(tot)), dim3(256), 0, s, o, (int)v, nvec, r2,
                       stride2, (double*)w.Sp, vp, (double*)w.Am, vm, prow, nrow);
  }
  PNO_HIP(hipGetLastError());
}

// unpacks the ladder result of nvec vectors into full [q][i][j][a][b] arrays (stride per vector)
void ladder_unpack(Context& c, int precision, int o, int nvec, double* out, int64_t stride,
                   const int* prow = nullptr, int64_t nrow = -1) {
  SigmaWork& w = c.sw;
  const int64_t v = c.v, tot = (int64_t)nvec * o * o * v * v;
  if (!prow) nrow = (int64_t)o * (o + 1) / 2;
  if (precision != PNOEOM_FP64)
    hipLaunchKernelGGL((ladder_unpack_kernel<float>), dim3(grid1(tot)), dim3(256), 0, c.stream, o, (int)v, nvec,
                       (const float*)w.SigPf, (const float*)w.SigMf, out, stride, prow, nrow);
  else
    hipLaunchKernelGGL((ladder_unpack_kernel<double>), dim3(grid1(tot)), dim3(256), 0, c.stream, o, (int)v, nvec,
                       (const double*)w.SigP, (const double*)w.SigM, out, stride, prow, nrow);
  PNO_HIP(hipGetLastError());
}
}  // namespace

void ladder_apply(Context& c, int nmat, const double* X, double* Y, int precision) {
  PNO_CHECK(c.have_lad, PNOEOM_ESTATE, "ladder_apply before build_df or build_ladder");
  PNO_CHECK(nmat >= 0, PNOEOM_EINVAL, "ladder_apply: nmat < 0");
  ladder_check(c, precision);
  if (nmat == 0) return;
  PNO_CHECK(X && Y, PNOEOM_EINVAL, "ladder_apply: null matrix pointer");
  const int64_t vv = (int64_t)c.v * c.v;
  // each matrix is the doubles block of one pair: the packing of a single occupied index
  ladder_pack(c, precision, 1, nmat, X, vv);
  ladder_contract(c, precision, nmat);
  ladder_unpack(c, precision, 1, nmat, Y, vv);
}

// ---------------------------------------------------------------- allocation-free ladder
// Staging of ladder_apply_noalloc (packed S/A rows and the sigma+/- rows of one call) in a
// file-scope device array: each GPU the library runs on holds its own copy until the
// process ends.  Host code never passes the array's name to a kernel (on the host it is
// only a stand-in for the symbol); it resolves the device address once per device with
// hipGetSymbolAddress and uses that.
namespace {
__device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex& scratch_mu() {
  static std::mutex m;
  return m;
}
unsigned char* scratch_dev[kMaxDevices] = {};

// device address of this GPU's copy of the scratch array (resolved at the first call on it)
unsigned char* scratch_address() {
  int dev = -1;
  PNO_HIP(hipGetDevice(&dev));
  PNO_CHECK(dev >= 0 && dev < kMaxDevices, PNOEOM_EINVAL, "ladder_apply_noalloc: device index out of range");
  std::lock_guard<std::mutex> lock(scratch_mu());
  if (!scratch_dev[dev]) {
    void* p = nullptr;
    PNO_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    PNO_CHECK(p != nullptr, PNOEOM_EHIP, "ladder_apply_noalloc: no device address for the scratch array");
    scratch_dev[dev] = static_cast<unsigned char*>(p);
  }
  return scratch_dev[dev];
}

int64_t align256(int64_t b) { return (b + 255) / 256 * 256; }
}  // namespace

int64_t ladder_noalloc_bytes(const Context& c, int nmat, int precision) {
  const int64_t v = c.v, vp = v * (v + 1) / 2, vm1 = std::max<int64_t>(v * (v - 1) / 2, 1);
  const bool bf = precision == PNOEOM_BF16;
  const int64_t in = precision == PNOEOM_FP64 ? 8 : precision == PNOEOM_FP32 ? 4 : 2;
  const int64_t out = precision == PNOEOM_FP64 ? 8 : 4;
  const int64_t lds = bf ? c.ldpb : vp, lda = bf ? c.ldmb : vm1;
  return align256(nmat * lds * in) + align256(nmat * lda * in) + align256(nmat * vp * out) +
         align256(nmat * vm1 * out);
}

void ladder_apply_noalloc(Context& c, int nmat, const double* X, double* Y, int precision) {
  PNO_CHECK(c.have_lad, PNOEOM_ESTATE, "ladder_apply_noalloc before build_df or build_ladder");
  PNO_CHECK(nmat >= 0, PNOEOM_EINVAL, "ladder_apply_noalloc: nmat < 0");
  ladder_check(c, precision);
  PNO_CHECK(!c.lad_streamed, PNOEOM_EINVAL,
            "ladder_apply_noalloc: needs the cached W+/- (the streamed ladder needs its slab workspace)");
  if (nmat == 0) return;
  PNO_CHECK(X && Y, PNOEOM_EINVAL, "ladder_apply_noalloc: null matrix pointer");
  const int64_t need = ladder_noalloc_bytes(c, nmat, precision);
  PNO_CHECK(need <= kNoAllocScratchBytes, PNOEOM_EINVAL,
            "ladder_apply_noalloc: nmat v^2 too large for the scratch array (" + std::to_string(need) + " > " +
                std::to_string(kNoAllocScratchBytes) + " bytes)");
  hipStream_t s = c.stream;
  const int64_t v = c.v, vp = v * (v + 1) / 2, vm = v * (v - 1) / 2, vm1 = std::max<int64_t>(vm, 1);
  const int64_t tot = (int64_t)nmat * v * v;
  const bool f32 = precision == PNOEOM_FP32, bf = precision == PNOEOM_BF16;
  const int64_t in = precision == PNOEOM_FP64 ? 8 : f32 ? 4 : 2, out = precision == PNOEOM_FP64 ? 8 : 4;
  const int64_t lds = bf ? c.ldpb : vp, lda = bf ? c.ldmb : vm1;
  unsigned char* p = scratch_address();
  unsigned char* Sb = p;
  unsigned char* Ab = Sb + align256(nmat * lds * in);
  unsigned char* Pb = Ab + align256(nmat * lda * in);
  unsigned char* Mb = Pb + align256(nmat * vp * out);
  // each matrix is the doubles block of one pair: the packing of a single occupied index
  if (f32) {
    hipLaunchKernelGGL((ladder_pack_kernel<float>), dim3(grid1(tot)), dim3(256), 0, s, 1, (int)v, nmat, X, v * v,
                       (float*)Sb, vp, (float*)Ab, vm, (const int*)nullptr, (int64_t)1);
    GemmDesc<float> d;
    d.tb = true; d.M = nmat; d.N = vp; d.K = vp; d.tag = 1; d.no_split = true;
    d.A = (const float*)Sb; d.lda = vp; d.B = c.Wpf; d.ldb = vp; d.C = (float*)Pb; d.ldc = vp;
    gemm(d, s);
    d.N = vm; d.K = vm; d.A = (const float*)Ab; d.lda = vm; d.B = c.Wmf; d.ldb = vm; d.C = (float*)Mb; d.ldc = vm;
    gemm(d, s);
  } else if (bf) {
    // the padding columns of the packed rows must be zero; the array keeps what the last
    // call on this GPU left, so the whole staging of this call is cleared first
    hipLaunchKernelGGL(zero_u16_kernel, dim3(grid1(nmat * lds)), dim3(256), 0, s, nmat * lds, (uint16_t*)Sb);
    hipLaunchKernelGGL(zero_u16_kernel, dim3(grid1(nmat * lda)), dim3(256), 0, s, nmat * lda, (uint16_t*)Ab);
    hipLaunchKernelGGL((ladder_pack_kernel<uint16_t>), dim3(grid1(tot)), dim3(256), 0, s, 1, (int)v, nmat, X,
                       v * v, (uint16_t*)Sb, lds, (uint16_t*)Ab, lda, (const int*)nullptr, (int64_t)1);
    GemmBf16Desc d;
    d.M = nmat; d.N = vp; d.K = c.ldpb; d.tag = 1; d.no_split = true;
    d.A = (const uint16_t*)Sb; d.lda = c.ldpb; d.B = c.Wpb; d.ldb = c.ldpb; d.C = (float*)Pb; d.ldc = vp;
    gemm_bf16(d, s);
    d.N = vm; d.K = c.ldmb; d.A = (const uint16_t*)Ab; d.lda = c.ldmb; d.B = c.Wmb; d.ldb = c.ldmb;
    d.C = (float*)Mb; d.ldc = vm;
    gemm_bf16(d, s);
  } else {
    hipLaunchKernelGGL((ladder_pack_kernel<double>), dim3(grid1(tot)), dim3(256), 0, s, 1, (int)v, nmat, X, v * v,
                       (double*)Sb, vp, (double*)Ab, vm, (const int*)nullptr, (int64_t)1);
    GemmDesc<double> d;
    d.tb = true; d.M = nmat; d.N = vp; d.K = vp; d.tag = 1; d.no_split = true;
    d.A = (const double*)Sb; d.lda = vp; d.B = c.Wp; d.ldb = vp; d.C = (double*)Pb; d.ldc = vp;
    gemm(d, s);
    d.N = vm; d.K = vm; d.A = (const double*)Ab; d.lda = vm; d.B = c.Wm; d.ldb = vm; d.C = (double*)Mb; d.ldc = vm;
    gemm(d, s);
  }
  PNO_HIP(hipGetLastError());
  if (precision != PNOEOM_FP64)
    hipLaunchKernelGGL((ladder_unpack_kernel<float>), dim3(grid1(tot)), dim3(256), 0, s, 1, (int)v, nmat,
                       (const float*)Pb, (const float*)Mb, Y, v * v, (const int*)nullptr, (int64_t)1);
  else
    hipLaunchKernelGGL((ladder_unpack_kernel<double>), dim3(grid1(tot)), dim3(256), 0, s, 1, (int)v, nmat,
                       (const double*)Pb, (const double*)Mb, Y, v * v, (const int*)nullptr, (int64_t)1);
  PNO_HIP(hipGetLastError());
}

namespace {
// one chunk of trial vectors: all of them go through the ladder and the rest together
void sigma_block_chunk(Context& c, int nvec, const double* r1, const double* r2, double* s1, double* s2,
                       int64_t stride1, int64_t stride2, int precision) {
  PNO_CHECK(c.have_df, PNOEOM_ESTATE, "sigma before build_df");
  PNO_CHECK(precision == PNOEOM_FP64 || precision == PNOEOM_FP32 || precision == PNOEOM_BF16, PNOEOM_EINVAL,
            "sigma: precision must be FP64, FP32 or BF16");
  ladder_check(c, precision);
  if (nvec <= 0) return;
  SigmaWork& w = c.sw;
  const int o = c.o;
  const int64_t oovv = c.oovv();
  // all pairs, or (PNO space with native pairs) the pairs that keep the canonical ladder
  const int* prow = c.lad_nsub >= 0 ? c.lad_prow : nullptr;
  const int64_t nrow = c.lad_nsub >= 0 ? c.lad_nsub : (int64_t)o * (o + 1) / 2;
  const int64_t rows = (int64_t)nvec * nrow;
  // (the fused BF16 ring mode adds the packed ladder results into its FP32 direct block inside
  // sigma_rest_block: no FP64 unpacked ladder)
  const bool defer = ring_fold(c, precision);
  trim_sigma_work(c, precision, stride2 != oovv);
  if (c.lad_nsub < 0 && (int64_t)c.slot_all.n < nrow) {
    std::vector<int> all;
    for (int i = 0; i < o; ++i)
      for (int j = i; j < o; ++j) all.push_back(i * o + j);
    c.slot_all.alloc((int64_t)all.size());
    PNO_HIP(hipMemcpy(c.slot_all, all.data(), all.size() * sizeof(int), hipMemcpyHostToDevice));
  }
  const int* slot = c.lad_nsub >= 0 ? c.lad_slot : (const int*)c.slot_all;
  if (defer)
    w.LadAll.release();
  else
    grow(w.LadAll, (int64_t)nvec * oovv);
  // ---------------------------------------------------------------- particle ladder, all vectors at once
  ladder_pack(c, precision, o, nvec, r2, stride2, prow, nrow, slot);
  ladder_contract(c, precision, rows);
  if (!defer) ladder_unpack(c, precision, o, nvec, w.LadAll, oovv, prow, nrow);
  // ---------------------------------------------------------------- everything else
  sigma_rest_block(c, nvec, r1, stride1, r2, stride2, s1, s2, precision, defer ? nullptr : (double*)w.LadAll);
}
}  // namespace

void sigma_block(Context& c, int nvec, const double* r1, const double* r2, double* s1, double* s2, int64_t stride1,
                 int64_t stride2, int precision) {
  TraceRange tr_("sigma block");
  PNO_CHECK(c.have_df, PNOEOM_ESTATE, "sigma before build_df");
  if (nvec <= 0) return;
  const int nb = sigma_chunk(c, nvec, precision, false);
  for (int q0 = 0; q0 < nvec; q0 += nb) {
    const int n = std::min(nb, nvec - q0);
    sigma_block_chunk(c, n, r1 + q0 * stride1, r2 + q0 * stride2, s1 + q0 * stride1, s2 + q0 * stride2, stride1,
                      stride2, precision);
  }
}


namespace {
// every device address the sigma path may touch besides the context's fixed
// intermediates (those change only in build_df / build_sapno, which drop the graphs)
uint64_t sigma_signature(Context& c, hipStream_t s) {
  uint64_t h = 1469598103934665603ull;
  auto mix = [&](const void* p, size_t n) {
    h ^= (uint64_t)(uintptr_t)p + 0x9e3779b97f4a7c15ull + (h << 6) + (h >> 2);
    h ^= (uint64_t)n * 0x100000001b3ull;
  };
  SigmaWork& w = c.sw;
  for (DBuf<double>* b : {&w.Bp, &w.Bc, &w.hp, &w.Jp, &w.Kp, &w.fp, &w.dp, &w.fp_ov, &w.fp_vv, &w.fp_oo, &w.BvopT, &w.BoopT,
                          &w.BvvpT, &w.R2c, &w.Ria, &w.UiaR, &w.S1p, &w.UR, &w.ZZ,
                          &w.RE, &w.Zp, &w.Xh, &w.O4p, &w.OOVVp, &w.M1, &w.R1c, &w.Ftv, &w.Fto, &w.LadAll, &w.Sp,
                          &w.Am, &w.SigP, &w.SigM, &c.pno.Tw, &c.pno.r1, &c.pno.r2, &c.pno.s1, &c.pno.s2, &c.gin,
                          &c.gout})
    mix(b->p, b->n);
  for (DBuf<float>* b : {&w.Spf, &w.Amf, &w.SigPf, &w.SigMf, &w.fa, &w.fc, &w.fz, &w.Sdf}) mix(b->p, b->n);
  mix(w.Spb.p, w.Spb.n);
  mix(w.RAb.p, w.RAb.n);
  mix(w.Amb.p, w.Amb.n);
  mix((const void*)(uintptr_t)gemm_workspace_signature(s), 0);
  return h;
}

void sigma_packed(Context& c, int space, int nv, const double* X, double* S, int64_t N, int precision) {
  if (space == PNOEOM_CANONICAL) {
    const int64_t ov = c.ov();
    sigma_block(c, nv, X, X + ov, S, S + ov, N, N, precision);
  } else {
    sigma_pno(c, nv, X, S, precision);
  }
}
}  // namespace

void sigma_apply(Context& c, int space, int nv, const double* X, double* S, int64_t N, int precision) {
  if (nv <= 0) return;
  if (!c.graph_mode) {
    sigma_packed(c, space, nv, X, S, N, precision);
    return;
  }
  hipStream_t s = c.stream;
  if (!c.gstream) {
    PNO_HIP(hipStreamCreateWithFlags(&c.gstream, hipStreamNonBlocking));
    PNO_HIP(hipEventCreateWithFlags(&c.gev[0], hipEventDisableTiming));
    PNO_HIP(hipEventCreateWithFlags(&c.gev[1], hipEventDisableTiming));
  }
  const int64_t need = (int64_t)nv * N;
  if ((int64_t)c.gin.n < need || (int64_t)c.gout.n < need) {  // new staging addresses: recapture all
    c.drop_graphs();
    c.gin.alloc(need);
    c.gout.alloc(need);
  }
  PNO_HIP(hipMemcpyAsync(c.gin, X, need * sizeof(double), hipMemcpyDeviceToDevice, s));
  Context::SigmaGraph* hit = nullptr;
  for (Context::SigmaGraph& g : c.graphs)
    if (g.nv == nv && g.prec == precision && g.space == space && g.N == N) hit = &g;
  if (hit && hit->sig == sigma_signature(c, c.gstream) && hit->sig != 0) {
    // replay on the graph stream, ordered after and before the context stream's work
    PNO_HIP(hipEventRecord(c.gev[0], s));
    PNO_HIP(hipStreamWaitEvent(c.gstream, c.gev[0], 0));
    PNO_HIP(hipGraphLaunch(hit->exec, c.gstream));
    PNO_HIP(hipEventRecord(c.gev[1], c.gstream));
    PNO_HIP(hipStreamWaitEvent(s, c.gev[1], 0));
    ++c.graph_launches;
  } else {
    if (hit) {  // a buffer moved since the capture
      (void)hipGraphExecDestroy(hit->exec);
      c.graphs.erase(c.graphs.begin() + (hit - c.graphs.data()));
    }
    // eager evaluation on the graph stream (its result is this call's answer and it
    // sizes every workspace), then the same calls, with the same chunking, captured
    // into a graph
    PNO_HIP(hipEventRecord(c.gev[0], s));
    PNO_HIP(hipStreamWaitEvent(c.gstream, c.gev[0], 0));
    c.stream = c.gstream;
    try {
      c.fixed_chunk = sigma_chunk(c, nv, precision, space == PNOEOM_PNO);
      sigma_packed(c, space, nv, c.gin, c.gout, N, precision);
      PNO_HIP(hipStreamSynchronize(c.gstream));
    } catch (...) {
      c.stream = s;
      c.fixed_chunk = 0;
      throw;
    }
    const uint64_t sig = sigma_signature(c, c.gstream);
    const bool saved_timing = c.timing;
    c.timing = false;
    hipGraph_t graph = nullptr;
    bool ok = hipStreamBeginCapture(c.gstream, hipStreamCaptureModeThreadLocal) == hipSuccess;
    hipError_t ec = hipErrorUnknown;
    if (ok) {
      try {
        sigma_packed(c, space, nv, c.gin, c.gout, N, precision);
      } catch (...) {
        ok = false;
      }
      ec = hipStreamEndCapture(c.gstream, &graph);
    }
    c.stream = s;
    c.timing = saved_timing;
    c.fixed_chunk = 0;
    (void)hipGetLastError();
    if (ok && ec == hipSuccess && graph && sigma_signature(c, c.gstream) == sig) {
      Context::SigmaGraph g;
      g.nv = nv; g.prec = precision; g.space = space; g.N = N; g.sig = sig;
      if (hipGraphInstantiate(&g.exec, graph, nullptr, nullptr, 0) == hipSuccess) {
        c.graphs.push_back(g);
        ++c.graph_captures;
      } else {
        (void)hipGetLastError();
      }
    }
    if (graph) (void)hipGraphDestroy(graph);
    PNO_HIP(hipEventRecord(c.gev[1], c.gstream));
    PNO_HIP(hipStreamWaitEvent(s, c.gev[1], 0));
  }
  PNO_HIP(hipMemcpyAsync(S, c.gout, need * sizeof(double), hipMemcpyDeviceToDevice, s));
}

void sigma_canonical(Context& c, const double* r1, const double* r2, double* s1, double* s2, int precision) {
  sigma_block(c, 1, r1, r2, s1, s2, c.ov(), c.oovv(), precision);
}

}  // namespace pnoeom
