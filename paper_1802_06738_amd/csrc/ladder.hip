// Streamed particle-particle ladder: sum_cd W_abcd X_cd with W never stored whole.
//
// W_abcd = sum_Q B~^Q_ac B~^Q_bd (the T1-dressed (ac|bd) of the H-bar definition,
// Methods) is the largest intermediate of the method; packed into its symmetric and
// antisymmetric halves W+/- it takes v^4/2 words (v = 900: 1.3 TB in FP64), more than
// one GPU holds.  Here the rows (a <= b) of W+/- are rebuilt inside every sigma, one
// slab of a-values at a time, and contracted at once with all trial vectors:
//
//   tmp[a-a0][c][b-a0][d] = sum_Q B~^Q_ac B~^Q_bd     for a in the slab, b >= a0  (MFMA GEMM)
//   W+[(a<=b),(c<=d)], W-[(a<b),(c<d)]  of the slab  <- tmp                 (LDS-tiled pack)
//   sigma+[:, slab rows] = S W+_slab^T,  sigma-[:, slab rows] = A W-_slab^T (MFMA GEMMs)
//
// S / A are the packed symmetric / antisymmetric parts of the trial vectors, so the
// result equals the contraction with the cached W+/-.  The slab size follows the
// workspace allocated by prepare_streamed_ladder: at a0 the slab holds na a-values
// with na * (v - a0) <= na0 * v, so both the tmp block and the W rows stay within it.
#include <algorithm>

#include "context.h"

namespace pnoeom {
namespace {

unsigned grid_of(int64_t n) {
  int64_t b = (n + 255) / 256;
  if (b > 65536) b = 65536;
  if (b < 1) b = 1;
  return (unsigned)b;
}

__host__ __device__ __forceinline__ int64_t tri_ix(int64_t c, int64_t d, int64_t v) {  // c <= d
  return c * v - c * (c - 1) / 2 + (d - c);
}
__host__ __device__ __forceinline__ int64_t stri_ix(int64_t c, int64_t d, int64_t v) {  // c < d
  return c * (v - 1) - c * (c - 1) / 2 + (d - c - 1);
}

template <typename T>
__device__ __forceinline__ T store_as(float x);
template <>
__device__ __forceinline__ float store_as<float>(float x) {
  return x;
}
template <>
__device__ __forceinline__ uint16_t store_as<uint16_t>(float x) {  // bfloat16, round to nearest even
  uint32_t u = __float_as_uint(x);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40u);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
template <typename T>
__device__ __forceinline__ T store_as(double x);
template <>
__device__ __forceinline__ double store_as<double>(double x) {
  return x;
}

// Packs the W+/- rows of a slab from tmp[al][c][bb][d] = W_{a0+al, c, a0+bb, d}
// (row stride of the (c) index: nbc * v, nbc = v - a0).  One block per (al, bb, tile
// pair): a 32 x 32 tile of M[c][d] = W_{a b c d} and its mirror tile M[d][c] go
// through LDS so that both the reads and the W row writes are contiguous.
//   W+[(a,b)][(c,d)] = M[c][d] + M[d][c] (c < d), M[c][c] (c = d)
//   W-[(a,b)][(c,d)] = M[c][d] - M[d][c]           (a < b, c < d)
// Rows are numbered from the slab's first row: tri(a,b) - tri(a0,a0), stri(a,b) - stri(a0,a0+1).
template <typename InT, typename AccT, typename OutT>
__global__ __launch_bounds__(256) void wslab_pack_kernel(int v, int a0, int na, const InT* __restrict__ tmp,
                                                         OutT* __restrict__ Wp, int64_t ldp,
                                                         OutT* __restrict__ Wm, int64_t ldm, int ntile) {
  __shared__ AccT T1[32][33];
  __shared__ AccT T2[32][33];
  const int64_t V = v, nbc = V - a0;
  const int64_t ntp = (int64_t)ntile * (ntile + 1) / 2;
  const int64_t L = blockIdx.x;
  const int64_t tp = L % ntp;
  const int64_t rest = L / ntp;
  const int64_t bb = rest % nbc, al = rest / nbc;
  if (al >= na || bb < al) return;  // b < a: no row
  // tile pair tp -> (ti <= tj)
  int64_t ti = 0, acc = 0;
  while (acc + (ntile - ti) <= tp) {
    acc += ntile - ti;
    ++ti;
  }
  const int64_t tj = ti + (tp - acc);
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  const InT* M = tmp + (al * V * nbc + bb) * V;  // M[c][d] at M[c * nbc * V + d]
  const int64_t rs = nbc * V;
  const int64_t c0 = ti * 32, d0 = tj * 32;
  for (int r = ty; r < 32; r += 8) {
    const int64_t c = c0 + r, d = d0 + tx;
    T1[r][tx] = (c < V && d < V) ? (AccT)M[c * rs + d] : (AccT)0;
    const int64_t c2 = d0 + r, d2 = c0 + tx;
    T2[r][tx] = (c2 < V && d2 < V) ? (AccT)M[c2 * rs + d2] : (AccT)0;
  }
  __syncthreads();
  const int64_t a = a0 + al, b = a0 + bb;
  const int64_t rowp = tri_ix(a, b, V) - tri_ix(a0, a0, V);
  const bool minus = a < b;
  const int64_t rowm = minus ? stri_ix(a, b, V) - stri_ix(a0, a0 + 1, V) : 0;
  for (int r = ty; r < 32; r += 8) {
    const int64_t c = c0 + r, d = d0 + tx;
    if (c >= V || d >= V || d < c) continue;
    const AccT w1 = T1[r][tx];    // M[c][d]
    const AccT w2 = T2[tx][r];    // M[d][c]
    Wp[rowp * ldp + tri_ix(c, d, V)] = store_as<OutT>(c < d ? w1 + w2 : w1);
    if (minus && c < d) Wm[rowm * ldm + stri_ix(c, d, V)] = store_as<OutT>(w1 - w2);
  }
}

// zero columns [c0, ld) of rows x ld (the bfloat16 K padding of W slab rows)
__global__ void zero_cols_kernel(int64_t rows, int64_t c0, int64_t ld, uint16_t* __restrict__ x) {
  const int64_t w = ld - c0, total = rows * w;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x)
    x[(e / w) * ld + c0 + e % w] = 0;
}

// bfloat16 rows of ld columns from FP64 rows of n columns (zeros past n)
__global__ void rows_to_bf16_kernel(int64_t rows, int64_t n, int64_t ld, const double* __restrict__ x,
                                    uint16_t* __restrict__ y) {
  const int64_t total = rows * ld;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = e / ld, k = e % ld;
    y[e] = k < n ? store_as<uint16_t>((float)x[r * n + k]) : (uint16_t)0;
  }
}

// out[c][r] = in[r][c] for a rows x cols matrix, through 32 x 32 LDS tiles
__global__ __launch_bounds__(256) void transpose_kernel(int64_t rows, int64_t cols, const double* __restrict__ in,
                                                        double* __restrict__ out) {
  __shared__ double t[32][33];
  const int64_t tcols = (cols + 31) / 32;
  const int64_t r0 = (int64_t)(blockIdx.x / tcols) * 32, c0 = (int64_t)(blockIdx.x % tcols) * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  for (int k = ty; k < 32; k += 8) {
    const int64_t r = r0 + k, c = c0 + tx;
    t[k][tx] = (r < rows && c < cols) ? in[r * cols + c] : 0.0;
  }
  __syncthreads();
  for (int k = ty; k < 32; k += 8) {
    const int64_t c = c0 + k, r = r0 + tx;
    if (r < rows && c < cols) out[c * rows + r] = t[tx][k];
  }
}

int64_t elt_tmp(int prec) { return prec == PNOEOM_FP64 ? 8 : 4; }
int64_t elt_w(int prec) { return prec == PNOEOM_FP64 ? 8 : prec == PNOEOM_FP32 ? 4 : 2; }

// packed row lengths of W+/- slabs in a precision (bfloat16 rows padded for the MFMA K loop)
void w_ld(const Context& c, int prec, int64_t& ldp, int64_t& ldm) {
  const int64_t v = c.v, vp = v * (v + 1) / 2, vm = std::max<int64_t>(v * (v - 1) / 2, 1);
  ldp = prec == PNOEOM_BF16 ? bf16_ld(vp) : vp;
  ldm = prec == PNOEOM_BF16 ? bf16_ld(vm) : vm;
}

// a-rows per slab at a0 = 0 that the allocated slab workspace holds in a precision
int64_t slab_rows0(const Context& c, int prec) {
  const int64_t v = c.v;
  int64_t ldp, ldm;
  w_ld(c, prec, ldp, ldm);
  const int64_t t = (int64_t)(c.lad_tmp.n * sizeof(double)) / (v * v * v * elt_tmp(prec));
  const int64_t p = (int64_t)(c.lad_wp.n * sizeof(double)) / (v * ldp * elt_w(prec));
  const int64_t m = (int64_t)(c.lad_wm.n * sizeof(double)) / (v * ldm * elt_w(prec));
  int64_t na0 = std::min(t, std::min(p, m));
  if (c.lad_max_slab > 0) na0 = std::min<int64_t>(na0, c.lad_max_slab);
  return std::min<int64_t>(na0, v);
}

}  // namespace

// default slab workspace: 30% of the free device memory, between 256 MB and 64 GB
int64_t ladder_budget() {
  size_t fr = 0, tot = 0;
  PNO_HIP(hipMemGetInfo(&fr, &tot));
  const int64_t b = (int64_t)(0.3 * (double)fr);
  return std::min<int64_t>(std::max<int64_t>(b, (int64_t)256 << 20), (int64_t)64 << 30);
}

int64_t streamed_ladder_bytes(const Context& c, int64_t na0, int precision) {
  const int64_t v = c.v;
  int64_t bytes = 0;
  for (int p : {(int)PNOEOM_FP64, precision}) {
    int64_t ldp, ldm;
    w_ld(c, p, ldp, ldm);
    bytes = std::max(bytes, na0 * v * (v * v * elt_tmp(p) + (ldp + ldm) * elt_w(p)));
  }
  return bytes;
}

// Low-precision copies of the dressed factors and the slab workspace: na0 a-rows at
// a0 = 0 fit in max(budget, one a-row); sized for FP64 (the refinement of mixed runs)
// and for the context's precision.
void prepare_streamed_ladder(Context& c, int precision, int64_t budget_bytes) {
  hipStream_t s = c.stream;
  const int64_t v = c.v, vv = v * v, naux = c.naux;
  PNO_CHECK(c.BvvT.p != nullptr, PNOEOM_ESTATE, "streamed ladder: dressed factors missing");
  c.BvvTf.release();
  c.BvvTb.release();
  c.lad_tmp.release();
  c.lad_wp.release();
  c.lad_wm.release();
  if (precision == PNOEOM_FP32) {
    c.BvvTf.alloc(vv * naux);
    to_float(s, vv * naux, c.BvvT, c.BvvTf);
  } else if (precision == PNOEOM_BF16) {
    c.ldq = bf16_ld(naux);
    c.BvvTb.alloc(vv * c.ldq);
    hipLaunchKernelGGL(rows_to_bf16_kernel, dim3(grid_of(vv * c.ldq)), dim3(256), 0, s, vv, naux, c.ldq,
                       (const double*)c.BvvT, (uint16_t*)c.BvvTb);
    PNO_HIP(hipGetLastError());
  }
  const int64_t per_row = streamed_ladder_bytes(c, 1, precision);
  int64_t na0 = std::max<int64_t>(1, budget_bytes / per_row);
  na0 = std::min<int64_t>(na0, v);
  if (c.lad_max_slab > 0) na0 = std::min<int64_t>(na0, c.lad_max_slab);
  int64_t tb = 0, pb = 0, mb = 0;
  for (int p : {(int)PNOEOM_FP64, precision}) {
    int64_t ldp, ldm;
    w_ld(c, p, ldp, ldm);
    tb = std::max(tb, na0 * v * vv * elt_tmp(p));
    pb = std::max(pb, na0 * v * ldp * elt_w(p));
    mb = std::max(mb, na0 * v * ldm * elt_w(p));
  }
  c.lad_tmp.alloc((tb + 7) / 8);
  c.lad_wp.alloc((pb + 7) / 8);
  c.lad_wm.alloc((mb + 7) / 8);
  c.lad_streamed = true;
  PNO_HIP(hipStreamSynchronize(s));
}

// sigma+[r][(a<=b)] = sum_{c<=d} W+[(ab),(cd)] S[r][(cd)], sigma-[r][(a<b)] likewise with W- and A,
// for rows r < rows; W+/- rebuilt slab by slab.  Operand types per precision: FP64 (double S, A,
// sigma), FP32 (float), BF16 (bfloat16 S, A with rows of ldS / ldA >= the padded lengths; float sigma).
// sigma+/- have row lengths vp / vm.
void ladder_streamed(Context& c, int precision, int64_t rows, const void* S, int64_t ldS, const void* A,
                     int64_t ldA, void* SigP, void* SigM) {
  PNO_CHECK(c.lad_streamed && c.BvvT.p, PNOEOM_ESTATE, "streamed ladder: factors not prepared");
  PNO_CHECK(precision == PNOEOM_FP64 || (precision == PNOEOM_FP32 && c.BvvTf.p) ||
                (precision == PNOEOM_BF16 && c.BvvTb.p),
            PNOEOM_EINVAL, "streamed ladder: the precision must be FP64 or the one the factors were built for");
  if (rows <= 0) return;
  hipStream_t s = c.stream;
  const int64_t V = c.v, naux = c.naux;
  const int64_t vp = V * (V + 1) / 2, vm = V * (V - 1) / 2;
  int64_t ldp, ldm;
  w_ld(c, precision, ldp, ldm);
  const int64_t na0 = slab_rows0(c, precision);
  PNO_CHECK(na0 >= 1, PNOEOM_ENOMEM, "streamed ladder: slab workspace too small");
  const int ntile = (int)((V + 31) / 32);
  const int64_t ntp = (int64_t)ntile * (ntile + 1) / 2;
  for (int64_t a0 = 0; a0 < V;) {
    const int64_t nbc = V - a0;
    const int64_t na = std::max<int64_t>(1, std::min<int64_t>(nbc, na0 * V / nbc));
    const int64_t Ms = na * V, Ns = nbc * V;
    const int64_t rows_p = na * V - na * (2 * a0 + na - 1) / 2;  // sum over the slab of (V - a)
    const int64_t rows_m = rows_p - na;
    const int64_t rp0 = tri_ix(a0, a0, V), rm0 = rows_m > 0 ? stri_ix(a0, a0 + 1, V) : 0;
    // ---------------------------------------------------------------- W slab from the factors
    hipEvent_t evb = c.region_begin(2, s);
    if (precision == PNOEOM_FP64) {
      GemmDesc<double> d;
      d.tb = true; d.M = Ms; d.N = Ns; d.K = naux; d.tag = 2;
      d.A = c.BvvT + a0 * V * naux; d.lda = naux; d.B = d.A; d.ldb = naux;
      d.C = (double*)c.lad_tmp.p; d.ldc = Ns;
      gemm(d, s);
    } else if (precision == PNOEOM_FP32) {
      GemmDesc<float> d;
      d.tb = true; d.M = Ms; d.N = Ns; d.K = naux; d.tag = 2;
      d.A = c.BvvTf + a0 * V * naux; d.lda = naux; d.B = d.A; d.ldb = naux;
      d.C = (float*)(void*)c.lad_tmp.p; d.ldc = Ns;
      gemm(d, s);
    } else {
      GemmBf16Desc d;
      d.M = Ms; d.N = Ns; d.K = c.ldq; d.tag = 2;
      d.A = c.BvvTb + a0 * V * c.ldq; d.lda = c.ldq; d.B = d.A; d.ldb = c.ldq;
      d.C = (float*)(void*)c.lad_tmp.p; d.ldc = Ns;
      gemm_bf16(d, s);
    }
    const int64_t nblk = na * nbc * ntp;
    PNO_CHECK(nblk < (1ll << 31), PNOEOM_EINVAL, "streamed ladder: slab too large for one pack launch");
    if (precision == PNOEOM_FP64) {
      hipLaunchKernelGGL((wslab_pack_kernel<double, double, double>), dim3((unsigned)nblk), dim3(256), 0, s, (int)V,
                         (int)a0, (int)na, (const double*)c.lad_tmp.p, (double*)c.lad_wp.p, ldp,
                         (double*)c.lad_wm.p, ldm, ntile);
    } else if (precision == PNOEOM_FP32) {
      hipLaunchKernelGGL((wslab_pack_kernel<float, float, float>), dim3((unsigned)nblk), dim3(256), 0, s, (int)V,
                         (int)a0, (int)na, (const float*)(void*)c.lad_tmp.p, (float*)(void*)c.lad_wp.p, ldp,
                         (float*)(void*)c.lad_wm.p, ldm, ntile);
    } else {
      hipLaunchKernelGGL(zero_cols_kernel, dim3(grid_of(rows_p * (ldp - vp))), dim3(256), 0, s, rows_p, vp, ldp,
                         (uint16_t*)(void*)c.lad_wp.p);
      if (rows_m > 0)
        hipLaunchKernelGGL(zero_cols_kernel, dim3(grid_of(rows_m * (ldm - vm))), dim3(256), 0, s, rows_m, vm, ldm,
                           (uint16_t*)(void*)c.lad_wm.p);
      hipLaunchKernelGGL((wslab_pack_kernel<float, float, uint16_t>), dim3((unsigned)nblk), dim3(256), 0, s,
                         (int)V, (int)a0, (int)na, (const float*)(void*)c.lad_tmp.p,
                         (uint16_t*)(void*)c.lad_wp.p, ldp, (uint16_t*)(void*)c.lad_wm.p, ldm, ntile);
    }
    PNO_HIP(hipGetLastError());
    c.region_end(evb, 2, s, 2, 2.0 * (double)Ms * (double)Ns * (double)naux,
                 (double)Ms * Ns * elt_tmp(precision) * 3.0 + (double)(rows_p * ldp + rows_m * ldm) * elt_w(precision));
    // ---------------------------------------------------------------- contraction with the slab rows
    hipEvent_t l0 = nullptr, l1 = nullptr;
    if (c.timing) {
      l0 = c.next_event();
      l1 = c.next_event();
      c.ev_prec.push_back(precision);
      PNO_HIP(hipEventRecord(l0, s));
    }
    if (precision == PNOEOM_FP64) {
      GemmDesc<double> d;
      d.tb = true; d.M = rows; d.N = rows_p; d.K = vp; d.tag = 1;
      d.A = (const double*)S; d.lda = ldS; d.B = (const double*)c.lad_wp.p; d.ldb = ldp;
      d.C = (double*)SigP + rp0; d.ldc = vp;
      gemm(d, s);
      if (rows_m > 0) {
        d.N = rows_m; d.K = vm; d.A = (const double*)A; d.lda = ldA; d.B = (const double*)c.lad_wm.p; d.ldb = ldm;
        d.C = (double*)SigM + rm0; d.ldc = vm;
        gemm(d, s);
      }
    } else if (precision == PNOEOM_FP32) {
      GemmDesc<float> d;
      d.tb = true; d.M = rows; d.N = rows_p; d.K = vp; d.tag = 1;
      d.A = (const float*)S; d.lda = ldS; d.B = (const float*)(void*)c.lad_wp.p; d.ldb = ldp;
      d.C = (float*)SigP + rp0; d.ldc = vp;
      gemm(d, s);
      if (rows_m > 0) {
        d.N = rows_m; d.K = vm; d.A = (const float*)A; d.lda = ldA; d.B = (const float*)(void*)c.lad_wm.p;
        d.ldb = ldm; d.C = (float*)SigM + rm0; d.ldc = vm;
        gemm(d, s);
      }
    } else {
      GemmBf16Desc d;
      d.M = rows; d.N = rows_p; d.K = ldp; d.tag = 1;
      d.A = (const uint16_t*)S; d.lda = ldS; d.B = (const uint16_t*)(void*)c.lad_wp.p; d.ldb = ldp;
      d.C = (float*)SigP + rp0; d.ldc = vp;
      gemm_bf16(d, s);
      if (rows_m > 0) {
        d.N = rows_m; d.K = ldm; d.A = (const uint16_t*)A; d.lda = ldA; d.B = (const uint16_t*)(void*)c.lad_wm.p;
        d.ldb = ldm; d.C = (float*)SigM + rm0; d.ldc = vm;
        gemm_bf16(d, s);
      }
    }
    if (c.timing) {
      PNO_HIP(hipEventRecord(l1, s));
      const double fl = 2.0 * (double)rows * ((double)rows_p * vp + (double)rows_m * vm);
      const int nl = rows_m > 0 ? 2 : 1;
      c.ladder_flops += fl;
      c.ladder_kernel_launches += nl;
      c.ladder_flops_p[precision] += fl;
      c.ladder_launches_p[precision] += nl;
    }
    a0 += na;
  }
}

// Ladder-only factors: B~_vv^Q = B_vv^Q - t1^T B_ov^Q (the virtual block of the T1
// similarity transformation (1 - t)^T B (1 + t^T); the (1 + t^T) factor leaves
// virtual columns unchanged), stored as BvvT[(a,c)][Q].
void build_ladder(Context& c, const double* B, const double* t1, int precision, int64_t budget_bytes) {
  hipStream_t s = c.stream;
  const int o = c.o, nmo = c.nmo;
  const int64_t v = c.v, vv = v * v, naux = c.naux, n2 = (int64_t)nmo * nmo;
  c.have_df = false;
  c.have_lad = false;
  c.drop_graphs();
  c.sw.release();
  c.pno.reset();
  c.precision = precision;
  // the cached ladder and the other intermediates of a previous build_df are not valid any more
  for (DBuf<double>* b : {&c.Wp, &c.Wm, &c.Bt, &c.BovT, &c.BvoT, &c.BooT, &c.BvvT, &c.Bvv2, &c.G, &c.GX, &c.T,
                          &c.U, &c.Tia, &c.Tsia, &c.UiaT, &c.OVVO, &c.OOVVx, &c.Dr, &c.Xr, &c.DX2, &c.YU, &c.BYU, &c.B,
                          &c.DXTT})
    b->release();
  for (DBuf<float>* b : {&c.Wpf, &c.Wmf, &c.DX2f, &c.DXTTf, &c.Whf, &c.g2f, &c.T32, &c.BovTf, &c.BYUf, &c.YUf,
                         &c.Foof, &c.Wvo2f, &c.Zrf})
    b->release();
  for (DBuf<uint16_t>* b : {&c.Whb, &c.Whbs, &c.g2b, &c.TTb, &c.BovQb, &c.BYUb, &c.YUb, &c.Yrb, &c.DXb, &c.DX2b, &c.Gqb,
                            &c.Tvb, &c.Fvob})
    b->release();
  c.Fvvd.release();
  c.Food.release();
  c.bf_rest = false;
  c.Yr.release();
  c.Zr.release();
  c.ring_y = false;
  c.Wpb.release();
  c.Wmb.release();
  {
    DBuf<double> tmp;
    tmp.alloc(naux * vv);
    Perm4 p;  // tmp[Q][a][c] = B[Q][o+a][o+c]
    p.d[0] = naux; p.d[1] = v; p.d[2] = v; p.d[3] = 1;
    p.is[0] = n2; p.is[1] = nmo; p.is[2] = 1; p.is[3] = 0;
    p.os[0] = vv; p.os[1] = v; p.os[2] = 1; p.os[3] = 0;
    permute4(s, p, 1.0, B + (int64_t)o * nmo + o, 0.0, tmp);
    if (t1) {
      DBuf<double> t;
      t.alloc((int64_t)o * v);
      PNO_HIP(hipMemcpyAsync(t, t1, (int64_t)o * v * sizeof(double), hipMemcpyDeviceToDevice, s));
      GemmDesc<double> d;  // tmp^Q -= t1^T B_ov^Q
      d.ta = true; d.M = v; d.N = v; d.K = o; d.alpha = -1.0; d.beta = 1.0;
      d.A = t; d.lda = v; d.sA = 0;
      d.B = B + o; d.ldb = nmo; d.sB = n2;
      d.C = tmp; d.ldc = v; d.sC = vv;
      d.batch = naux;
      gemm(d, s);
      PNO_HIP(hipStreamSynchronize(s));
    }
    c.BvvT.alloc(vv * naux);
    const int64_t ntiles = ((naux + 31) / 32) * ((vv + 31) / 32);
    PNO_CHECK(ntiles < (1ll << 31), PNOEOM_EINVAL, "build_ladder: factor block too large");
    hipLaunchKernelGGL(transpose_kernel, dim3((unsigned)ntiles), dim3(256), 0, s, naux, vv, (const double*)tmp,
                       (double*)c.BvvT);
    PNO_HIP(hipGetLastError());
    PNO_HIP(hipStreamSynchronize(s));
  }
  const int64_t vp = v * (v + 1) / 2, vm = std::max<int64_t>(v * (v - 1) / 2, 1);
  c.ldpb = bf16_ld(vp);
  c.ldmb = bf16_ld(vm);
  prepare_streamed_ladder(c, precision, budget_bytes);
  c.have_lad = true;
}

}  // namespace pnoeom
