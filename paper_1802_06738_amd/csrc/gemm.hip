// MFMA-tiled strided/batched GEMM for gfx950 (FP64 and FP32 operands).
//
// One 256-thread workgroup (4 wave64s in a 2 x 2 arrangement) computes a BM x BN
// tile of C.  Operand tiles of BK columns are staged through LDS as As[k][m] and
// Bs[k][n] (m / n contiguous), the next tile is prefetched into registers while
// the current one feeds the matrix cores, and each wave accumulates a
// (BM/2) x (BN/2) block with 16x16x4 MFMA instructions
// (v_mfma_f64_16x16x4_f64 / v_mfma_f32_16x16x4_f32).  Operand layout of both:
// lane l supplies A[l%16][k0 + l/16] and B[k0 + l/16][l%16].  Accumulator r of
// lane l holds column l%16 and row 4*(l/16) + r (FP32) or row l/16 + 4*r (FP64),
// as measured on gfx950.
//
// Occupancy: the kernel is limited to 256 registers per lane so that two
// workgroups share a CU; one workgroup's global loads, LDS stores and barriers
// then overlap the other's MFMA stream (a single workgroup per CU leaves the
// matrix cores idle during those phases).  The library is built with MFMA
// accumulators in ordinary VGPRs, which avoids per-iteration copies between the
// VGPR and AGPR halves of the register file.
//
// Tile order: workgroup b runs on XCD b % 8, so tiles are handed out in eight
// contiguous chunks, one per XCD; the workgroups that share an XCD's L2 then
// work on neighbouring tiles and share their A and B panels.
#include <algorithm>
#include <map>
#include <mutex>
#include <set>

#include "common.h"

namespace pnoeom {
namespace {

template <typename T>
struct Mfma;
template <>
struct Mfma<double> {
  typedef double v4 __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ int row(int lk, int r) { return lk + 4 * r; }
  static __device__ __forceinline__ v4 mac(double a, double b, v4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
};
template <>
struct Mfma<float> {
  typedef float v4 __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ int row(int lk, int r) { return 4 * lk + r; }
  static __device__ __forceinline__ v4 mac(float a, float b, v4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
};

template <typename T>
struct KArgs {
  int64_t M, N, K;
  T alpha, beta;
  const T* A;
  int64_t lda, sA;
  const T* B;
  int64_t ldb, sB;
  T* C;
  int64_t ldc, sC;
  int64_t batch;
  int reduce;
  int tiles_m, tiles_n;
  int64_t xper;       // tiles per XCD chunk; 0: grid index = tile index
  int64_t it_split;   // K-loop iterations per split (split-K); 0: no split
  // split launches: one 1-D grid over the units (tile, batch entry, split), tile fastest,
  // handed to the XCDs in 8 contiguous chunks of uper units (0: 3-D grid)
  int64_t uper, nbz, nsplit;
  int nfast;  // tile order N fastest (few tile columns: the A panel of a row of tiles is read
              // once by neighbouring workgroups, the few B panels stay in L2); else M fastest
  T* ws;              // split-K partials [split][batch_out][M][N]
  int vec_a, vec_b;   // FP32 operands whose interior tiles load as 16-byte vectors (aligned rows)
};

constexpr int NT = 256;


// ==== dense GEMM kernel and its launch: begin
template <typename T, int BM, int BN, int BK, bool TA, bool TB, int TAG>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(2))) void gemm_kernel(KArgs<T> g) {
  constexpr int PADA = (sizeof(T) == 8) ? 1 : 2;
  __shared__ T As[BK][BM + PADA];
  __shared__ T Bs[BK][BN + PADA];
  constexpr int WM = BM / 2, WN = BN / 2;
  constexpr int TM = WM / 16, TN = WN / 16;
  constexpr int LA = BM * BK / NT, LB = BN * BK / NT;
  static_assert(LA * NT == BM * BK && LB * NT == BN * BK, "tile/thread mismatch");
  static_assert(NT % BK == 0 && NT % BM == 0 && NT % BN == 0, "staging map needs NT divisible by the tile");

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int lr = lane & 15, lk = lane >> 4;

  // tile index -> (tm, tn): column-of-tiles major so that consecutive workgroups
  // share the same B panel
  int64_t tile = blockIdx.x;
  int64_t bz = blockIdx.y, kz = blockIdx.z, nbz = gridDim.y;
  if (g.uper > 0) {
    // the tiles of one (batch entry, split) run side by side on one XCD and share their
    // operand panels in its L2
    const int64_t tiles = (int64_t)g.tiles_m * g.tiles_n;
    const int64_t u = (int64_t)(blockIdx.x % 8) * g.uper + blockIdx.x / 8;
    if (u >= tiles * g.nbz * g.nsplit) return;  // padding of the last chunk
    tile = u % tiles;
    bz = (u / tiles) % g.nbz;
    kz = u / (tiles * g.nbz);
    nbz = g.nbz;
  } else if (g.xper > 0) {
    tile = (int64_t)(blockIdx.x % 8) * g.xper + blockIdx.x / 8;
    if (tile >= (int64_t)g.tiles_m * g.tiles_n) return;  // padding of the last chunk
  }
  const int64_t tmi = g.nfast ? tile / g.tiles_n : tile % g.tiles_m;
  const int64_t tni = g.nfast ? tile % g.tiles_n : tile / g.tiles_m;
  const int64_t m0 = tmi * BM, n0 = tni * BN;

  typedef typename Mfma<T>::v4 v4;
  v4 acc[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) acc[i][j] = v4{0, 0, 0, 0};

  const int64_t ktiles = (g.K + BK - 1) / BK;
  const int64_t nb = g.reduce ? g.batch : 1;
  const int64_t total = ktiles * nb;

  T ra[LA], rb[LB];
  // which staging map the registers hold: scalar (element e = tid + q NT) or, for FP32
  // interior tiles of 16-byte aligned operands, vector (four consecutive elements of the
  // contiguous dimension per load: float4 f = tid + q NT holds elements 4f .. 4f + 3)
  bool va = false, vb = false;
  constexpr bool kVec = sizeof(T) == 4 && LA % 4 == 0 && LB % 4 == 0;

  // Staging map: element e = tid + q * NT of the A tile sits at (mm, kk) with
  // mm = e / BK, kk = e % BK (A row-major) or kk = e / BM, mm = e % BM (A^T given);
  // B likewise.  Because NT is a multiple of the tile sides, a thread's elements
  // lie on one column (or row) at a fixed stride, so a tile that lies inside the
  // operands is fetched with one pointer per thread and unguarded loads.
  const bool interior = (m0 + BM <= g.M) && (n0 + BN <= g.N);
  auto load = [&](int64_t it) {
    const int64_t b = g.reduce ? (it / ktiles) : bz;
    const int64_t k0 = (it % ktiles) * BK;
    const T* A = g.A + b * g.sA;
    const T* B = g.B + b * g.sB;
    if (interior && k0 + BK <= g.K) {
      if constexpr (kVec) {
        typedef float f4 __attribute__((ext_vector_type(4)));
        va = g.vec_a != 0;
        vb = g.vec_b != 0;
        if (va) {
#pragma unroll
          for (int q = 0; q < LA / 4; ++q) {
            const int f = tid + q * NT;
            const f4 x = TA ? *(const f4*)(A + (k0 + f / (BM / 4)) * g.lda + m0 + 4 * (f % (BM / 4)))
                            : *(const f4*)(A + (m0 + f / (BK / 4)) * g.lda + k0 + 4 * (f % (BK / 4)));
            ra[4 * q] = x.x; ra[4 * q + 1] = x.y; ra[4 * q + 2] = x.z; ra[4 * q + 3] = x.w;
          }
        }
        if (vb) {
#pragma unroll
          for (int q = 0; q < LB / 4; ++q) {
            const int f = tid + q * NT;
            const f4 x = TB ? *(const f4*)(B + (n0 + f / (BK / 4)) * g.ldb + k0 + 4 * (f % (BK / 4)))
                            : *(const f4*)(B + (k0 + f / (BN / 4)) * g.ldb + n0 + 4 * (f % (BN / 4)));
            rb[4 * q] = x.x; rb[4 * q + 1] = x.y; rb[4 * q + 2] = x.z; rb[4 * q + 3] = x.w;
          }
        }
        if (va && vb) return;
      }
      if (!TA && !va) {
        const T* p = A + (m0 + tid / BK) * g.lda + k0 + tid % BK;
        const int64_t st = (int64_t)(NT / BK) * g.lda;
#pragma unroll
        for (int q = 0; q < LA; ++q) ra[q] = p[q * st];
      } else if (TA && !va) {
        const T* p = A + (k0 + tid / BM) * g.lda + m0 + tid % BM;
        const int64_t st = (int64_t)(NT / BM) * g.lda;
#pragma unroll
        for (int q = 0; q < LA; ++q) ra[q] = p[q * st];
      }
      if (TB && !vb) {
        const T* p = B + (n0 + tid / BK) * g.ldb + k0 + tid % BK;
        const int64_t st = (int64_t)(NT / BK) * g.ldb;
#pragma unroll
        for (int q = 0; q < LB; ++q) rb[q] = p[q * st];
      } else if (!TB && !vb) {
        const T* p = B + (k0 + tid / BN) * g.ldb + n0 + tid % BN;
        const int64_t st = (int64_t)(NT / BN) * g.ldb;
#pragma unroll
        for (int q = 0; q < LB; ++q) rb[q] = p[q * st];
      }
      return;
    }
    va = vb = false;
#pragma unroll
    for (int q = 0; q < LA; ++q) {
      const int e = tid + q * NT;
      int mm, kk;
      if (TA) { kk = e / BM; mm = e % BM; } else { mm = e / BK; kk = e % BK; }
      const int64_t gm = m0 + mm, gk = k0 + kk;
      T val = 0;
      if (gm < g.M && gk < g.K) val = TA ? A[gk * g.lda + gm] : A[gm * g.lda + gk];
      ra[q] = val;
    }
#pragma unroll
    for (int q = 0; q < LB; ++q) {
      const int e = tid + q * NT;
      int nn, kk;
      if (TB) { nn = e / BK; kk = e % BK; } else { kk = e / BN; nn = e % BN; }
      const int64_t gn = n0 + nn, gk = k0 + kk;
      T val = 0;
      if (gn < g.N && gk < g.K) val = TB ? B[gn * g.ldb + gk] : B[gk * g.ldb + gn];
      rb[q] = val;
    }
  };
  auto store = [&]() {
    if (kVec && va) {
#pragma unroll
      for (int q = 0; q < LA / 4; ++q) {
        const int f = tid + q * NT;
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          if (TA) As[f / (BM / 4)][4 * (f % (BM / 4)) + t] = ra[4 * q + t];
          else As[4 * (f % (BK / 4)) + t][f / (BK / 4)] = ra[4 * q + t];
        }
      }
    } else {
#pragma unroll
      for (int q = 0; q < LA; ++q) {
        const int e = tid + q * NT;
        int mm, kk;
        if (TA) { kk = e / BM; mm = e % BM; } else { mm = e / BK; kk = e % BK; }
        As[kk][mm] = ra[q];
      }
    }
    if (kVec && vb) {
#pragma unroll
      for (int q = 0; q < LB / 4; ++q) {
        const int f = tid + q * NT;
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          if (TB) Bs[4 * (f % (BK / 4)) + t][f / (BK / 4)] = rb[4 * q + t];
          else Bs[f / (BN / 4)][4 * (f % (BN / 4)) + t] = rb[4 * q + t];
        }
      }
    } else {
#pragma unroll
      for (int q = 0; q < LB; ++q) {
        const int e = tid + q * NT;
        int nn, kk;
        if (TB) { nn = e / BK; kk = e % BK; } else { kk = e / BN; nn = e % BN; }
        Bs[kk][nn] = rb[q];
      }
    }
  };
  auto compute = [&]() {
#pragma unroll
    for (int kk = 0; kk < BK; kk += 4) {
      T av[TM], bv[TN];
#pragma unroll
      for (int i = 0; i < TM; ++i) av[i] = As[kk + lk][wm * WM + i * 16 + lr];
#pragma unroll
      for (int j = 0; j < TN; ++j) bv[j] = Bs[kk + lk][wn * WN + j * 16 + lr];
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) acc[i][j] = Mfma<T>::mac(av[i], bv[j], acc[i][j]);
    }
  };

  int64_t it_begin = 0, it_end = total;
  if (g.it_split > 0) {
    it_begin = kz * g.it_split;
    it_end = it_begin + g.it_split < total ? it_begin + g.it_split : total;
  }
  if (it_begin < it_end) load(it_begin);
  for (int64_t it = it_begin; it < it_end; ++it) {
    store();
    __syncthreads();
    if (it + 1 < it_end) load(it + 1);
    compute();
    __syncthreads();
  }

  const bool split = g.it_split > 0;
  T* C;
  int64_t ldc;
  if (split) {
    C = g.ws + (kz * nbz + bz) * g.M * g.N;
    ldc = g.N;
  } else {
    C = g.C + (g.reduce ? 0 : bz * g.sC);
    ldc = g.ldc;
  }
  // (with beta != 0 the values of C of one row block are all read before any is written, so
  // that the reads are in flight together; rows and columns past the end read the last one)
  const bool rd = !split && g.beta != T(0);
#pragma unroll
  for (int i = 0; i < TM; ++i) {
    T cv[TN][4];
    if (rd) {
#pragma unroll
      for (int j = 0; j < TN; ++j) {
        const int64_t gn = min(n0 + wn * WN + j * 16 + lr, g.N - 1);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int64_t gm = min(m0 + wm * WM + i * 16 + Mfma<T>::row(lk, r), g.M - 1);
          cv[j][r] = g.beta * C[gm * ldc + gn];
        }
      }
    } else {
#pragma unroll
      for (int j = 0; j < TN; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r) cv[j][r] = T(0);
    }
#pragma unroll
    for (int j = 0; j < TN; ++j) {
      const int64_t gn = n0 + wn * WN + j * 16 + lr;
      if (gn >= g.N) continue;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t gm = m0 + wm * WM + i * 16 + Mfma<T>::row(lk, r);
        if (gm >= g.M) continue;
        C[gm * ldc + gn] = g.alpha * acc[i][j][r] + cv[j][r];
      }
    }
  }
}

// C[b][m][n] = beta * C[b][m][n] + sum_z ws[z][b][m][n], summed in split order
template <typename T>
__global__ void splitk_reduce_kernel(int64_t M, int64_t N, int64_t nb, int64_t nsplit, T beta, const T* __restrict__ ws,
                                     T* __restrict__ C, int64_t ldc, int64_t sC) {
  const int64_t per = M * N;
  const int64_t total = per * nb;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t b = e / per, r = e % per;
    const int64_t m = r / N, n = r % N;
    T acc = 0;
    for (int64_t z = 0; z < nsplit; ++z) acc += ws[(z * nb + b) * per + r];
    T* c = C + b * sC + m * ldc + n;
    if (beta != T(0)) acc += beta * (*c);
    *c = acc;
  }
}

// split-K workspace: one per stream (work on one stream is ordered, so launches on it
// can share it), grown on demand and kept for the life of the process.  hipFree of a
// smaller one synchronises the device first.
struct SplitWs {
  void* p = nullptr;
  size_t bytes = 0;
};
std::mutex& splitk_mu() {
  static std::mutex mu;
  return mu;
}
std::map<hipStream_t, SplitWs>& splitk_map() {
  static std::map<hipStream_t, SplitWs> m;
  return m;
}

template <typename T>
T* splitk_ws(hipStream_t s, size_t count) {
  std::lock_guard<std::mutex> lock(splitk_mu());
  SplitWs& w = splitk_map()[s];
  const size_t bytes = count * sizeof(T);
  if (bytes > w.bytes) {
    if (w.p) PNO_HIP(hipFree(w.p));
    w.p = nullptr;
    w.bytes = 0;
    PNO_HIP(hipMalloc(&w.p, bytes));
    w.bytes = bytes;
  }
  return (T*)w.p;
}

// split_mode: 0 = split K when the output has fewer tiles than CUs (target 512 work
// items), 1 = never split, 2 = split towards 1024 work items
template <typename T, int BM, int BN, int BK>
void launch_tile(const GemmDesc<T>& d, hipStream_t s, int split_mode = 0) {
  KArgs<T> g;
  g.M = d.M; g.N = d.N; g.K = d.K; g.alpha = d.alpha; g.beta = d.beta;
  g.A = d.A; g.lda = d.lda; g.sA = d.sA;
  g.B = d.B; g.ldb = d.ldb; g.sB = d.sB;
  g.C = d.C; g.ldc = d.ldc; g.sC = d.sC;
  g.batch = d.batch; g.reduce = d.reduce ? 1 : 0;
  // 16-byte vector loads of FP32 interior tiles: rows (and batch strides) of whole float4s
  g.vec_a = g.vec_b = 0;
#ifndef PNO_NO_F32_VEC
  if (sizeof(T) == 4) {
    g.vec_a = (d.lda % 4 == 0 && d.sA % 4 == 0 && ((uintptr_t)d.A % 16) == 0) ? 1 : 0;
    g.vec_b = (d.ldb % 4 == 0 && d.sB % 4 == 0 && ((uintptr_t)d.B % 16) == 0) ? 1 : 0;
  }
#endif
  g.tiles_m = (int)((d.M + BM - 1) / BM);
  g.tiles_n = (int)((d.N + BN - 1) / BN);
  g.nfast = g.tiles_n <= 8 && g.tiles_m > g.tiles_n ? 1 : 0;
  const int64_t tiles = (int64_t)g.tiles_m * g.tiles_n;
  PNO_CHECK(tiles < (1ll << 31), PNOEOM_EINVAL, "gemm: too many tiles");
  const int64_t gy = d.reduce ? 1 : d.batch;
  PNO_CHECK(gy <= 65535, PNOEOM_EINVAL, "gemm: batch too large for grid.y");
  // split the K loop when the output has too few tiles to fill the 256 CUs
  const int64_t loop = ((d.K + BK - 1) / BK) * (d.reduce ? d.batch : 1);
  int64_t nsplit = 1;
  if (split_mode != 1 && tiles * gy < (split_mode == 2 ? 512 : 256) && loop >= 32) {
    const int64_t target = split_mode == 2 ? 1024 : 512;
    nsplit = std::min<int64_t>(loop / 8, (target + tiles * gy - 1) / (tiles * gy));
    // a long K loop over a few tiles streams its operands at the rate the loads in flight
    // allow, one K step per workgroup at a time: up to 2048 units (8 per CU) while each
    // keeps at least 32 K steps
    if (split_mode == 0)
      nsplit = std::max<int64_t>(nsplit, std::min<int64_t>(loop / 32, (2048 + tiles * gy - 1) / (tiles * gy)));
    nsplit = std::max<int64_t>(1, std::min<int64_t>(nsplit, 2048));
  } else if (split_mode == 0 && loop >= 4096 && tiles * gy < 2048) {
    // very long K with a few waves of tiles: the last, partly filled wave of workgroups
    // idles most of the chip for a whole K loop; splitting K gives at least four waves
    nsplit = std::min<int64_t>(loop / 1024, (2048 + tiles * gy - 1) / (tiles * gy));
    nsplit = std::max<int64_t>(1, nsplit);
  }
  g.it_split = 0;
  g.ws = nullptr;
  if (nsplit > 1) {
    g.it_split = (loop + nsplit - 1) / nsplit;
    nsplit = (loop + g.it_split - 1) / g.it_split;
    g.ws = splitk_ws<T>(s, (size_t)nsplit * gy * d.M * d.N);
  }
  // XCD-contiguous tile order (the grid is padded to a multiple of 8); a split launch runs
  // as one 1-D grid over (tile, batch entry, split) units in XCD-contiguous chunks
  g.xper = 0;
  g.uper = 0;
  g.nbz = gy;
  g.nsplit = nsplit;
  int64_t gx = tiles;
  dim3 grid;
  if (nsplit > 1) {
    g.uper = (tiles * gy * nsplit + 7) / 8;
    gx = 8 * g.uper;
    PNO_CHECK(gx < (1ll << 31), PNOEOM_EINVAL, "gemm: too many tiles");
    grid = dim3((unsigned)gx, 1, 1);
  } else {
    if (tiles >= 64) {
      g.xper = (tiles + 7) / 8;
      gx = 8 * g.xper;
    }
    PNO_CHECK(gx < (1ll << 31), PNOEOM_EINVAL, "gemm: too many tiles");
    grid = dim3((unsigned)gx, (unsigned)gy, (unsigned)nsplit);
  }
  if (d.tag == 1 && !d.ta && d.tb)
    hipLaunchKernelGGL((gemm_kernel<T, BM, BN, BK, false, true, 1>), grid, dim3(NT), 0, s, g);
  else if (d.tag == 2 && !d.ta && d.tb)
    hipLaunchKernelGGL((gemm_kernel<T, BM, BN, BK, false, true, 2>), grid, dim3(NT), 0, s, g);
  else if (d.tag == 3 && !d.ta && !d.tb)
    hipLaunchKernelGGL((gemm_kernel<T, BM, BN, BK, false, false, 3>), grid, dim3(NT), 0, s, g);
  else if (!d.ta && !d.tb)
    hipLaunchKernelGGL((gemm_kernel<T, BM, BN, BK, false, false, 0>), grid, dim3(NT), 0, s, g);
  else if (d.ta && !d.tb)
    hipLaunchKernelGGL((gemm_kernel<T, BM, BN, BK, true, false, 0>), grid, dim3(NT), 0, s, g);
  else if (!d.ta && d.tb)
    hipLaunchKernelGGL((gemm_kernel<T, BM, BN, BK, false, true, 0>), grid, dim3(NT), 0, s, g);
  else
    hipLaunchKernelGGL((gemm_kernel<T, BM, BN, BK, true, true, 0>), grid, dim3(NT), 0, s, g);
  PNO_HIP(hipGetLastError());
  if (nsplit > 1) {
    const int64_t total = gy * d.M * d.N;
    int64_t blocks = (total + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL((splitk_reduce_kernel<T>), dim3((unsigned)blocks), dim3(256), 0, s, (int64_t)d.M,
                       (int64_t)d.N, gy, nsplit, d.beta, (const T*)g.ws, d.C, d.ldc, d.reduce ? 0 : d.sC);
    PNO_HIP(hipGetLastError());
  }
}

// ==== dense GEMM kernel and its launch: end

// ---------------------------------------------------------------- tile selection and tuning
// A tuning table (filled by the project's autotuner, paper_1802_06738_amd/autotune.py)
// maps a GEMM shape key {element size, ta, tb, reduce, M, N, K, batch} to a variant
// = 3 * tile kind + split mode, tile kinds 128x128, 64x64, 32x128, 128x32.  Shapes
// without an entry use the built-in rule.  Recording collects the keys a workload
// launches, for the tuner.
struct TuneState {
  std::mutex mu;
  bool recording = false;
  std::set<GemmKey> recorded;
  std::map<GemmKey, int> table;
};
TuneState& tune_state() {
  static TuneState st;
  return st;
}

template <typename T>
GemmKey key_of(const GemmDesc<T>& d) {
  return GemmKey{(int64_t)sizeof(T), d.ta ? 1 : 0, d.tb ? 1 : 0, d.reduce ? 1 : 0, d.M, d.N, d.K, d.batch};
}

template <typename T>
void launch_variant(const GemmDesc<T>& d, hipStream_t s, int variant) {
  const int kind = variant / 3, split = variant % 3;
  switch (kind) {
    case 0: launch_tile<T, 128, 128, (sizeof(T) == 8 ? 16 : 32)>(d, s, split); break;
    case 1: launch_tile<T, 64, 64, 16>(d, s, split); break;
    case 2: launch_tile<T, 32, 128, 16>(d, s, split); break;
    default: launch_tile<T, 128, 32, 16>(d, s, split); break;
  }
}

template <typename T>
void gemm_impl(const GemmDesc<T>& d, hipStream_t s) {
  PNO_CHECK(d.M >= 0 && d.N >= 0 && d.K >= 0 && d.batch >= 0, PNOEOM_EINVAL, "gemm: negative size");
  if (d.M == 0 || d.N == 0 || d.batch == 0) return;
  PNO_CHECK(d.A && d.B && d.C, PNOEOM_EINVAL, "gemm: null operand");
  {
    TuneState& ts = tune_state();
    std::lock_guard<std::mutex> lock(ts.mu);
    const GemmKey key = key_of(d);
    if (ts.recording) ts.recorded.insert(key);
    auto it = ts.table.find(key);
    if (it != ts.table.end()) {
      launch_variant(d, s, d.no_split ? 3 * (it->second / 3) + 1 : it->second);
      return;
    }
  }
  // built-in rule: large tiles when both output dimensions fill them
  int kind = 1;
  if (d.M >= 128 && d.N >= 128)
    kind = 0;
  else if (d.M <= 32 && d.N >= 128)
    kind = 2;
  else if (d.N <= 32 && d.M >= 128)
    kind = 3;
  launch_variant(d, s, 3 * kind + (d.no_split ? 1 : 0));
}

// ---------------------------------------------------------------- grouped (64 x 64 tiles, FP64)
constexpr int GBM = 64, GBN = 64, GBK = 16;

// Persistent: a fixed grid of workgroups walks the tiles of all groups (tile t, t + grid,
// ...); every workgroup leaves once it is past the last tile.
template <bool TA, bool TB>
__global__ __launch_bounds__(NT) void gemm_grouped_kernel(const GroupDesc* __restrict__ groups, int ngroups,
                                                          int64_t total_tiles, double alpha,
                                                          const double* __restrict__ Abase,
                                                          const double* __restrict__ Bbase, double beta,
                                                          double* __restrict__ Cbase) {
  typedef double T;
  __shared__ T As[GBK][GBM + 1];
  __shared__ T Bs[GBK][GBN + 1];
  constexpr int WM = GBM / 2, WN = GBN / 2, TM = WM / 16, TN = WN / 16;
  constexpr int LA = GBM * GBK / NT, LB = GBN * GBK / NT;
  for (int64_t tile = blockIdx.x; tile < total_tiles; tile += gridDim.x) {
    int lo = 0, hi = ngroups - 1;
    while (lo < hi) {  // last group with tile_start <= tile
      const int mid = (lo + hi + 1) / 2;
      if (groups[mid].tile_start <= tile) lo = mid; else hi = mid - 1;
    }
    const GroupDesc g = groups[lo];
    const int64_t local = tile - g.tile_start;
    const int64_t m0 = (local % g.tiles_m) * GBM, n0 = (local / g.tiles_m) * GBN;
    const T* A = Abase + g.offA;
    const T* B = Bbase + g.offB;
    T* C = Cbase + g.offC;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave >> 1, wn = wave & 1, lr = lane & 15, lk = lane >> 4;
    typedef Mfma<T>::v4 v4;
    v4 acc[TM][TN];
  #pragma unroll
    for (int i = 0; i < TM; ++i)
  #pragma unroll
      for (int j = 0; j < TN; ++j) acc[i][j] = v4{0, 0, 0, 0};
    const int64_t kt = (g.K + GBK - 1) / GBK;
    // the next K-tile's operands are loaded into registers while the current one is used
    T ra[LA], rb[LB];
    auto gload = [&](int64_t it) {
      const int64_t k0 = it * GBK;
  #pragma unroll
      for (int q = 0; q < LA; ++q) {
        const int e = tid + q * NT;
        int mm, kk;
        if (TA) { kk = e / GBM; mm = e % GBM; } else { mm = e / GBK; kk = e % GBK; }
        const int64_t gm = m0 + mm, gk = k0 + kk;
        T val = 0;
        if (gm < g.M && gk < g.K) val = TA ? A[gk * g.lda + gm] : A[gm * g.lda + gk];
        ra[q] = val;
      }
  #pragma unroll
      for (int q = 0; q < LB; ++q) {
        const int e = tid + q * NT;
        int nn, kk;
        if (TB) { nn = e / GBK; kk = e % GBK; } else { kk = e / GBN; nn = e % GBN; }
        const int64_t gn = n0 + nn, gk = k0 + kk;
        T val = 0;
        if (gn < g.N && gk < g.K) val = TB ? B[gn * g.ldb + gk] : B[gk * g.ldb + gn];
        rb[q] = val;
      }
    };
    if (kt > 0) gload(0);
    for (int64_t it = 0; it < kt; ++it) {
  #pragma unroll
      for (int q = 0; q < LA; ++q) {
        const int e = tid + q * NT;
        if (TA) As[e / GBM][e % GBM] = ra[q]; else As[e % GBK][e / GBK] = ra[q];
      }
  #pragma unroll
      for (int q = 0; q < LB; ++q) {
        const int e = tid + q * NT;
        if (TB) Bs[e % GBK][e / GBK] = rb[q]; else Bs[e / GBN][e % GBN] = rb[q];
      }
      __syncthreads();
      if (it + 1 < kt) gload(it + 1);
  #pragma unroll
      for (int kk = 0; kk < GBK; kk += 4) {
        T av[TM], bv[TN];
  #pragma unroll
        for (int i = 0; i < TM; ++i) av[i] = As[kk + lk][wm * WM + i * 16 + lr];
  #pragma unroll
        for (int j = 0; j < TN; ++j) bv[j] = Bs[kk + lk][wn * WN + j * 16 + lr];
  #pragma unroll
        for (int i = 0; i < TM; ++i)
  #pragma unroll
          for (int j = 0; j < TN; ++j) acc[i][j] = Mfma<T>::mac(av[i], bv[j], acc[i][j]);
      }
      __syncthreads();
    }
  #pragma unroll
    for (int i = 0; i < TM; ++i)
  #pragma unroll
      for (int j = 0; j < TN; ++j) {
        const int64_t gn = n0 + wn * WN + j * 16 + lr;
        if (gn >= g.N) continue;
  #pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int64_t gm = m0 + wm * WM + i * 16 + Mfma<T>::row(lk, r);
          if (gm >= g.M) continue;
          T* c = C + gm * g.ldc + gn;
          T val = alpha * acc[i][j][r];
          if (beta != 0.0) val += beta * (*c);
          *c = val;
        }
      }
  }
}

}  // namespace

void gemm_grouped_prepare(std::vector<GroupDesc>& g, bool ta, bool tb, GroupTable& t) {
  int64_t start = 0;
  std::vector<GroupDesc> keep;
  for (GroupDesc d : g) {
    if (d.M <= 0 || d.N <= 0) continue;
    d.tiles_m = (int32_t)((d.M + GBM - 1) / GBM);
    const int64_t tiles_n = (d.N + GBN - 1) / GBN;
    d.tile_start = start;
    start += d.tiles_m * tiles_n;
    keep.push_back(d);
  }
  if (t.d) PNO_HIP(hipFree(t.d));
  t.d = nullptr;
  t.n = (int)keep.size();
  t.total_tiles = start;
  t.ta = ta;
  t.tb = tb;
  if (t.n == 0) return;
  PNO_HIP(hipMalloc(&t.d, keep.size() * sizeof(GroupDesc)));
  PNO_HIP(hipMemcpy(t.d, keep.data(), keep.size() * sizeof(GroupDesc), hipMemcpyHostToDevice));
}

void gemm_grouped(const GroupTable& t, double alpha, const double* A, const double* B, double beta, double* C,
                  hipStream_t s) {
  if (t.n == 0 || t.total_tiles == 0) return;
  PNO_CHECK(t.total_tiles < (1ll << 31), PNOEOM_EINVAL, "grouped gemm: too many tiles");
  // eight workgroups per CU at most; each walks its share of the tiles
  dim3 grid((unsigned)std::min<int64_t>(t.total_tiles, 8 * 256));
  const int64_t nt = t.total_tiles;
  if (!t.ta && !t.tb)
    hipLaunchKernelGGL((gemm_grouped_kernel<false, false>), grid, dim3(NT), 0, s, t.d, t.n, nt, alpha, A, B, beta, C);
  else if (t.ta && !t.tb)
    hipLaunchKernelGGL((gemm_grouped_kernel<true, false>), grid, dim3(NT), 0, s, t.d, t.n, nt, alpha, A, B, beta, C);
  else if (!t.ta && t.tb)
    hipLaunchKernelGGL((gemm_grouped_kernel<false, true>), grid, dim3(NT), 0, s, t.d, t.n, nt, alpha, A, B, beta, C);
  else
    hipLaunchKernelGGL((gemm_grouped_kernel<true, true>), grid, dim3(NT), 0, s, t.d, t.n, nt, alpha, A, B, beta, C);
  PNO_HIP(hipGetLastError());
}

// ---------------------------------------------------------------- bfloat16 x bfloat16 -> FP32, A B^T
// v_mfma_f32_16x16x32_bf16: lane l supplies 8 consecutive-k values of row l%16 of
// A and of column l%16 of B (the k-slot of each of the 8 values is the same for A
// and B, so any fixed assignment of k to slots is valid; slot block l/16 takes
// k = 8 (l/16) .. 8 (l/16) + 7, a 16-byte LDS read).  The FP32 accumulator layout
// is the one of the 16x16x4 FP32 instruction (row 4 (l/16) + r, column l%16).
// Tiles are staged through LDS as rows of BK = 64 k-values plus 8 of padding
// (144-byte pitch: the 16 rows that one 16-byte read instruction touches fall on
// disjoint bank quadruples).
namespace {
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

struct Bf16Args {
  int64_t M, N, K;
  float alpha, beta;
  const uint16_t* A;
  int64_t lda;
  const uint16_t* B;
  int64_t ldb;
  float* C;
  int64_t ldc;
  int tiles_m, tiles_n;
  int64_t xper;
};

template <int BM, int BN, int TAG>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(2))) void gemm_bf16_kernel(Bf16Args g) {
  constexpr int BK = 64, LD = BK + 8;
  constexpr int WM = BM / 2, WN = BN / 2, TM = WM / 16, TN = WN / 16;
  constexpr int CA = BM * BK / 8 / NT, CB = BN * BK / 8 / NT;  // 16-byte chunks per thread
  static_assert(CA * NT * 8 == BM * BK && CB * NT * 8 == BN * BK, "tile/thread mismatch");
  __shared__ __attribute__((aligned(16))) uint16_t As[BM * LD];
  __shared__ __attribute__((aligned(16))) uint16_t Bs[BN * LD];

  int64_t tile = blockIdx.x;
  if (g.xper > 0) {
    tile = (int64_t)(blockIdx.x % 8) * g.xper + blockIdx.x / 8;
    if (tile >= (int64_t)g.tiles_m * g.tiles_n) return;
  }
  const int64_t m0 = (tile % g.tiles_m) * BM, n0 = (tile / g.tiles_m) * BN;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int lr = lane & 15, lk = lane >> 4;

  // chunk c = tid + NT q covers row c / 8, k-chunk c % 8 (= tid % 8); rows past the
  // end are clamped to the last row (their results are never stored)
  const u32x4* pa[CA];
  const u32x4* pb[CB];
#pragma unroll
  for (int q = 0; q < CA; ++q) {
    int64_t row = m0 + (tid + NT * q) / 8;
    if (row > g.M - 1) row = g.M - 1;
    pa[q] = reinterpret_cast<const u32x4*>(g.A + row * g.lda + (tid % 8) * 8);
  }
#pragma unroll
  for (int q = 0; q < CB; ++q) {
    int64_t row = n0 + (tid + NT * q) / 8;
    if (row > g.N - 1) row = g.N - 1;
    pb[q] = reinterpret_cast<const u32x4*>(g.B + row * g.ldb + (tid % 8) * 8);
  }
  f32x4 acc[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) acc[i][j] = f32x4{0, 0, 0, 0};

  u32x4 ra[CA], rb[CB];
  const int64_t ktiles = g.K / BK;
  if (ktiles > 0) {
#pragma unroll
    for (int q = 0; q < CA; ++q) ra[q] = pa[q][0];
#pragma unroll
    for (int q = 0; q < CB; ++q) rb[q] = pb[q][0];
  }
  for (int64_t kt = 0; kt < ktiles; ++kt) {
#pragma unroll
    for (int q = 0; q < CA; ++q)
      *reinterpret_cast<u32x4*>(&As[((tid + NT * q) / 8) * LD + (tid % 8) * 8]) = ra[q];
#pragma unroll
    for (int q = 0; q < CB; ++q)
      *reinterpret_cast<u32x4*>(&Bs[((tid + NT * q) / 8) * LD + (tid % 8) * 8]) = rb[q];
    __syncthreads();
    if (kt + 1 < ktiles) {
      const int64_t off = (kt + 1) * (BK / 8);  // in 16-byte chunks
#pragma unroll
      for (int q = 0; q < CA; ++q) ra[q] = pa[q][off];
#pragma unroll
      for (int q = 0; q < CB; ++q) rb[q] = pb[q][off];
    }
#pragma unroll
    for (int ks = 0; ks < BK; ks += 32) {
      bf16x8 av[TM], bv[TN];
#pragma unroll
      for (int i = 0; i < TM; ++i)
        av[i] = *reinterpret_cast<const bf16x8*>(&As[(wm * WM + i * 16 + lr) * LD + ks + 8 * lk]);
#pragma unroll
      for (int j = 0; j < TN; ++j)
        bv[j] = *reinterpret_cast<const bf16x8*>(&Bs[(wn * WN + j * 16 + lr) * LD + ks + 8 * lk]);
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[i], bv[j], acc[i][j], 0, 0, 0);
    }
    __syncthreads();
  }
  // (beta != 0: the values of C of one row block read before any is written, as above)
  const bool rd = g.beta != 0.f;
#pragma unroll
  for (int i = 0; i < TM; ++i) {
    float cv[TN][4];
    if (rd) {
#pragma unroll
      for (int j = 0; j < TN; ++j) {
        const int64_t gn = min(n0 + wn * WN + j * 16 + lr, g.N - 1);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int64_t gm = min(m0 + wm * WM + i * 16 + 4 * lk + r, g.M - 1);
          cv[j][r] = g.beta * g.C[gm * g.ldc + gn];
        }
      }
    } else {
#pragma unroll
      for (int j = 0; j < TN; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r) cv[j][r] = 0.f;
    }
#pragma unroll
    for (int j = 0; j < TN; ++j) {
      const int64_t gn = n0 + wn * WN + j * 16 + lr;
      if (gn >= g.N) continue;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t gm = m0 + wm * WM + i * 16 + 4 * lk + r;
        if (gm >= g.M) continue;
        g.C[gm * g.ldc + gn] = g.alpha * acc[i][j][r] + cv[j][r];
      }
    }
  }
}
}  // namespace

// ==== bf16 GEMM dispatch: begin
void gemm_bf16(const GemmBf16Desc& d, hipStream_t s) {
  PNO_CHECK(d.M >= 0 && d.N >= 0 && d.K >= 0, PNOEOM_EINVAL, "gemm_bf16: negative size");
  if (d.M == 0 || d.N == 0) return;
  PNO_CHECK(d.A && d.B && d.C, PNOEOM_EINVAL, "gemm_bf16: null operand");
  PNO_CHECK(d.K % kBf16K == 0 && d.lda % 8 == 0 && d.ldb % 8 == 0 && d.lda >= d.K && d.ldb >= d.K, PNOEOM_EINVAL,
            "gemm_bf16: K and the leading dimensions must be padded to multiples of 64 and 8");
  PNO_CHECK(((uintptr_t)d.A % 16) == 0 && ((uintptr_t)d.B % 16) == 0, PNOEOM_EINVAL,
            "gemm_bf16: operands must be 16-byte aligned");
  PNO_CHECK(d.variant >= 0 && d.variant <= 5, PNOEOM_EINVAL, "gemm_bf16: unknown variant");
  PNO_CHECK(d.variant < 2 || gemm_bf16_big_fits(d.M, d.N), PNOEOM_EINVAL,
            "gemm_bf16: the 256 x 256 tiles need M, N >= 160");
  const int64_t tiles256 = ((d.M + 255) / 256) * ((d.N + 255) / 256);
  const int64_t ktiles = d.K / kBf16K;
  // (a K loop of at most 8 K-tiles leaves the 256 x 256 tile's serial load / MFMA / store
  // phases exposed, one workgroup per CU: the 128 x 128 kernel overlaps them across
  // workgroups; 640000 x 400 x 448: 0.55 against 0.69 ms)
  if (d.variant >= 2 || (d.variant == 0 && gemm_bf16_big_fits(d.M, d.N) && ktiles > 8 &&
                         (tiles256 >= 256 || ktiles >= 32))) {
    // split K when the tiles fill the 256 CUs poorly (fraction of the waves of workgroups that
    // has work) and the K loop is long: partials in the split-K workspace, summed in split
    // order by splitk_reduce_kernel.  A split costs about one write and one read of the
    // output per partial against 2 K flops per output element: sp 1000 / K of the time
    int nsplit = 1;
    if (!d.no_split && (d.variant == 0 || d.variant == 3)) {
      auto fill = [](int64_t t) { return (double)t / (double)(((t + 255) / 256) * 256); };
      double best = fill(tiles256) + 0.05;
      for (int sp = 2; sp <= 64 && ktiles / sp >= 16; ++sp) {
        const double f = fill(tiles256 * sp) - sp * 1000.0 / (double)d.K;
        if (f > best) {
          best = f;
          nsplit = sp;
        }
      }
      if (nsplit > 1) {
        const int64_t kper = (ktiles + nsplit - 1) / nsplit;
        nsplit = (int)((ktiles + kper - 1) / kper);
      }
    }
    // tile order: with at most 32 rows of tiles and a long K loop, M-fastest order keeps every
    // row of a tile column running at once on each XCD (the B panel shared in the XCD's L2,
    // the A panels shared across XCDs in the memory-side cache; 4920 x 80200 x 80256: 1111
    // against 999 TFLOP/s grouped); otherwise groups of 4 tile columns (96000 x 16000 x 16000:
    // 1215 against 1054 M-fastest)
    int group = (d.M + 255) / 256 <= 32 && d.K >= 8192 ? 0 : 4;
    if (d.variant == 4) group = 0;
    if (d.variant == 5) group = 8;
    if (nsplit > 1) {
      float* ws = splitk_ws<float>(s, (size_t)nsplit * d.M * d.N);
      gemm_bf16_big(d, s, d.variant != 2, group, nsplit, ws);
      const int64_t total = d.M * d.N;
      int64_t blocks = (total + 255) / 256;
      if (blocks > 65536) blocks = 65536;
      hipLaunchKernelGGL((splitk_reduce_kernel<float>), dim3((unsigned)blocks), dim3(256), 0, s, d.M, d.N,
                         (int64_t)1, (int64_t)nsplit, d.beta, (const float*)ws, d.C, d.ldc, (int64_t)0);
      PNO_HIP(hipGetLastError());
    } else {
      gemm_bf16_big(d, s, d.variant != 2, group);
    }
    return;
  }
  constexpr int BM = 128, BN = 128;
  Bf16Args g;
  g.M = d.M; g.N = d.N; g.K = d.K; g.alpha = d.alpha; g.beta = d.beta;
  g.A = d.A; g.lda = d.lda; g.B = d.B; g.ldb = d.ldb; g.C = d.C; g.ldc = d.ldc;
  g.tiles_m = (int)((d.M + BM - 1) / BM);
  g.tiles_n = (int)((d.N + BN - 1) / BN);
  const int64_t tiles = (int64_t)g.tiles_m * g.tiles_n;
  g.xper = 0;
  int64_t gx = tiles;
  if (tiles >= 64) {
    g.xper = (tiles + 7) / 8;
    gx = 8 * g.xper;
  }
  PNO_CHECK(gx < (1ll << 31), PNOEOM_EINVAL, "gemm_bf16: too many tiles");
  if (d.tag == 1)
    hipLaunchKernelGGL((gemm_bf16_kernel<BM, BN, 1>), dim3((unsigned)gx), dim3(NT), 0, s, g);
  else if (d.tag == 2)
    hipLaunchKernelGGL((gemm_bf16_kernel<BM, BN, 2>), dim3((unsigned)gx), dim3(NT), 0, s, g);
  else if (d.tag == 3)
    hipLaunchKernelGGL((gemm_bf16_kernel<BM, BN, 3>), dim3((unsigned)gx), dim3(NT), 0, s, g);
  else
    hipLaunchKernelGGL((gemm_bf16_kernel<BM, BN, 0>), dim3((unsigned)gx), dim3(NT), 0, s, g);
  PNO_HIP(hipGetLastError());
}
// ==== bf16 GEMM dispatch: end

namespace {
__global__ void fill_bf16_kernel(int64_t n, uint16_t* x) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
    const float f = 1e-3f * (float)((e * 2654435761ll) % 1000) - 0.5f;
    x[e] = (uint16_t)(__float_as_uint(f) >> 16);
  }
}
}  // namespace

double gemm_bf16_time(hipStream_t s, int64_t M, int64_t N, int64_t K, int variant, int reps) {
  PNO_CHECK(M > 0 && N > 0 && K > 0 && K % kBf16K == 0 && reps > 0, PNOEOM_EINVAL, "gemm_bf16_time: bad shape");
  if ((M * K + N * K) * 2 + M * N * 4 > (16ll << 30)) return -1.0;  // not timed: too large
  DBuf<uint16_t> A, B;
  DBuf<float> C;
  A.alloc(M * K);
  B.alloc(N * K);
  C.alloc(M * N);
  hipLaunchKernelGGL(fill_bf16_kernel, dim3(1024), dim3(256), 0, s, M * K, (uint16_t*)A);
  hipLaunchKernelGGL(fill_bf16_kernel, dim3(1024), dim3(256), 0, s, N * K, (uint16_t*)B);
  PNO_HIP(hipGetLastError());
  GemmBf16Desc d;
  d.M = M; d.N = N; d.K = K; d.A = A; d.lda = K; d.B = B; d.ldb = K; d.C = C; d.ldc = N; d.variant = variant;
  gemm_bf16(d, s);  // warm-up
  hipEvent_t e0, e1;
  PNO_HIP(hipEventCreate(&e0));
  PNO_HIP(hipEventCreate(&e1));
  PNO_HIP(hipEventRecord(e0, s));
  for (int r = 0; r < reps; ++r) gemm_bf16(d, s);
  PNO_HIP(hipEventRecord(e1, s));
  PNO_HIP(hipEventSynchronize(e1));
  float ms = 0.f;
  PNO_HIP(hipEventElapsedTime(&ms, e0, e1));
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return (double)ms / reps;
}

namespace {
__global__ void tune_fill_kernel(int64_t n, double* x) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
    x[e] = 1e-3 * (double)((e * 2654435761ll) % 1000) - 0.5;
}
__global__ void tune_fill_kernel_f(int64_t n, float* x) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
    x[e] = 1e-3f * (float)((e * 2654435761ll) % 1000) - 0.5f;
}

template <typename T>
double time_variant(hipStream_t s, const GemmKey& k, int variant, int reps) {
  GemmDesc<T> d;
  d.ta = k[1] != 0; d.tb = k[2] != 0; d.reduce = k[3] != 0;
  d.M = k[4]; d.N = k[5]; d.K = k[6]; d.batch = k[7];
  const int64_t na = d.batch * d.M * d.K, nbv = d.K * d.N;
  const int64_t nc = (d.reduce ? 1 : d.batch) * d.M * d.N;
  if ((na + nbv + nc) * (int64_t)sizeof(T) > (8ll << 30)) return -1.0;  // not timed: too large
  DBuf<T> A, B, C;
  A.alloc(std::max<int64_t>(na, 1)); B.alloc(std::max<int64_t>(nbv, 1)); C.alloc(std::max<int64_t>(nc, 1));
  if (sizeof(T) == 8) {
    hipLaunchKernelGGL(tune_fill_kernel, dim3(1024), dim3(256), 0, s, na, (double*)(void*)A.p);
    hipLaunchKernelGGL(tune_fill_kernel, dim3(1024), dim3(256), 0, s, nbv, (double*)(void*)B.p);
  } else {
    hipLaunchKernelGGL(tune_fill_kernel_f, dim3(1024), dim3(256), 0, s, na, (float*)(void*)A.p);
    hipLaunchKernelGGL(tune_fill_kernel_f, dim3(1024), dim3(256), 0, s, nbv, (float*)(void*)B.p);
  }
  d.A = A; d.lda = d.ta ? d.M : d.K; d.sA = d.M * d.K;
  d.B = B; d.ldb = d.tb ? d.K : d.N; d.sB = 0;
  d.C = C; d.ldc = d.N; d.sC = d.reduce ? 0 : d.M * d.N;
  d.alpha = 1; d.beta = 0;
  launch_variant(d, s, variant);  // warm-up (sizes the split-K workspace)
  hipEvent_t e0, e1;
  PNO_HIP(hipEventCreate(&e0));
  PNO_HIP(hipEventCreate(&e1));
  PNO_HIP(hipEventRecord(e0, s));
  for (int r = 0; r < reps; ++r) launch_variant(d, s, variant);
  PNO_HIP(hipEventRecord(e1, s));
  PNO_HIP(hipEventSynchronize(e1));
  float ms = 0.f;
  PNO_HIP(hipEventElapsedTime(&ms, e0, e1));
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return (double)ms / std::max(reps, 1);
}
}  // namespace

uint64_t gemm_workspace_signature(hipStream_t s) {
  std::lock_guard<std::mutex> lock(splitk_mu());
  auto it = splitk_map().find(s);
  return it == splitk_map().end() ? 0 : (uint64_t)(uintptr_t)it->second.p;
}

void gemm_tune_record(bool on) {
  TuneState& ts = tune_state();
  std::lock_guard<std::mutex> lock(ts.mu);
  ts.recording = on;
  if (on) ts.recorded.clear();
}

std::vector<GemmKey> gemm_tune_recorded() {
  TuneState& ts = tune_state();
  std::lock_guard<std::mutex> lock(ts.mu);
  return std::vector<GemmKey>(ts.recorded.begin(), ts.recorded.end());
}

void gemm_tune_set(const std::vector<GemmKey>& keys, const std::vector<int>& variants) {
  TuneState& ts = tune_state();
  std::lock_guard<std::mutex> lock(ts.mu);
  ts.table.clear();
  for (size_t i = 0; i < keys.size(); ++i) ts.table[keys[i]] = variants[i];
}

double gemm_tune_time(hipStream_t s, const GemmKey& key, int variant, int reps) {
  PNO_CHECK(variant >= 0 && variant < kGemmVariants, PNOEOM_EINVAL, "gemm_tune_time: bad variant");
  PNO_CHECK((key[0] == 8 || key[0] == 4) && key[4] > 0 && key[5] > 0 && key[6] >= 0 && key[7] >= 1, PNOEOM_EINVAL,
            "gemm_tune_time: bad shape key");
  return key[0] == 8 ? time_variant<double>(s, key, variant, reps) : time_variant<float>(s, key, variant, reps);
}

void gemm(const GemmDesc<double>& d, hipStream_t s) { gemm_impl<double>(d, s); }
void gemm(const GemmDesc<float>& d, hipStream_t s) { gemm_impl<float>(d, s); }

}  // namespace pnoeom
