// Large-tile bfloat16 GEMM for gfx950: C = alpha A B^T + beta C, A [M][K] and B [N][K]
// bfloat16 (K contiguous, K a multiple of 64), C [M][N] FP32, FP32 accumulation.
//
// One 256-thread workgroup (4 wave64s, 2 x 2) computes a 256 x 256 tile of C; each wave
// a 128 x 128 block as 4 x 4 tiles of v_mfma_f32_32x32x16_bf16 (256 FP32 accumulators
// per lane, kept in the accumulation registers: this file is built without the
// ordinary-VGPR MFMA form used elsewhere in the library, which cannot hold them).
//
// Operand staging: K-tiles of 64 go from global memory straight into LDS
// (global_load_lds_dwordx4: each lane of a wave writes 16 bytes at LDS base + 16 x lane, one
// instruction fills 8 rows of 128 bytes), two buffers of A and B (128 KB, one workgroup per
// CU).  The next K-tile's loads are issued before the current tile's MFMAs, and one barrier
// (after the loads have landed) per K-tile separates the buffers.  Rows have no padding; the
// 16-byte chunk c of row r sits at slot c ^ (r & 7), so the 16 rows one fragment read touches
// fall on distinct bank groups (the loads take the matching global chunk per lane).
//
// Fragments of the next 16-deep k-step are read from LDS while the current step's 16 MFMAs
// run (register double buffer); scheduling barriers keep the compiler from moving the reads
// back next to their use and interleave them with the MFMAs.
//
// MFMA operand layout: lane l supplies 8 consecutive-k values of row l%32 of the A tile
// and of column l%32 of the B tile, k-block l/32 (any fixed assignment of k to slots is
// valid as long as A and B agree).  Accumulator r of lane l holds column l%32 and row
// 8 (r/4) + 4 (l/32) + r%4 of the 32 x 32 tile.
//
// Tile order: workgroup b runs on XCD b % 8, so tiles are handed out in eight contiguous
// chunks, one per XCD.  Within the tile sequence, columns of tiles are taken in groups of
// `group` (M fastest across a group's rows, N fastest within a row of the group), so the ~32
// workgroups an XCD runs at once cover about 32/group rows x group columns of tiles and
// share their A and B panels in that XCD's L2 (group 0: plain M-fastest order, one B panel
// and 32 A panels).
#include "common.h"

namespace pnoeom {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

struct BigArgs {
  int64_t M, N, K;
  float alpha, beta;
  const uint16_t* A;
  int64_t lda;
  const uint16_t* B;
  int64_t ldb;
  float* C;
  int64_t ldc;
  int tiles_m, tiles_n;
  int64_t xper;  // tiles per XCD chunk; 0: grid index = tile index
  int group;     // tile columns per group of the tile order (0: M fastest over all rows)
};

// origin of tile t of the tile order
__device__ __forceinline__ void tile_origin(const BigArgs& g, int64_t t, int64_t& m0, int64_t& n0) {
  if (g.group > 0) {
    const int64_t per = (int64_t)g.tiles_m * g.group;
    const int64_t grp = t / per;
    const int64_t fn = grp * g.group;
    const int64_t gw = g.tiles_n - fn < g.group ? g.tiles_n - fn : g.group;
    const int64_t u = t - grp * per;  // < tiles_m * gw
    m0 = (u / gw) * 256;
    n0 = (fn + u % gw) * 256;
  } else {
    m0 = (t % g.tiles_m) * 256;
    n0 = (t / g.tiles_m) * 256;
  }
}

constexpr int BT = 256;                 // threads
constexpr int TM = 256, TN = 256, TK = 64;
constexpr int WM = TM / 2, WN = TN / 2, FM = WM / 32, FN = WN / 32;
constexpr int NQA = TM / 32, NQB = TN / 32;  // 1 KB direct loads per wave per operand tile

typedef __attribute__((address_space(3))) void lds_void;

template <int TAG>
__global__ __launch_bounds__(BT) __attribute__((amdgpu_waves_per_eu(1))) void gemm_bf16_big_kernel(BigArgs g) {
  __shared__ __attribute__((aligned(1024))) uint16_t lds[2 * (TM + TN) * TK];

  int64_t tile = blockIdx.x;
  if (g.xper > 0) {
    tile = (int64_t)(blockIdx.x % 8) * g.xper + blockIdx.x / 8;
    if (tile >= (int64_t)g.tiles_m * g.tiles_n) return;
  }
  int64_t m0, n0;
  tile_origin(g, tile, m0, n0);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int lr = lane & 31, lk = lane >> 5;

  // direct load q of this wave fills tile rows 8 (wave NQ + q) .. + 8: lane i writes row + i/8,
  // slot i%8, and so reads global chunk (i%8) ^ (row & 7); rows past the end of A / B are
  // clamped to the last row (their results are never stored)
  const int drow = lane >> 3, dslot = lane & 7;
  const uint16_t* ga[NQA];
  const uint16_t* gb[NQB];
#pragma unroll
  for (int q = 0; q < NQA; ++q) {
    const int r = 8 * (wave * NQA + q) + drow;
    int64_t gr = m0 + r;
    if (gr > g.M - 1) gr = g.M - 1;
    ga[q] = g.A + gr * g.lda + 8 * (dslot ^ (r & 7));
  }
#pragma unroll
  for (int q = 0; q < NQB; ++q) {
    const int r = 8 * (wave * NQB + q) + drow;
    int64_t gr = n0 + r;
    if (gr > g.N - 1) gr = g.N - 1;
    gb[q] = g.B + gr * g.ldb + 8 * (dslot ^ (r & 7));
  }
  auto issue = [&](int64_t kt, int buf) {
    uint16_t* as = lds + buf * (TM + TN) * TK;
    uint16_t* bs = as + TM * TK;
    const int64_t k0 = kt * TK;
#pragma unroll
    for (int q = 0; q < NQA; ++q)
      __builtin_amdgcn_global_load_lds((const void*)(ga[q] + k0), (lds_void*)(as + (wave * NQA + q) * 8 * TK), 16, 0,
                                       0);
#pragma unroll
    for (int q = 0; q < NQB; ++q)
      __builtin_amdgcn_global_load_lds((const void*)(gb[q] + k0), (lds_void*)(bs + (wave * NQB + q) * 8 * TK), 16, 0,
                                       0);
  };
  // 16-byte chunk c (k = 8c .. 8c + 7) of tile row r
  auto frag = [&](const uint16_t* base, int row, int c) -> bf16x8 {
    return *reinterpret_cast<const bf16x8*>(base + row * TK + 8 * (c ^ (row & 7)));
  };

  f32x16 acc[FM][FN];
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.f;

  const int64_t ktiles = g.K / TK;
  if (ktiles > 0) issue(0, 0);
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  bf16x8 fa[2][FM], fb[2][FN];
  for (int64_t kt = 0; kt < ktiles; ++kt) {
    const int cur = (int)(kt & 1);
    if (kt + 1 < ktiles) issue(kt + 1, cur ^ 1);  // its buffer was last read before the barrier
    const uint16_t* as = lds + cur * (TM + TN) * TK;
    const uint16_t* bs = as + TM * TK;
#pragma unroll
    for (int i = 0; i < FM; ++i) fa[0][i] = frag(as, wm * WM + i * 32 + lr, lk);
#pragma unroll
    for (int j = 0; j < FN; ++j) fb[0][j] = frag(bs, wn * WN + j * 32 + lr, lk);
#pragma unroll
    for (int st = 0; st < TK / 16; ++st) {
      const int p = st & 1;
      if (st + 1 < TK / 16) {
#pragma unroll
        for (int i = 0; i < FM; ++i) fa[p ^ 1][i] = frag(as, wm * WM + i * 32 + lr, 2 * (st + 1) + lk);
#pragma unroll
        for (int j = 0; j < FN; ++j) fb[p ^ 1][j] = frag(bs, wn * WN + j * 32 + lr, 2 * (st + 1) + lk);
      }
#pragma unroll
      for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fa[p][i], fb[p][j], acc[i][j], 0, 0, 0);
      if (st + 1 < TK / 16) {
        // one fragment read per MFMA for the first FM + FN MFMAs, then the rest of the MFMAs
#pragma unroll
        for (int q = 0; q < FM + FN; ++q) {
          __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);
          __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
        }
        __builtin_amdgcn_sched_group_barrier(0x008, FM * FN - FM - FN, 0);
      }
      __builtin_amdgcn_sched_barrier(0);
    }
    __builtin_amdgcn_s_waitcnt(0);  // the next K-tile's direct loads have landed
    __syncthreads();
  }

#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j) {
      const int64_t gn = n0 + wn * WN + j * 32 + lr;
      if (gn >= g.N) continue;
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int64_t gm = m0 + wm * WM + i * 32 + 8 * (r >> 2) + 4 * lk + (r & 3);
        if (gm >= g.M) continue;
        float* c = g.C + gm * g.ldc + gn;
        float val = g.alpha * acc[i][j][r];
        if (g.beta != 0.f) val += g.beta * (*c);
        *c = val;
      }
    }
}

// The same tile and staging with the k-steps rotated across the barrier: the last k-step's
// MFMAs of a K-tile run after the barrier, overlapping the first fragment reads of the next
// K-tile (which could not start before its direct loads had landed), so that every k-step
// has its fragment reads in flight under the previous step's MFMAs.  Each step opens with
// one MFMA before its first read, so the wait for the previous step's reads is exact.  The
// chunk swizzle uses (r >> 1) & 7: the 16 rows of one fragment read then fall on 16 distinct
// 4-bank groups of a 64-bank LDS (row pairs share a slot but not a bank half).
template <int TAG>
__global__ __launch_bounds__(BT) __attribute__((amdgpu_waves_per_eu(1))) void gemm_bf16_rot_kernel(BigArgs g) {
  __shared__ __attribute__((aligned(1024))) uint16_t lds[2 * (TM + TN) * TK];

  int64_t tile = blockIdx.x;
  if (g.xper > 0) {
    tile = (int64_t)(blockIdx.x % 8) * g.xper + blockIdx.x / 8;
    if (tile >= (int64_t)g.tiles_m * g.tiles_n) return;
  }
  int64_t m0, n0;
  tile_origin(g, tile, m0, n0);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int lr = lane & 31, lk = lane >> 5;
  const int drow = lane >> 3, dslot = lane & 7;
  const uint16_t* ga[NQA];
  const uint16_t* gb[NQB];
#pragma unroll
  for (int q = 0; q < NQA; ++q) {
    const int r = 8 * (wave * NQA + q) + drow;
    int64_t gr = m0 + r;
    if (gr > g.M - 1) gr = g.M - 1;
    ga[q] = g.A + gr * g.lda + 8 * (dslot ^ ((r >> 1) & 7));
  }
#pragma unroll
  for (int q = 0; q < NQB; ++q) {
    const int r = 8 * (wave * NQB + q) + drow;
    int64_t gr = n0 + r;
    if (gr > g.N - 1) gr = g.N - 1;
    gb[q] = g.B + gr * g.ldb + 8 * (dslot ^ ((r >> 1) & 7));
  }
  auto issue = [&](int64_t kt, int buf) {
    uint16_t* as = lds + buf * (TM + TN) * TK;
    uint16_t* bs = as + TM * TK;
    const int64_t k0 = kt * TK;
#pragma unroll
    for (int q = 0; q < NQA; ++q)
      __builtin_amdgcn_global_load_lds((const void*)(ga[q] + k0), (lds_void*)(as + (wave * NQA + q) * 8 * TK), 16, 0,
                                       0);
#pragma unroll
    for (int q = 0; q < NQB; ++q)
      __builtin_amdgcn_global_load_lds((const void*)(gb[q] + k0), (lds_void*)(bs + (wave * NQB + q) * 8 * TK), 16, 0,
                                       0);
  };
  auto frag = [&](const uint16_t* base, int row, int c) -> bf16x8 {
    return *reinterpret_cast<const bf16x8*>(base + row * TK + 8 * (c ^ ((row >> 1) & 7)));
  };
  f32x16 acc[FM][FN];
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.f;
  bf16x8 fa[2][FM], fb[2][FN];
  auto load_frags = [&](int set, const uint16_t* as, const uint16_t* bs, int st) {
#pragma unroll
    for (int i = 0; i < FM; ++i) fa[set][i] = frag(as, wm * WM + i * 32 + lr, 2 * st + lk);
#pragma unroll
    for (int j = 0; j < FN; ++j) fb[set][j] = frag(bs, wn * WN + j * 32 + lr, 2 * st + lk);
  };
  auto mma = [&](int set) {
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
      for (int j = 0; j < FN; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fa[set][i], fb[set][j], acc[i][j], 0, 0, 0);
  };
  auto interleave = [&]() {  // MFMA, read, MFMA, read, ... then the remaining MFMAs
#pragma unroll
    for (int q = 0; q < FM + FN; ++q) {
      __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
      __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);
    }
    __builtin_amdgcn_sched_group_barrier(0x008, FM * FN - FM - FN, 0);
    __builtin_amdgcn_sched_barrier(0);
  };
  // K-tile kt + 1 is loaded while tile kt is multiplied: its direct loads are issued right
  // after the barrier that ends the reads of the buffer it replaces (tile kt - 1's)
  const int64_t ktiles = g.K / TK;
  if (ktiles > 0) {
    issue(0, 0);
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (ktiles > 1) issue(1, 1);
    load_frags(0, lds, lds + TM * TK, 0);
  }
  for (int64_t kt = 0; kt < ktiles; ++kt) {
    const int cur = (int)(kt & 1);
    const uint16_t* as = lds + cur * (TM + TN) * TK;
    const uint16_t* bs = as + TM * TK;
    load_frags(1, as, bs, 1);
    mma(0);
    interleave();
    load_frags(0, as, bs, 2);
    mma(1);
    interleave();
    load_frags(1, as, bs, 3);
    mma(0);
    interleave();
    __builtin_amdgcn_s_waitcnt(0);  // tile kt + 1 has landed and tile kt's reads are done
    __syncthreads();
    if (kt + 2 < ktiles) issue(kt + 2, cur);
    // first fragments of the next K-tile (after the last one: read but unused) under step 3
    const uint16_t* an = lds + (cur ^ 1) * (TM + TN) * TK;
    load_frags(0, an, an + TM * TK, 0);
    mma(1);
    interleave();
  }

#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j) {
      const int64_t gn = n0 + wn * WN + j * 32 + lr;
      if (gn >= g.N) continue;
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int64_t gm = m0 + wm * WM + i * 32 + 8 * (r >> 2) + 4 * lk + (r & 3);
        if (gm >= g.M) continue;
        float* c = g.C + gm * g.ldc + gn;
        float val = g.alpha * acc[i][j][r];
        if (g.beta != 0.f) val += g.beta * (*c);
        *c = val;
      }
    }
}

}  // namespace

bool gemm_bf16_big_fits(int64_t M, int64_t N) { return M >= TM && N >= TN; }

void gemm_bf16_big(const GemmBf16Desc& d, hipStream_t s, bool rotated, int group) {
  static_assert(TM == 256 && TN == 256, "tile_origin assumes 256 x 256 tiles");
  BigArgs g;
  g.group = group;
  g.M = d.M; g.N = d.N; g.K = d.K; g.alpha = d.alpha; g.beta = d.beta;
  g.A = d.A; g.lda = d.lda; g.B = d.B; g.ldb = d.ldb; g.C = d.C; g.ldc = d.ldc;
  g.tiles_m = (int)((d.M + TM - 1) / TM);
  g.tiles_n = (int)((d.N + TN - 1) / TN);
  const int64_t tiles = (int64_t)g.tiles_m * g.tiles_n;
  g.xper = 0;
  int64_t gx = tiles;
  if (tiles >= 64) {
    g.xper = (tiles + 7) / 8;
    gx = 8 * g.xper;
  }
  PNO_CHECK(gx < (1ll << 31), PNOEOM_EINVAL, "gemm_bf16: too many tiles");
  if (rotated) {
    switch (d.tag) {
      case 1: hipLaunchKernelGGL(gemm_bf16_rot_kernel<1>, dim3((unsigned)gx), dim3(BT), 0, s, g); break;
      case 2: hipLaunchKernelGGL(gemm_bf16_rot_kernel<2>, dim3((unsigned)gx), dim3(BT), 0, s, g); break;
      case 3: hipLaunchKernelGGL(gemm_bf16_rot_kernel<3>, dim3((unsigned)gx), dim3(BT), 0, s, g); break;
      default: hipLaunchKernelGGL(gemm_bf16_rot_kernel<0>, dim3((unsigned)gx), dim3(BT), 0, s, g); break;
    }
  } else {
    switch (d.tag) {
      case 1: hipLaunchKernelGGL(gemm_bf16_big_kernel<1>, dim3((unsigned)gx), dim3(BT), 0, s, g); break;
      case 2: hipLaunchKernelGGL(gemm_bf16_big_kernel<2>, dim3((unsigned)gx), dim3(BT), 0, s, g); break;
      case 3: hipLaunchKernelGGL(gemm_bf16_big_kernel<3>, dim3((unsigned)gx), dim3(BT), 0, s, g); break;
      default: hipLaunchKernelGGL(gemm_bf16_big_kernel<0>, dim3((unsigned)gx), dim3(BT), 0, s, g); break;
    }
  }
  PNO_HIP(hipGetLastError());
}

}  // namespace pnoeom
