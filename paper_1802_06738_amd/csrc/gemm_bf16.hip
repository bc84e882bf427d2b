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
// Epilogue: the accumulators go through LDS (half a tile at a time) so that C is written in
// whole rows, 16 bytes per lane, and for beta != 0 read in batches ahead of the writes.
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
  int64_t kper;  // split K: K-tiles per split (grid.y = splits), partials alpha A B^T into
  float* ws;     // ws[split][M][N]; kper = 0: no split, C = alpha A B^T + beta C
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

// C tile store, through LDS in two halves of 128 rows (the operand buffers are free by then):
// the accumulators of a half go to LDS as [128][256] FP32 (accumulator r of lane l holds
// column l%32 and row 8 (r/4) + 4 (l/32) + r%4 of each 32 x 32 block), then each wave writes
// whole rows of C, 16 bytes per lane.  For beta != 0 eight rows of C per lane are read before
// any is written, so that the reads are in flight together (read after the stores before them,
// each would wait for the previous store).  Edge tiles (or C rows not 16-byte aligned) take
// the element-wise form.  With split K the partial alpha A B^T goes to ws[split] (rows of N).
__device__ __forceinline__ void store_tile(const BigArgs& g, const f32x16 (&acc)[FM][FN], int64_t m0, int64_t n0,
                                           int wm, int wn, int lr, int lk, uint16_t* lds) {
  float* sm = reinterpret_cast<float*>(lds);
  float* C = g.C;
  int64_t ldc = g.ldc;
  float beta = g.beta;
  if (g.kper > 0) {
    C = g.ws + (int64_t)blockIdx.y * g.M * g.N;
    ldc = g.N;
    beta = 0.f;
  }
  const float alpha = g.alpha;
  const int tid = threadIdx.x, c4 = tid & 63, r0 = tid >> 6;
  const bool vec = m0 + TM <= g.M && n0 + TN <= g.N && (ldc & 3) == 0 && ((uintptr_t)C & 15) == 0;
  float* Ct = C + m0 * ldc + n0;
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    __syncthreads();  // LDS free: operand reads (or the previous half) done
#pragma unroll
    for (int ii = 0; ii < 2; ++ii)
#pragma unroll
      for (int j = 0; j < FN; ++j)
#pragma unroll
        for (int r = 0; r < 16; ++r)
          sm[(wm * 64 + ii * 32 + 8 * (r >> 2) + 4 * lk + (r & 3)) * TN + wn * WN + j * 32 + lr] =
              acc[2 * h + ii][j][r];
    __syncthreads();
    // local row lr of the half is tile row (lr / 64) 128 + 64 h + lr % 64
    if (vec) {
#pragma unroll
      for (int kb = 0; kb < 32; kb += 8) {
        float4 cv[8];
        if (beta != 0.f) {
#pragma unroll
          for (int k = 0; k < 8; ++k) {
            const int lrow = r0 + 4 * (kb + k);
            const int64_t trow = (lrow >> 6) * WM + h * 64 + (lrow & 63);
            cv[k] = *reinterpret_cast<const float4*>(Ct + trow * ldc + 4 * c4);
          }
        }
#pragma unroll
        for (int k = 0; k < 8; ++k) {
          const int lrow = r0 + 4 * (kb + k);
          const int64_t trow = (lrow >> 6) * WM + h * 64 + (lrow & 63);
          const float4 a = *reinterpret_cast<const float4*>(sm + lrow * TN + 4 * c4);
          float4 o;
          o.x = alpha * a.x;
          o.y = alpha * a.y;
          o.z = alpha * a.z;
          o.w = alpha * a.w;
          if (beta != 0.f) {
            o.x += beta * cv[k].x;
            o.y += beta * cv[k].y;
            o.z += beta * cv[k].z;
            o.w += beta * cv[k].w;
          }
          *reinterpret_cast<float4*>(Ct + trow * ldc + 4 * c4) = o;
        }
      }
    } else {
      for (int k = 0; k < 32; ++k) {
        const int lrow = r0 + 4 * k;
        const int64_t gm = m0 + (lrow >> 6) * WM + h * 64 + (lrow & 63);
        if (gm >= g.M) continue;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int64_t gn = n0 + 4 * c4 + e;
          if (gn >= g.N) continue;
          float* c = C + gm * ldc + gn;
          float val = alpha * sm[lrow * TN + 4 * c4 + e];
          if (beta != 0.f) val += beta * (*c);
          *c = val;
        }
      }
    }
  }
}

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

  int64_t kb = 0, ke = g.K / TK;  // this workgroup's K-tiles
  if (g.kper > 0) {
    kb = (int64_t)blockIdx.y * g.kper;
    ke = kb + g.kper < ke ? kb + g.kper : ke;
  }
  if (kb < ke) issue(kb, 0);
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  bf16x8 fa[2][FM], fb[2][FN];
  for (int64_t kt = kb; kt < ke; ++kt) {
    const int cur = (int)((kt - kb) & 1);
    if (kt + 1 < ke) issue(kt + 1, cur ^ 1);  // its buffer was last read before the barrier
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

  store_tile(g, acc, m0, n0, wm, wn, lr, lk, lds);
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
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // uniform: LDS bases in scalar registers
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
  // direct loads q = 2p, 2p + 1 of the A tile and of the B tile
  auto issue_part = [&](int64_t kt, int buf, int p) {
    uint16_t* as = lds + buf * (TM + TN) * TK;
    uint16_t* bs = as + TM * TK;
    const int64_t k0 = kt * TK;
#pragma unroll
    for (int q = 2 * p; q < 2 * p + 2; ++q) {
      __builtin_amdgcn_global_load_lds((const void*)(ga[q] + k0), (lds_void*)(as + (wave * NQA + q) * 8 * TK), 16, 0,
                                       0);
      __builtin_amdgcn_global_load_lds((const void*)(gb[q] + k0), (lds_void*)(bs + (wave * NQB + q) * 8 * TK), 16, 0,
                                       0);
    }
  };
  auto mma_row = [&](int set, int i) {
#pragma unroll
    for (int j = 0; j < FN; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fa[set][i], fb[set][j], acc[i][j], 0, 0, 0);
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
  int64_t kb = 0, ke = g.K / TK;  // this workgroup's K-tiles
  if (g.kper > 0) {
    kb = (int64_t)blockIdx.y * g.kper;
    ke = kb + g.kper < ke ? kb + g.kper : ke;
  }
  if (kb < ke) {
    issue(kb, 0);
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (kb + 1 < ke) issue(kb + 1, 1);
    load_frags(0, lds, lds + TM * TK, 0);
  }
  for (int64_t kt = kb; kt < ke; ++kt) {
    const int cur = (int)((kt - kb) & 1);
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
    // first fragments of the next K-tile (after the last one: read but unused), then step 3's
    // MFMAs row by row, each row beside a quarter of the direct loads of tile kt + 2 into the
    // buffer just freed (so that the load issue does not hold the matrix cores); in the last
    // two K-tiles the loads repeat the last K-tile (unused), which keeps them in the same
    // block as the MFMAs
    const uint16_t* an = lds + (cur ^ 1) * (TM + TN) * TK;
    load_frags(0, an, an + TM * TK, 0);
    __builtin_amdgcn_sched_barrier(0);
    const int64_t kn = kt + 2 < ke ? kt + 2 : ke - 1;
#pragma unroll
    for (int p = 0; p < FM; ++p) {
      issue_part(kn, cur, p);
      mma_row(1, p);
      __builtin_amdgcn_sched_barrier(0);
    }
  }
  __builtin_amdgcn_s_waitcnt(0);  // no direct load is left in flight

  store_tile(g, acc, m0, n0, wm, wn, lr, lk, lds);
}

}  // namespace

// rows and columns past the end of A / B are clamped on load and never stored, so any shape
// runs; below 5/8 of a tile in either dimension the 128 x 128 kernel wastes less
bool gemm_bf16_big_fits(int64_t M, int64_t N) { return M >= 160 && N >= 160; }

void gemm_bf16_big(const GemmBf16Desc& d, hipStream_t s, bool rotated, int group, int nsplit, float* ws) {
  static_assert(TM == 256 && TN == 256, "tile_origin assumes 256 x 256 tiles");
  BigArgs g;
  g.group = group;
  g.kper = 0;
  g.ws = nullptr;
  const int64_t ktiles = d.K / TK;
  if (nsplit > 1) {
    PNO_CHECK(ws != nullptr && nsplit <= 65535, PNOEOM_EINVAL, "gemm_bf16: split K without a workspace");
    g.kper = (ktiles + nsplit - 1) / nsplit;
    PNO_CHECK((ktiles + g.kper - 1) / g.kper == nsplit, PNOEOM_EINVAL, "gemm_bf16: empty K split");
    g.ws = ws;
  } else {
    nsplit = 1;
  }
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
      case 1: hipLaunchKernelGGL(gemm_bf16_rot_kernel<1>, dim3((unsigned)gx, (unsigned)nsplit), dim3(BT), 0, s, g); break;
      case 2: hipLaunchKernelGGL(gemm_bf16_rot_kernel<2>, dim3((unsigned)gx, (unsigned)nsplit), dim3(BT), 0, s, g); break;
      case 3: hipLaunchKernelGGL(gemm_bf16_rot_kernel<3>, dim3((unsigned)gx, (unsigned)nsplit), dim3(BT), 0, s, g); break;
      default: hipLaunchKernelGGL(gemm_bf16_rot_kernel<0>, dim3((unsigned)gx, (unsigned)nsplit), dim3(BT), 0, s, g); break;
    }
  } else {
    switch (d.tag) {
      case 1: hipLaunchKernelGGL(gemm_bf16_big_kernel<1>, dim3((unsigned)gx, (unsigned)nsplit), dim3(BT), 0, s, g); break;
      case 2: hipLaunchKernelGGL(gemm_bf16_big_kernel<2>, dim3((unsigned)gx, (unsigned)nsplit), dim3(BT), 0, s, g); break;
      case 3: hipLaunchKernelGGL(gemm_bf16_big_kernel<3>, dim3((unsigned)gx, (unsigned)nsplit), dim3(BT), 0, s, g); break;
      default: hipLaunchKernelGGL(gemm_bf16_big_kernel<0>, dim3((unsigned)gx, (unsigned)nsplit), dim3(BT), 0, s, g); break;
    }
  }
  PNO_HIP(hipGetLastError());
}

}  // namespace pnoeom
