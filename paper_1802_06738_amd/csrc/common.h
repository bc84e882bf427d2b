// Shared declarations for the pnoeom HIP library (gfx950 / MI355X only).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <stdexcept>
#include <string>
#include <array>
#include <vector>

#include <rocprofiler-sdk-roctx/roctx.h>

#include "../../include/pnoeom.h"

namespace pnoeom {

// Named roctx range for the lifetime of a scope (seen by rocprofv3 --marker-trace).
struct TraceRange {
  explicit TraceRange(const char* name) { roctxRangePushA(name); }
  ~TraceRange() { roctxRangePop(); }
  TraceRange(const TraceRange&) = delete;
  TraceRange& operator=(const TraceRange&) = delete;
};

struct Error : std::runtime_error {
  int code;
  Error(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};

#define PNO_HIP(x)                                                                      \
  do {                                                                                  \
    hipError_t e_ = (x);                                                                \
    if (e_ != hipSuccess)                                                               \
      throw ::pnoeom::Error(PNOEOM_EHIP, std::string(#x " failed: ") + hipGetErrorString(e_) + \
                                             " at " __FILE__ ":" + std::to_string(__LINE__)); \
  } while (0)

#define PNO_CHECK(cond, code, msg)                 \
  do {                                             \
    if (!(cond)) throw ::pnoeom::Error(code, msg); \
  } while (0)

// Device buffer owned by the library.
template <typename T>
struct DBuf {
  T* p = nullptr;
  size_t n = 0;
  DBuf() = default;
  DBuf(const DBuf&) = delete;
  DBuf& operator=(const DBuf&) = delete;
  ~DBuf() { release(); }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    n = 0;
  }
  void alloc(size_t count) {
    if (count == n && p) return;
    release();
    if (count == 0) return;
    hipError_t e = hipMalloc(&p, count * sizeof(T));
    if (e != hipSuccess) {
      p = nullptr;
      throw Error(PNOEOM_ENOMEM, "hipMalloc of " + std::to_string(count * sizeof(T)) + " bytes failed (" +
                                     hipGetErrorString(e) + ")");
    }
    n = count;
  }
  operator T*() const { return p; }
};

// ----------------------------------------------------------------------------- GEMM
// Row-major strided (batched) matrix product on MFMA:
//   C[b] = alpha * op(A[b]) * op(B[b]) + beta * C[b]
// op(A) is M x K: A[m*lda + k] (transA = false) or A[k*lda + m] (transA = true).
// op(B) is K x N: B[k*ldb + n] (transB = false) or B[n*ldb + k] (transB = true).
// C[m*ldc + n].  With reduce = true the batch index is summed into one C.
template <typename T>
struct GemmDesc {
  bool ta = false, tb = false;
  int64_t M = 0, N = 0, K = 0;
  T alpha = 1, beta = 0;
  const T* A = nullptr;
  int64_t lda = 0, sA = 0;
  const T* B = nullptr;
  int64_t ldb = 0, sB = 0;
  T* C = nullptr;
  int64_t ldc = 0, sC = 0;
  int64_t batch = 1;
  bool reduce = false;
  int tag = 0;  // 1: particle-particle ladder, 2: its W slab build, 3: ring products (own kernel symbols, for profiling)
  bool no_split = false;  // never split K (split-K partials live in a workspace the library allocates)
};

void gemm(const GemmDesc<double>& d, hipStream_t s);
void gemm(const GemmDesc<float>& d, hipStream_t s);

// tuning of the tile / split-K choice per shape: key {element size, ta, tb, reduce, M, N, K, batch},
// variant = 3 * tile kind (128x128, 64x64, 32x128, 128x32) + split mode (auto, none, wide)
typedef std::array<int64_t, 8> GemmKey;
constexpr int kGemmVariants = 12;
void gemm_tune_record(bool on);
std::vector<GemmKey> gemm_tune_recorded();
void gemm_tune_set(const std::vector<GemmKey>& keys, const std::vector<int>& variants);
double gemm_tune_time(hipStream_t s, const GemmKey& key, int variant, int reps);  // ms; < 0: not timed
// address of the split-K workspace of a stream (0 if none): part of the buffer
// signature that a captured graph depends on
uint64_t gemm_workspace_signature(hipStream_t s);

// bfloat16 operands (stored as their 16-bit patterns), FP32 accumulation and output:
// C[m][n] = alpha * sum_k A[m][k] B[n][k] + beta * C[m][n].  Both operands are
// K-contiguous rows; K, lda and ldb are multiples of kBf16K (the caller zero-pads
// the columns past the true contraction length).
constexpr int64_t kBf16K = 64;
inline int64_t bf16_ld(int64_t k) { return (k + kBf16K - 1) / kBf16K * kBf16K; }
struct GemmBf16Desc {
  int64_t M = 0, N = 0, K = 0;
  float alpha = 1, beta = 0;
  const uint16_t* A = nullptr;
  int64_t lda = 0;
  const uint16_t* B = nullptr;
  int64_t ldb = 0;
  float* C = nullptr;
  int64_t ldc = 0;
  int tag = 0;      // 1: the particle-particle ladder, 2: its W slab build, 3: ring products
  // 0: by shape; 1: 128 x 128 tiles; 2: 256 x 256 tiles (M, N >= 256); 3: 256 x 256, rotated
  // k-steps (tile order by shape); 4, 5: variant 3 with the tile order M-fastest / in groups
  // of 8 tile columns
  int variant = 0;
  bool no_split = false;  // never split K (the split partials live in an allocated workspace)
};
void gemm_bf16(const GemmBf16Desc& d, hipStream_t s);
// the 256 x 256-tile kernel (gemm_bf16.hip) and the shapes it takes
bool gemm_bf16_big_fits(int64_t M, int64_t N);
// nsplit > 1: K split over grid.y, partials alpha A B^T into ws[split][M][N] (the caller sums them)
void gemm_bf16_big(const GemmBf16Desc& d, hipStream_t s, bool rotated, int group, int nsplit = 1,
                   float* ws = nullptr);
// average ms of one launch of a variant on scratch operands of shape M x N x K (K padded to 64)
double gemm_bf16_time(hipStream_t s, int64_t M, int64_t N, int64_t K, int variant, int reps);

// Grouped GEMM: many independent products of different shapes in one launch.
// Operand addresses are offsets from per-launch base pointers, so a descriptor
// table built once can be reused for different vectors.
struct GroupDesc {
  int64_t M, N, K;
  int64_t offA, lda, offB, ldb, offC, ldc;
  int64_t tile_start;  // filled by gemm_grouped_prepare
  int32_t tiles_m, pad;
};
struct GroupTable {
  GroupDesc* d = nullptr;  // device copy
  int n = 0;
  int64_t total_tiles = 0;
  bool ta = false, tb = false;
  GroupTable() = default;
  GroupTable(const GroupTable&) = delete;
  GroupTable& operator=(const GroupTable&) = delete;
  ~GroupTable() {
    if (d) (void)hipFree(d);
  }
};
// fill tile_start / tiles_m and upload (synchronous)
void gemm_grouped_prepare(std::vector<GroupDesc>& g, bool ta, bool tb, GroupTable& t);
// C_g = alpha op(A_g) op(B_g) + beta C_g for every group g
void gemm_grouped(const GroupTable& t, double alpha, const double* A, const double* B, double beta, double* C,
                  hipStream_t s);

// convenience: plain row-major C = alpha op(A) op(B) + beta C with leading dims = widths
template <typename T>
inline void mm(hipStream_t s, bool ta, bool tb, int64_t M, int64_t N, int64_t K, T alpha, const T* A,
               const T* B, T beta, T* C) {
  GemmDesc<T> d;
  d.ta = ta; d.tb = tb; d.M = M; d.N = N; d.K = K; d.alpha = alpha; d.beta = beta;
  d.A = A; d.lda = ta ? M : K;
  d.B = B; d.ldb = tb ? K : N;
  d.C = C; d.ldc = N;
  gemm(d, s);
}

// ----------------------------------------------------------------------------- tensor ops
// out[o0,o1,o2,o3] (strides os*) = alpha * in[o0*is0 + o1*is1 + o2*is2 + o3*is3] + beta * out,
// repeated for nb batches at input / output offsets ibs, obs
struct Perm4 {
  int64_t d[4];
  int64_t is[4];
  int64_t os[4];
  int64_t nb = 1, ibs = 0, obs = 0;
};
void permute4(hipStream_t s, const Perm4& p, double alpha, const double* in, double beta, double* out);
// contiguous output of a permuted contiguous input: out axes taken from input axes perm[]
void permute_c(hipStream_t s, const int64_t in_dims[4], const int perm[4], double alpha, const double* in,
               double beta, double* out, int64_t nb = 1);
void axpby(hipStream_t s, int64_t n, double alpha, const double* x, double beta, double* y);
void fill(hipStream_t s, int64_t n, double val, double* y);
void to_float(hipStream_t s, int64_t n, const double* x, float* y);
void to_double(hipStream_t s, int64_t n, const float* x, double* y, double beta);

}  // namespace pnoeom
