// Closed-shell CCSD ground state: the projected amplitude equations and the CC energy
// (paper, Methods: the CC energy and the projected equations of the ground state), solved
// by Jacobi steps with orbital-energy denominators accelerated by Pulay's DIIS.
//
// Residual.  With T1 absorbed into the similarity dressing, the doubles residual is a
// quadratic polynomial in T2 at the dressed Hamiltonian H~ and the singles residual is
// affine in T2:
//   Omega2(T2) = c2 + l2(T2) + q2(T2, T2),   Omega1(T2) = c1 + l1(T2),
// with c1 = f~_ai and c2 = (ai|bj)~.  The sigma of an R with R1 = 0, built around amplitudes
// T', is l2(R) + q2(T', R) + q2(R, T') (and l1(R)): the polarised form of the same
// polynomial.  Built around T' = T2 / 2 and applied to R = T2 it gives l2(T2) + q2(T2, T2),
// so the residual is one sigma of the existing contractions plus the two constant terms:
//   Omega(T1, T2) = (c1, c2) + sigma[T1, T2 / 2](0, T2).
// The energy is E_CC - E_ref = sum_ijab [2 (ia|jb) - (ib|ja)] (t_ij^ab + t_i^a t_j^b)
// (f_ia = 0 for the canonical reference).
#include <cmath>
#include <vector>

#include "context.h"

namespace pnoeom {
namespace {

constexpr int kRedThreads = 256;
constexpr int kRedBlocks = 1024;

unsigned grid_of(int64_t n) {
  int64_t g = (n + 255) / 256;
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>(g, 1 << 16));
}

__device__ double block_sum(double x, double* sh) {
  sh[threadIdx.x] = x;
  __syncthreads();
  for (int w = kRedThreads / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  return sh[0];
}

__device__ double block_max(double x, double* sh) {
  sh[threadIdx.x] = x;
  __syncthreads();
  for (int w = kRedThreads / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + w]);
    __syncthreads();
  }
  return sh[0];
}

// partial[blockIdx] = sum over this block's grid-stride share of x[k] * y[k]
__global__ void __launch_bounds__(kRedThreads) dot_partial_kernel(int64_t n, const double* __restrict__ x,
                                                                  const double* __restrict__ y,
                                                                  double* __restrict__ partial) {
  __shared__ double sh[kRedThreads];
  double acc = 0.0;
  for (int64_t k = blockIdx.x * (int64_t)kRedThreads + threadIdx.x; k < n; k += (int64_t)gridDim.x * kRedThreads)
    acc += x[k] * y[k];
  const double s = block_sum(acc, sh);
  if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

__global__ void __launch_bounds__(kRedThreads) maxabs_partial_kernel(int64_t n, const double* __restrict__ x,
                                                                     double* __restrict__ partial) {
  __shared__ double sh[kRedThreads];
  double acc = 0.0;
  for (int64_t k = blockIdx.x * (int64_t)kRedThreads + threadIdx.x; k < n; k += (int64_t)gridDim.x * kRedThreads)
    acc = fmax(acc, fabs(x[k]));
  const double s = block_max(acc, sh);
  if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

// partial sums of [2 (ia|jb) - (ib|ja)] (t_ij^ab + t_i^a t_j^b); G[(i,a),(j,b)] = (ia|jb)
__global__ void __launch_bounds__(kRedThreads) energy_partial_kernel(int o, int v, const double* __restrict__ G,
                                                                     const double* __restrict__ t1,
                                                                     const double* __restrict__ t2,
                                                                     double* __restrict__ partial) {
  __shared__ double sh[kRedThreads];
  const int64_t ov = (int64_t)o * v, n = ov * ov;
  double acc = 0.0;
  for (int64_t k = blockIdx.x * (int64_t)kRedThreads + threadIdx.x; k < n; k += (int64_t)gridDim.x * kRedThreads) {
    // k enumerates t2 as [i][j][a][b]
    const int b = (int)(k % v);
    const int a = (int)((k / v) % v);
    const int64_t ij = k / ((int64_t)v * v);
    const int j = (int)(ij % o), i = (int)(ij / o);
    const double L = 2.0 * G[((int64_t)i * v + a) * ov + (int64_t)j * v + b] -
                     G[((int64_t)i * v + b) * ov + (int64_t)j * v + a];
    acc += L * (t2[k] + t1[(int64_t)i * v + a] * t1[(int64_t)j * v + b]);
  }
  const double s = block_sum(acc, sh);
  if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

// r1[i][a] += f~_(o+a),i   (c1: the vo block of the dressed Fock matrix)
__global__ void add_fvo_kernel(int o, int v, int nmo, const double* __restrict__ fd, double* __restrict__ r1) {
  const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (k >= (int64_t)o * v) return;
  const int i = (int)(k / v), a = (int)(k % v);
  r1[k] += fd[(int64_t)(o + a) * nmo + i];
}

// Jacobi step on the packed amplitudes x = [t1 | t2] with residual w = [Omega1 | Omega2]:
// s = w / D, xn = x + s, D = eps_i - eps_a (singles), eps_i + eps_j - eps_a - eps_b (doubles)
__global__ void jacobi_kernel(int o, int v, const double* __restrict__ eps, const double* __restrict__ w,
                              const double* __restrict__ x, double* __restrict__ s, double* __restrict__ xn) {
  const int64_t ov = (int64_t)o * v, n = ov + ov * ov;
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x) {
    double d;
    if (k < ov) {
      d = eps[k / v] - eps[o + k % v];
    } else {
      const int64_t e = k - ov;
      const int b = (int)(e % v);
      const int a = (int)((e / v) % v);
      const int64_t ij = e / ((int64_t)v * v);
      d = eps[ij / o] + eps[ij % o] - eps[o + a] - eps[o + b];
    }
    const double st = w[k] / d;
    s[k] = st;
    xn[k] = x[k] + st;
  }
}

struct CcsdWork {
  DBuf<double> th, z1, M, part;
  std::vector<double> hpart;
};

double reduce_host(hipStream_t s, CcsdWork& w, int nblk, bool is_max) {
  w.hpart.resize(nblk);
  PNO_HIP(hipMemcpyAsync(w.hpart.data(), w.part, nblk * sizeof(double), hipMemcpyDeviceToHost, s));
  PNO_HIP(hipStreamSynchronize(s));
  double r = 0.0;
  for (int k = 0; k < nblk; ++k) r = is_max ? std::max(r, w.hpart[k]) : r + w.hpart[k];
  return r;
}

int red_blocks(int64_t n) {
  return (int)std::max<int64_t>(1, std::min<int64_t>(kRedBlocks, (n + kRedThreads - 1) / kRedThreads));
}

double dot(hipStream_t s, CcsdWork& w, int64_t n, const double* x, const double* y) {
  const int nb = red_blocks(n);
  hipLaunchKernelGGL(dot_partial_kernel, dim3(nb), dim3(kRedThreads), 0, s, n, x, y, (double*)w.part);
  PNO_HIP(hipGetLastError());
  return reduce_host(s, w, nb, false);
}

double maxabs(hipStream_t s, CcsdWork& w, int64_t n, const double* x) {
  const int nb = red_blocks(n);
  hipLaunchKernelGGL(maxabs_partial_kernel, dim3(nb), dim3(kRedThreads), 0, s, n, x, (double*)w.part);
  PNO_HIP(hipGetLastError());
  return reduce_host(s, w, nb, true);
}

// Omega(T1, T2) into r1, r2 and the correlation energy of (t1, t2).  Leaves the context
// with the intermediates of (T1, T2 / 2); the caller rebuilds or invalidates them.
double residual(Context& c, CcsdWork& w, const double* B, const double* eps, const double* t1, const double* t2,
                double* r1, double* r2) {
  hipStream_t s = c.stream;
  const int o = c.o, v = c.v;
  const int64_t ov = c.ov(), oovv = c.oovv();
  w.th.alloc(oovv);
  w.z1.alloc(ov);
  w.M.alloc(oovv);
  w.part.alloc(kRedBlocks);
  axpby(s, oovv, 0.5, t2, 0.0, w.th);
  fill(s, ov, 0.0, w.z1);
  build_df(c, B, eps, t1, w.th, PNOEOM_FP64);
  sigma_block(c, 1, w.z1, t2, r1, r2, ov, oovv, PNOEOM_FP64);
  // c1 = f~_ai
  hipLaunchKernelGGL(add_fvo_kernel, dim3(grid_of(ov)), dim3(256), 0, s, o, v, c.nmo, (const double*)c.fd, r1);
  PNO_HIP(hipGetLastError());
  // c2 = (ai|bj)~ = sum_Q B~^Q_ai B~^Q_bj: [(i,a),(j,b)], added as [i][j][a][b]
  mm<double>(s, false, true, ov, ov, c.naux, 1.0, c.BvoT, c.BvoT, 0.0, w.M);
  {
    const int64_t dims[4] = {o, v, o, v};
    const int pp[4] = {0, 2, 1, 3};
    permute_c(s, dims, pp, 1.0, w.M, 1.0, r2);
  }
  // energy from the bare (= dressed) (ia|jb) of the context
  const int nb = red_blocks(oovv);
  hipLaunchKernelGGL(energy_partial_kernel, dim3(nb), dim3(kRedThreads), 0, s, o, v, (const double*)c.G, t1, t2,
                     (double*)w.part);
  PNO_HIP(hipGetLastError());
  return reduce_host(s, w, nb, false);
}

// solves A x = b (n x n, row-major, copied) by Gaussian elimination with partial pivoting;
// false when a pivot vanishes relative to the largest entry
bool small_solve(int n, std::vector<double> A, std::vector<double>& b) {
  double big = 0.0;
  for (double x : A) big = std::max(big, std::fabs(x));
  for (int k = 0; k < n; ++k) {
    int p = k;
    for (int r = k + 1; r < n; ++r)
      if (std::fabs(A[r * n + k]) > std::fabs(A[p * n + k])) p = r;
    if (!(std::fabs(A[p * n + k]) > 1e-300 + 1e-15 * big)) return false;
    if (p != k) {
      for (int j = 0; j < n; ++j) std::swap(A[k * n + j], A[p * n + j]);
      std::swap(b[k], b[p]);
    }
    for (int r = k + 1; r < n; ++r) {
      const double f = A[r * n + k] / A[k * n + k];
      for (int j = k; j < n; ++j) A[r * n + j] -= f * A[k * n + j];
      b[r] -= f * b[k];
    }
  }
  for (int k = n - 1; k >= 0; --k) {
    double acc = b[k];
    for (int j = k + 1; j < n; ++j) acc -= A[k * n + j] * b[j];
    b[k] = acc / A[k * n + k];
  }
  return true;
}

// Marks the context's intermediates invalid when the scope is left without done(): the
// iterations build them around T2 / 2, which sigma must never use.
struct InvalidateUnlessDone {
  Context& c;
  bool ok = false;
  explicit InvalidateUnlessDone(Context& cc) : c(cc) {}
  void done() { ok = true; }
  ~InvalidateUnlessDone() {
    if (!ok) {
      c.have_df = false;
      c.have_lad = false;
    }
  }
};

}  // namespace

double ccsd_residual(Context& c, const double* B, const double* eps, const double* t1, const double* t2,
                     double* r1, double* r2) {
  InvalidateUnlessDone guard(c);  // never done: the intermediates are those of T2 / 2
  CcsdWork w;
  return residual(c, w, B, eps, t1, t2, r1, r2);
}

CcsdResult ccsd_solve(Context& c, const double* B, const double* eps, double* t1, double* t2, bool start_mp1,
                      const pnoeom_ccsd_opts& opt) {
  hipStream_t s = c.stream;
  const int o = c.o, v = c.v;
  const int64_t ov = c.ov(), oovv = c.oovv(), N = ov + oovv;
  const int m = std::max(1, opt.diis_size);
  const bool gs = opt.gs_tcut_pno >= 0.0;  // ground-state PNO simulation
  CcsdWork w;
  InvalidateUnlessDone guard(c);  // done only after the final build at the solution
  // the build-time temporaries stay allocated across the repeated builds of the iteration
  struct KeepTmp {
    Context& c;
    explicit KeepTmp(Context& cc) : c(cc) { c.keep_build_tmp = true; }
    ~KeepTmp() { c.keep_build_tmp = false; }
  } keep(c);
  DBuf<double> x, r;
  x.alloc(N);
  r.alloc(N);
  if (start_mp1 || gs) {
    // the first-order T2 that build_df forms when no T2 is given: the start, and the guess
    // amplitudes of the ground-state pair densities
    build_df(c, B, eps, nullptr, nullptr, PNOEOM_FP64);
    if (gs) {
      const double tosv = opt.gs_tcut_osv < 0.0 ? opt.gs_tcut_pno / 10.0 : opt.gs_tcut_osv;
      build_gs_pnos(c, c.T, opt.gs_tcut_pno, tosv);
    }
  }
  if (!gs) c.gs.reset();  // ground-state PNOs of an earlier simulation describe other amplitudes
  if (start_mp1) {
    fill(s, ov, 0.0, x);
    PNO_HIP(hipMemcpyAsync(x + ov, c.T, oovv * sizeof(double), hipMemcpyDeviceToDevice, s));
  } else {
    PNO_HIP(hipMemcpyAsync(x, t1, ov * sizeof(double), hipMemcpyDeviceToDevice, s));
    PNO_HIP(hipMemcpyAsync(x + ov, t2, oovv * sizeof(double), hipMemcpyDeviceToDevice, s));
  }
  // the iterated vector: the canonical amplitudes, or (PNO simulation) their components in
  // the semicanonical OSV / PNO basis (the start projected onto that space); DIIS runs on it
  PNOData& P = c.gs;
  const int64_t Nd = gs ? P.len : N;
  DBuf<double> xb, rb, X, E;
  if (gs) {
    xb.alloc(Nd);
    rb.alloc(Nd);
    pno_compress(c, P, 1, x, x + ov, xb);
    project_pno(c, P, xb);
  }
  double* xs = gs ? (double*)xb : (double*)x;
  X.alloc((int64_t)m * Nd);
  E.alloc((int64_t)m * Nd);
  CcsdResult res;
  std::vector<double> gram((size_t)m * m, 0.0);
  int stored = 0;
  double e_prev = INFINITY;
  for (int it = 0;; ++it) {
    TraceRange tr_("ccsd step");
    if (gs) pno_expand(c, P, 1, xs, x, x + ov);
    const double e = residual(c, w, B, eps, x, x + ov, r, r + ov);
    if (gs) pno_compress(c, P, 1, r, r + ov, rb);
    const double* rs = gs ? (const double*)rb : (const double*)r;
    const double rmax = maxabs(s, w, Nd, rs);
    res.energies.push_back(e);
    res.resmax.push_back(rmax);
    res.e_corr = e;
    res.rmax = rmax;
    res.iters = it;
    if (!std::isfinite(e) || !std::isfinite(rmax)) break;
    if (rmax < opt.tol_r && std::fabs(e - e_prev) < opt.tol_e) {
      res.converged = true;
      break;
    }
    if (it == opt.max_iter) break;
    // Jacobi step into DIIS slot k (the oldest entry is overwritten once m are stored)
    const int k = it % m;
    double* Xk = X + (int64_t)k * Nd;
    double* Ek = E + (int64_t)k * Nd;
    if (gs) {
      // step in the semicanonical OSV / PNO basis: rbar / (f_ii (+ f_jj) - fbar_a (- fbar_b))
      PNO_HIP(hipMemcpyAsync(Ek, rs, Nd * sizeof(double), hipMemcpyDeviceToDevice, s));
      precond_pno(c, P, Ek, 0.0);
      PNO_HIP(hipMemcpyAsync(Xk, xs, Nd * sizeof(double), hipMemcpyDeviceToDevice, s));
      axpby(s, Nd, 1.0, Ek, 1.0, Xk);
    } else {
      hipLaunchKernelGGL(jacobi_kernel, dim3(grid_of(N)), dim3(256), 0, s, o, v, (const double*)c.eps,
                         (const double*)r, (const double*)x, Ek, Xk);
      PNO_HIP(hipGetLastError());
    }
    stored = std::min(stored + 1, m);
    for (int l = 0; l < stored; ++l) {
      const double g = dot(s, w, Nd, Ek, E + (int64_t)l * Nd);
      gram[(size_t)k * m + l] = gram[(size_t)l * m + k] = g;
    }
    bool extrapolated = false;
    if (stored > 1) {
      // the Gram block is normalised by its largest diagonal entry (the coefficients do not
      // change), so that the pivots stay comparable to the unit border near convergence
      const int n = stored + 1;
      double gmax = 0.0;
      for (int a = 0; a < stored; ++a) gmax = std::max(gmax, gram[(size_t)a * m + a]);
      std::vector<double> A((size_t)n * n, 0.0), rhs(n, 0.0);
      for (int a = 0; a < stored; ++a) {
        for (int b = 0; b < stored; ++b) A[(size_t)a * n + b] = gmax > 0.0 ? gram[(size_t)a * m + b] / gmax : 0.0;
        A[(size_t)a * n + stored] = A[(size_t)stored * n + a] = -1.0;
      }
      rhs[stored] = -1.0;
      if (small_solve(n, A, rhs)) {
        axpby(s, Nd, rhs[0], X, 0.0, xs);
        for (int l = 1; l < stored; ++l) axpby(s, Nd, rhs[l], X + (int64_t)l * Nd, 1.0, xs);
        extrapolated = true;
      }
    }
    if (!extrapolated) PNO_HIP(hipMemcpyAsync(xs, Xk, Nd * sizeof(double), hipMemcpyDeviceToDevice, s));
    e_prev = e;
  }
  if (gs) pno_expand(c, P, 1, xs, x, x + ov);
  PNO_HIP(hipMemcpyAsync(t1, x, ov * sizeof(double), hipMemcpyDeviceToDevice, s));
  PNO_HIP(hipMemcpyAsync(t2, x + ov, oovv * sizeof(double), hipMemcpyDeviceToDevice, s));
  c.keep_build_tmp = false;
  if (!std::isfinite(res.e_corr) || !std::isfinite(res.rmax)) {
    // diverged: the amplitudes are returned as they are, and the context is left without
    // intermediates (the guard marks them invalid) rather than holding them at non-finite T
    for (DBuf<double>& b : c.btmp) b.release();
    c.sw.release();
    c.gs.reset();  // ground-state PNOs built in this call come from the same diverged run
    PNO_HIP(hipStreamSynchronize(s));
    return res;
  }
  // intermediates of the final amplitudes, in the contraction precision asked for (this
  // build releases the temporaries)
  build_df(c, B, eps, t1, t2, opt.precision);
  PNO_HIP(hipStreamSynchronize(s));
  guard.done();
  return res;
}

}  // namespace pnoeom
