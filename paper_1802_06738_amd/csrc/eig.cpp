// Dense real non-symmetric eigenproblem for the small Davidson subspace matrix.
//
// 1. Householder reduction to upper Hessenberg form.
// 2. Francis implicit double-shift QR iteration on the active window with
//    deflation of negligible subdiagonals (eigenvalues only).
// 3. Right eigenvectors by inverse iteration on the original matrix (complex
//    arithmetic for complex pairs; one LU factorisation per eigenvalue, three
//    solves), re-orthogonalised against the vectors of numerically coincident
//    eigenvalues; only for the first nvec eigenvalues in sorted order when asked.
#include <algorithm>
#include <cfloat>
#include <cmath>
#include <complex>
#include <atomic>
#include <numeric>
#include <thread>
#include <vector>

#include "../../include/pnoeom.h"

namespace pnoeom {
namespace {

typedef std::complex<double> cd;

void hessenberg(int n, std::vector<double>& H) {
  auto h = [&](int i, int j) -> double& { return H[(size_t)i * n + j]; };
  std::vector<double> u(n);
  for (int k = 0; k < n - 2; ++k) {
    double alpha = 0.0;
    for (int i = k + 1; i < n; ++i) alpha += h(i, k) * h(i, k);
    alpha = std::sqrt(alpha);
    if (alpha == 0.0) continue;
    if (h(k + 1, k) > 0) alpha = -alpha;
    double unorm2 = 0.0;
    for (int i = k + 1; i < n; ++i) {
      u[i] = h(i, k);
      if (i == k + 1) u[i] -= alpha;
      unorm2 += u[i] * u[i];
    }
    if (unorm2 == 0.0) continue;
    const double beta = 2.0 / unorm2;
    // H <- P H  (rows k+1..n-1)
    for (int j = k; j < n; ++j) {
      double s = 0.0;
      for (int i = k + 1; i < n; ++i) s += u[i] * h(i, j);
      s *= beta;
      for (int i = k + 1; i < n; ++i) h(i, j) -= s * u[i];
    }
    // H <- H P  (columns k+1..n-1)
    for (int i = 0; i < n; ++i) {
      double s = 0.0;
      for (int j = k + 1; j < n; ++j) s += h(i, j) * u[j];
      s *= beta;
      for (int j = k + 1; j < n; ++j) h(i, j) -= s * u[j];
    }
    for (int i = k + 2; i < n; ++i) h(i, k) = 0.0;
  }
}

// Householder reflector v = x - alpha e1 for a 2- or 3-vector; returns beta = 2/v.v (0: skip)
double reflector(double& x, double& y, double& z, int len, double& v0, double& v1, double& v2) {
  const double nrm = std::sqrt(x * x + y * y + (len == 3 ? z * z : 0.0));
  if (nrm == 0.0) return 0.0;
  const double alpha = (x >= 0) ? -nrm : nrm;
  v0 = x - alpha;
  v1 = y;
  v2 = (len == 3) ? z : 0.0;
  const double vv = v0 * v0 + v1 * v1 + v2 * v2;
  return vv == 0.0 ? 0.0 : 2.0 / vv;
}

bool francis(int n, std::vector<double>& H, double* wr, double* wi) {
  auto h = [&](int i, int j) -> double& { return H[(size_t)i * n + j]; };
  double anorm = 0.0;
  for (double x : H) anorm = std::max(anorm, std::fabs(x));
  if (anorm == 0.0) anorm = 1.0;
  int p = n - 1;
  int its = 0;
  while (p >= 0) {
    int l = p;
    for (; l > 0; --l) {
      double s = std::fabs(h(l - 1, l - 1)) + std::fabs(h(l, l));
      if (s == 0.0) s = anorm;
      if (std::fabs(h(l, l - 1)) <= DBL_EPSILON * s) {
        h(l, l - 1) = 0.0;
        break;
      }
    }
    if (l == p) {
      wr[p] = h(p, p);
      wi[p] = 0.0;
      --p;
      its = 0;
      continue;
    }
    if (l == p - 1) {
      const double a = h(p - 1, p - 1), b = h(p - 1, p), c = h(p, p - 1), d = h(p, p);
      const double m = 0.5 * (a + d);
      const double disc = 0.25 * (a - d) * (a - d) + b * c;
      if (disc >= 0.0) {
        const double sq = std::sqrt(disc);
        const double l1 = m + (m >= 0 ? sq : -sq);
        const double det = a * d - b * c;
        const double l2 = (l1 != 0.0) ? det / l1 : m - sq;
        wr[p - 1] = l1;
        wr[p] = l2;
        wi[p - 1] = wi[p] = 0.0;
      } else {
        const double sq = std::sqrt(-disc);
        wr[p - 1] = wr[p] = m;
        wi[p - 1] = sq;
        wi[p] = -sq;
      }
      p -= 2;
      its = 0;
      continue;
    }
    if (++its > 60 * n) return false;
    double ssum, sprod;
    if (its % 11 == 0) {  // exceptional shift to break a cycle
      const double w = std::fabs(h(p, p - 1)) + std::fabs(h(p - 1, p - 2));
      ssum = 1.5 * w;
      sprod = w * w;
    } else {
      ssum = h(p - 1, p - 1) + h(p, p);
      sprod = h(p - 1, p - 1) * h(p, p) - h(p - 1, p) * h(p, p - 1);
    }
    double x = h(l, l) * h(l, l) + h(l, l + 1) * h(l + 1, l) - ssum * h(l, l) + sprod;
    double y = h(l + 1, l) * (h(l, l) + h(l + 1, l + 1) - ssum);
    double z = h(l + 1, l) * h(l + 2, l + 1);
    for (int k = l; k <= p - 2; ++k) {
      double v0, v1, v2;
      const double beta = reflector(x, y, z, 3, v0, v1, v2);
      if (beta != 0.0) {
        const int c0 = (k > l) ? k - 1 : l;
        for (int j = c0; j <= p; ++j) {
          const double s = beta * (v0 * h(k, j) + v1 * h(k + 1, j) + v2 * h(k + 2, j));
          h(k, j) -= s * v0;
          h(k + 1, j) -= s * v1;
          h(k + 2, j) -= s * v2;
        }
        const int rmax = std::min(k + 3, p);
        for (int i = l; i <= rmax; ++i) {
          const double s = beta * (v0 * h(i, k) + v1 * h(i, k + 1) + v2 * h(i, k + 2));
          h(i, k) -= s * v0;
          h(i, k + 1) -= s * v1;
          h(i, k + 2) -= s * v2;
        }
      }
      x = h(k + 1, k);
      y = h(k + 2, k);
      if (k < p - 2) z = h(k + 3, k);
    }
    {
      const int k = p - 1;
      double v0, v1, v2, zz = 0.0;
      const double beta = reflector(x, y, zz, 2, v0, v1, v2);
      if (beta != 0.0) {
        for (int j = k - 1; j <= p; ++j) {
          const double s = beta * (v0 * h(k, j) + v1 * h(k + 1, j));
          h(k, j) -= s * v0;
          h(k + 1, j) -= s * v1;
        }
        for (int i = l; i <= p; ++i) {
          const double s = beta * (v0 * h(i, k) + v1 * h(i, k + 1));
          h(i, k) -= s * v0;
          h(i, k + 1) -= s * v1;
        }
      }
    }
  }
  return true;
}

// LU factorisation with partial pivoting (complex, in place); tiny pivots are replaced
// by tiny * scale so that a (nearly) singular shifted matrix still yields the
// inverse-iteration direction.
void lu_factor(int n, std::vector<cd>& M, std::vector<int>& piv, double tiny) {
  piv.resize(n);
  for (int k = 0; k < n; ++k) {
    int pr = k;
    double best = std::abs(M[(size_t)k * n + k]);
    for (int i = k + 1; i < n; ++i) {
      const double a = std::abs(M[(size_t)i * n + k]);
      if (a > best) { best = a; pr = i; }
    }
    piv[k] = pr;
    if (pr != k)
      for (int j = 0; j < n; ++j) std::swap(M[(size_t)k * n + j], M[(size_t)pr * n + j]);
    if (std::abs(M[(size_t)k * n + k]) < tiny) M[(size_t)k * n + k] = tiny;
    const cd d = M[(size_t)k * n + k];
    for (int i = k + 1; i < n; ++i) {
      cd& f = M[(size_t)i * n + k];
      f /= d;
      if (f == cd(0.0)) continue;
      for (int j = k + 1; j < n; ++j) M[(size_t)i * n + j] -= f * M[(size_t)k * n + j];
    }
  }
}

// solve with the factors of lu_factor (b overwritten by x)
void lu_solve(int n, const std::vector<cd>& M, const std::vector<int>& piv, std::vector<cd>& b) {
  for (int k = 0; k < n; ++k) {
    if (piv[k] != k) std::swap(b[k], b[piv[k]]);
    for (int i = k + 1; i < n; ++i) b[i] -= M[(size_t)i * n + k] * b[k];
  }
  for (int i = n - 1; i >= 0; --i) {
    cd s = b[i];
    for (int j = i + 1; j < n; ++j) s -= M[(size_t)i * n + j] * b[j];
    b[i] = s / M[(size_t)i * n + i];
  }
}

}  // namespace

int host_eig(int n, const double* a, double* wr, double* wi, double* vr, int nvec) {
  if (n < 1 || !a || !wr || !wi) return PNOEOM_EINVAL;
  if (nvec < 0 || nvec > n) nvec = n;
  std::vector<double> H(a, a + (size_t)n * n);
  hessenberg(n, H);
  std::vector<double> er(n), ei(n);
  if (!francis(n, H, er.data(), ei.data())) return PNOEOM_ENOTCONV;
  std::vector<int> ord(n);
  std::iota(ord.begin(), ord.end(), 0);
  std::stable_sort(ord.begin(), ord.end(), [&](int x, int y) {
    if (er[x] != er[y]) return er[x] < er[y];
    return ei[x] > ei[y];
  });
  for (int k = 0; k < n; ++k) {
    wr[k] = er[ord[k]];
    wi[k] = ei[ord[k]];
  }
  if (!vr) return PNOEOM_OK;
  double anorm = 0.0;
  for (int i = 0; i < n * n; ++i) anorm = std::max(anorm, std::fabs(a[i]));
  if (anorm == 0.0) anorm = 1.0;
  const double tiny = anorm * 1e-14;
  std::vector<std::vector<double>> done;
  std::vector<double> done_lam;
  std::fill(vr, vr + (size_t)n * n, 0.0);
  std::vector<cd> M((size_t)n * n);
  std::vector<int> piv;
  for (int k = 0; k < nvec; ++k) {
    const cd lam(wr[k], wi[k]);
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) M[(size_t)i * n + j] = cd(a[(size_t)i * n + j], 0.0) - (i == j ? lam : cd(0.0));
    lu_factor(n, M, piv, tiny);
    std::vector<cd> x(n);
    for (int i = 0; i < n; ++i) x[i] = cd(1.0 + 0.01 * ((i * 7919) % 101), 0.0);
    for (int it = 0; it < 3; ++it) {
      lu_solve(n, M, piv, x);
      // keep away from vectors already found for (numerically) the same eigenvalue
      if (wi[k] == 0.0) {
        for (size_t q = 0; q < done.size(); ++q) {
          if (std::fabs(done_lam[q] - wr[k]) > 1e-9 * anorm) continue;
          cd dot = 0.0;
          for (int i = 0; i < n; ++i) dot += done[q][i] * x[i];
          for (int i = 0; i < n; ++i) x[i] -= dot * done[q][i];
        }
      }
      double nrm = 0.0;
      for (int i = 0; i < n; ++i) nrm += std::norm(x[i]);
      nrm = std::sqrt(nrm);
      if (nrm == 0.0) nrm = 1.0;
      for (int i = 0; i < n; ++i) x[i] /= nrm;
    }
    // fix the phase so that the largest component is real and positive
    int imax = 0;
    for (int i = 1; i < n; ++i)
      if (std::abs(x[i]) > std::abs(x[imax])) imax = i;
    const cd ph = std::conj(x[imax]) / std::abs(x[imax]);
    std::vector<double> re(n);
    double nrm = 0.0;
    for (int i = 0; i < n; ++i) {
      re[i] = (x[i] * ph).real();
      nrm += re[i] * re[i];
    }
    nrm = std::sqrt(nrm);
    for (int i = 0; i < n; ++i) vr[(size_t)i * n + k] = re[i] / nrm;
    if (wi[k] == 0.0) {
      done.push_back(std::vector<double>(re.begin(), re.end()));
      for (double& y : done.back()) y /= nrm;
      done_lam.push_back(wr[k]);
    }
  }
  return PNOEOM_OK;
}

// ----------------------------------------------------------------------------- symmetric
// Real symmetric eigensolver for the large per-pair density matrices of the PNO build:
// Householder reduction to tridiagonal form (A = Q T Q^T, reflectors I - 2 v v^T with
// unit v, trailing block updated as A <- A - 2 (v q^T + q v^T), q = A v - (v^T A v) v),
// backward accumulation of Q, then the implicit symmetric QR iteration with the
// Wilkinson shift of the trailing 2 x 2 block, chasing the bulge with Givens rotations
// G = [[c, s], [-s, c]] (T <- G^T T G, Z <- Z G) and deflating when
// |t_{k,k+1}| <= eps (|t_kk| + |t_{k+1,k+1}|).
namespace {

int syev_one(int n, double* a, double* w, double* z) {
  // a: n x n row-major symmetric (destroyed); w: eigenvalues; z: n x n, column k = vector k
  std::vector<double> d(n), e(n > 1 ? n - 1 : 1, 0.0);
  std::vector<std::vector<double>> vs(n > 2 ? n - 2 : 0);
  std::vector<double> p(n), q(n);
  for (int k = 0; k + 2 < n; ++k) {
    const int m = n - k - 1;
    double* row = a + (int64_t)k * n + k + 1;
    double sig = 0.0;
    for (int i = 0; i < m; ++i) sig += row[i] * row[i];
    sig = std::sqrt(sig);
    d[k] = a[(int64_t)k * n + k];
    if (sig == 0.0) {
      e[k] = 0.0;
      continue;
    }
    const double alpha = row[0] >= 0.0 ? -sig : sig;
    std::vector<double>& v = vs[k];
    v.assign(row, row + m);
    v[0] -= alpha;
    double vn = 0.0;
    for (int i = 0; i < m; ++i) vn += v[i] * v[i];
    vn = std::sqrt(vn);
    if (vn == 0.0) {
      v.clear();
      e[k] = row[0];
      continue;
    }
    for (int i = 0; i < m; ++i) v[i] /= vn;
    e[k] = alpha;
    // p = A' v over the trailing block (rows / columns k+1..n-1)
    double kap = 0.0;
    for (int i = 0; i < m; ++i) {
      const double* ar = a + (int64_t)(k + 1 + i) * n + k + 1;
      double acc = 0.0;
      for (int j = 0; j < m; ++j) acc += ar[j] * v[j];
      p[i] = acc;
      kap += v[i] * acc;
    }
    for (int i = 0; i < m; ++i) q[i] = p[i] - kap * v[i];
    for (int i = 0; i < m; ++i) {
      double* ar = a + (int64_t)(k + 1 + i) * n + k + 1;
      const double vi = 2.0 * v[i], qi = 2.0 * q[i];
      for (int j = 0; j < m; ++j) ar[j] -= vi * q[j] + qi * v[j];
    }
  }
  if (n >= 2) {
    d[n - 2] = a[(int64_t)(n - 2) * n + n - 2];
    e[n - 2] = a[(int64_t)(n - 2) * n + n - 1];
  }
  d[n - 1] = a[(int64_t)(n - 1) * n + n - 1];
  // Z = H_0 H_1 ... H_{n-3}, accumulated backwards on rows k+1..n-1
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) z[(int64_t)i * n + j] = i == j ? 1.0 : 0.0;
  for (int k = n - 3; k >= 0; --k) {
    const std::vector<double>& v = vs[k];
    if (v.empty()) continue;
    const int m = n - k - 1;
    // rows k+1.. of Z have nonzeros only in columns k+1..n-1
    std::fill(p.begin(), p.end(), 0.0);
    for (int i = 0; i < m; ++i) {
      const double* zr = z + (int64_t)(k + 1 + i) * n + k + 1;
      for (int j = 0; j < m; ++j) p[j] += v[i] * zr[j];
    }
    for (int i = 0; i < m; ++i) {
      double* zr = z + (int64_t)(k + 1 + i) * n + k + 1;
      const double vi = 2.0 * v[i];
      for (int j = 0; j < m; ++j) zr[j] -= vi * p[j];
    }
  }
  // implicit symmetric QR on (d, e); Z columns rotated along
  int hi = n - 1, iters = 0;
  const int max_iters = 60 * n + 100;
  while (hi > 0) {
    if (std::fabs(e[hi - 1]) <= DBL_EPSILON * (std::fabs(d[hi - 1]) + std::fabs(d[hi]))) {
      e[hi - 1] = 0.0;
      --hi;
      continue;
    }
    int lo = hi - 1;
    while (lo > 0 && std::fabs(e[lo - 1]) > DBL_EPSILON * (std::fabs(d[lo - 1]) + std::fabs(d[lo]))) --lo;
    if (++iters > max_iters) return PNOEOM_ENOTCONV;
    const double dd = 0.5 * (d[hi - 1] - d[hi]);
    const double bb = e[hi - 1];
    const double den = dd + (dd >= 0.0 ? 1.0 : -1.0) * std::hypot(dd, bb);
    const double mu = den != 0.0 ? d[hi] - bb * bb / den : d[hi] - std::fabs(bb);
    double x = d[lo] - mu, y = e[lo];
    for (int k = lo; k < hi; ++k) {
      const double r = std::hypot(x, y);
      double c = 1.0, s = 0.0;
      if (r != 0.0) {
        c = x / r;
        s = -y / r;
      }
      if (k > lo) e[k - 1] = r;
      const double pk = d[k], qk = d[k + 1], tk = e[k];
      d[k] = c * c * pk - 2.0 * c * s * tk + s * s * qk;
      d[k + 1] = s * s * pk + 2.0 * c * s * tk + c * c * qk;
      e[k] = c * s * (pk - qk) + (c * c - s * s) * tk;
      if (k + 1 < hi) {
        y = -s * e[k + 1];
        e[k + 1] = c * e[k + 1];
        x = e[k];
      }
      for (int i = 0; i < n; ++i) {
        double* zr = z + (int64_t)i * n;
        const double zk = zr[k], zk1 = zr[k + 1];
        zr[k] = c * zk - s * zk1;
        zr[k + 1] = s * zk + c * zk1;
      }
    }
  }
  for (int i = 0; i < n; ++i) w[i] = d[i];
  return PNOEOM_OK;
}

}  // namespace

int host_syev(int n, const double* a, double* w, double* v) {
  if (n < 1 || !a || !w || !v) return PNOEOM_EINVAL;
  std::vector<double> work(a, a + (int64_t)n * n);
  return syev_one(n, work.data(), w, v);
}

int host_syev_batched(int nmat, const int* nsz, int ld, double* A, double* ev, double* Vt, int nthreads) {
  // A[m]: nsz[m] x nsz[m] in an ld x ld slot (destroyed); ev[m*ld + k]; Vt[m] row k = eigenvector k
  if (nmat <= 0) return PNOEOM_OK;
  if (nthreads < 1) nthreads = 1;
  std::atomic<int> next(0), status(PNOEOM_OK);
  auto work = [&]() {
    std::vector<double> a, z, w;
    for (;;) {
      const int m = next.fetch_add(1);
      if (m >= nmat) break;
      const int n = nsz[m];
      if (n <= 0) continue;
      a.resize((size_t)n * n);
      z.resize((size_t)n * n);
      w.resize(n);
      const int64_t base = (int64_t)m * ld * ld;
      for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) a[(size_t)i * n + j] = A[base + (int64_t)i * ld + j];
      const int st = syev_one(n, a.data(), w.data(), z.data());
      if (st != PNOEOM_OK) status = st;
      for (int k = 0; k < n; ++k) {
        ev[(int64_t)m * ld + k] = w[k];
        for (int i = 0; i < n; ++i) Vt[base + (int64_t)k * ld + i] = z[(size_t)i * n + k];
      }
    }
  };
  std::vector<std::thread> pool;
  const int nt = std::min(nthreads, nmat);
  for (int t = 1; t < nt; ++t) pool.emplace_back(work);
  work();
  for (auto& th : pool) th.join();
  return status.load();
}

}  // namespace pnoeom
