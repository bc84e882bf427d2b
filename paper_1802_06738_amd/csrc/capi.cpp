// C ABI of libpnoeom: argument checks, exception-to-status mapping, timing.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstring>

#include "context.h"

struct pnoeom_ctx {
  pnoeom::Context c;
};

namespace {

template <typename F>
int guarded(pnoeom_ctx* ctx, F&& f) {
  if (!ctx) return PNOEOM_EINVAL;
  try {
    ctx->c.err.clear();
    f(ctx->c);
    return PNOEOM_OK;
  } catch (const pnoeom::Error& e) {
    ctx->c.err = e.what();
    (void)hipGetLastError();  // do not let a reported failure resurface in the next call
    return e.code;
  } catch (const std::exception& e) {
    ctx->c.err = e.what();
    return PNOEOM_EHIP;
  } catch (...) {
    ctx->c.err = "unknown error";
    return PNOEOM_EHIP;
  }
}

struct Timer {
  pnoeom::Context& c;
  hipEvent_t a = nullptr, b = nullptr;
  explicit Timer(pnoeom::Context& cc) : c(cc) {
    c.last_ladder_ms = 0;
    c.last_ladder_launches = 0;
    c.ladder_flops = 0;
    c.ladder_kernel_launches = 0;
    for (int r = 0; r < pnoeom::Context::kRegions; ++r) {
      c.reg_flops[r] = c.reg_bytes[r] = 0;
      c.reg_launches[r] = 0;
      c.last_reg_ms[r] = c.last_reg_flops[r] = c.last_reg_bytes[r] = 0;
      c.last_reg_launches[r] = 0;
    }
    for (int p = 0; p < 3; ++p) {
      c.ladder_flops_p[p] = 0;
      c.ladder_launches_p[p] = 0;
      c.last_ladder_ms_p[p] = 0;
      c.last_ladder_flops_p[p] = 0;
      c.last_ladder_launches_p[p] = 0;
    }
    c.timing = true;
    c.ev_used = 0;
    c.ev_prec.clear();
    PNO_HIP(hipEventCreate(&a));
    PNO_HIP(hipEventCreate(&b));
    PNO_HIP(hipEventRecord(a, c.stream));
  }
  void stop() {
    PNO_HIP(hipEventRecord(b, c.stream));
    PNO_HIP(hipEventSynchronize(b));
    float ms = 0.f;
    PNO_HIP(hipEventElapsedTime(&ms, a, b));
    c.last_total_ms = ms;
    double lad = 0.0;
    for (size_t k = 0; k + 1 < c.ev_used; k += 2) {
      float t = 0.f;
      PNO_HIP(hipEventElapsedTime(&t, c.ev_pool[k], c.ev_pool[k + 1]));
      const int cat = k / 2 < c.ev_prec.size() ? c.ev_prec[k / 2] : 0;
      if (cat < 3) {
        lad += t;
        c.last_ladder_ms_p[cat] += t;
      } else {
        c.last_reg_ms[cat - 3] += t;
      }
    }
    for (int r = 0; r < pnoeom::Context::kRegions; ++r) {
      c.last_reg_flops[r] = c.reg_flops[r];
      c.last_reg_bytes[r] = c.reg_bytes[r];
      c.last_reg_launches[r] = c.reg_launches[r];
    }
    c.last_ladder_ms = lad;
    c.last_ladder_launches = c.ladder_kernel_launches;
    c.last_ladder_flops = c.ladder_flops;
    for (int p = 0; p < 3; ++p) {
      c.last_ladder_flops_p[p] = c.ladder_flops_p[p];
      c.last_ladder_launches_p[p] = c.ladder_launches_p[p];
    }
  }
  ~Timer() {
    c.timing = false;
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
  }
};

}  // namespace

extern "C" {

int pnoeom_create(int o, int v, int naux, void* hip_stream, pnoeom_ctx** out) {
  if (!out) return PNOEOM_EINVAL;
  *out = nullptr;
  if (o < 1 || v < 1 || naux < 1) return PNOEOM_EINVAL;
  pnoeom_ctx* ctx = new (std::nothrow) pnoeom_ctx();
  if (!ctx) return PNOEOM_ENOMEM;
  ctx->c.o = o;
  ctx->c.v = v;
  ctx->c.naux = naux;
  ctx->c.nmo = o + v;
  ctx->c.stream = (hipStream_t)hip_stream;
  *out = ctx;
  return PNOEOM_OK;
}

void pnoeom_destroy(pnoeom_ctx* ctx) {
  if (!ctx) return;
  delete ctx;  // the context's destructor releases its graphs, events, stream and buffers
}

const char* pnoeom_last_error(const pnoeom_ctx* ctx) { return ctx ? ctx->c.err.c_str() : "null context"; }

int pnoeom_build_df(pnoeom_ctx* ctx, const double* B, const double* eps, const double* t1, const double* t2,
                    int precision) {
  return guarded(ctx, [&](pnoeom::Context& c) {
    pnoeom::TraceRange tr_("pnoeom_build_df");
    PNO_CHECK(B && eps, PNOEOM_EINVAL, "build_df: B and eps are required");
    PNO_CHECK(precision == PNOEOM_FP64 || precision == PNOEOM_FP32 || precision == PNOEOM_BF16, PNOEOM_EINVAL,
              "build_df: precision must be PNOEOM_FP64, PNOEOM_FP32 or PNOEOM_BF16");
    pnoeom::build_df(c, B, eps, t1, t2, precision);
  });
}

int pnoeom_cis(pnoeom_ctx* ctx, int nroots, double* omega_out, double* vec_out) {
  return guarded(ctx, [&](pnoeom::Context& c) {
    pnoeom::TraceRange tr_("pnoeom_cis");
    PNO_CHECK(omega_out, PNOEOM_EINVAL, "cis: omega_out is required");
    pnoeom::cis_roots(c, nroots, omega_out, vec_out);
  });
}

int pnoeom_build_sapno(pnoeom_ctx* ctx, int nstates, double tcut_pno, double tcut_osv, int* npno_out,
                       int* nosv_out) {
  return guarded(ctx, [&](pnoeom::Context& c) {
    pnoeom::TraceRange tr_("pnoeom_build_sapno");
    PNO_CHECK(c.have_df, PNOEOM_ESTATE, "build_sapno before build_df");
    PNO_CHECK(nstates >= 1 && tcut_pno >= 0.0, PNOEOM_EINVAL, "build_sapno: bad arguments");
    pnoeom::build_sapno(c, nstates, tcut_pno, tcut_osv < 0 ? tcut_pno / 10.0 : tcut_osv);
    const int np = c.o * (c.o + 1) / 2;
    if (npno_out) std::memcpy(npno_out, c.pno.npno.data(), np * sizeof(int));
    if (nosv_out) std::memcpy(nosv_out, c.pno.nosv.data(), c.o * sizeof(int));
  });
}

int pnoeom_pno_layout(const pnoeom_ctx* cctx, long long* offsets, long long* len) {
  pnoeom_ctx* ctx = const_cast<pnoeom_ctx*>(cctx);
  return guarded(ctx, [&](pnoeom::Context& c) {
    PNO_CHECK(c.pno.built, PNOEOM_ESTATE, "pno_layout before build_sapno");
    if (len) *len = c.pno.len;
    if (offsets)
      for (size_t k = 0; k < c.pno.off.size(); ++k) offsets[k] = c.pno.off[k];
  });
}

int pnoeom_pno_transform(pnoeom_ctx* ctx, int nvec, int direction, double* r1, double* r2, double* x) {
  return guarded(ctx, [&](pnoeom::Context& c) {
    pnoeom::TraceRange tr_("pnoeom_pno_transform");
    PNO_CHECK(c.pno.built, PNOEOM_ESTATE, "pno_transform before build_sapno");
    PNO_CHECK(nvec >= 0 && (direction == 0 || direction == 1), PNOEOM_EINVAL, "pno_transform: bad arguments");
    PNO_CHECK(r1 && r2 && x, PNOEOM_EINVAL, "pno_transform: null pointer");
    if (direction == 0)
      pnoeom::pno_compress(c, nvec, r1, r2, x);
    else
      pnoeom::pno_expand(c, nvec, x, r1, r2);
    PNO_HIP(hipStreamSynchronize(c.stream));
  });
}

int pnoeom_apply_sigma(pnoeom_ctx* ctx, int nvec, const double* r1, const double* r2, double* s1, double* s2,
                       int space, int precision) {
  return guarded(ctx, [&](pnoeom::Context& c) {
    pnoeom::TraceRange tr_("pnoeom_apply_sigma");
    PNO_CHECK(c.have_df, PNOEOM_ESTATE, "apply_sigma before build_df");
    PNO_CHECK(nvec >= 0, PNOEOM_EINVAL, "apply_sigma: nvec < 0");
    PNO_CHECK(precision == PNOEOM_FP64 || precision == PNOEOM_FP32 || precision == PNOEOM_BF16, PNOEOM_EINVAL,
              "apply_sigma: precision must be PNOEOM_FP64, PNOEOM_FP32 or PNOEOM_BF16");
    PNO_CHECK(space == PNOEOM_CANONICAL || space == PNOEOM_PNO, PNOEOM_EINVAL, "apply_sigma: bad space");
    if (nvec == 0) return;
    Timer t(c);
    if (space == PNOEOM_CANONICAL) {
      PNO_CHECK(r1 && r2 && s1 && s2, PNOEOM_EINVAL, "apply_sigma: null vector pointer");
      if (c.graph_mode) {
        // packed [r1 | r2] vectors for the captured path
        const int64_t ov = c.ov(), oovv = c.oovv(), N = ov + oovv;
        if ((int64_t)c.pack_in.n < nvec * N) c.pack_in.alloc(nvec * N);
        if ((int64_t)c.pack_out.n < nvec * N) c.pack_out.alloc(nvec * N);
        for (int q = 0; q < nvec; ++q) {
          PNO_HIP(hipMemcpyAsync(c.pack_in + q * N, r1 + q * ov, ov * sizeof(double), hipMemcpyDeviceToDevice,
                                 c.stream));
          PNO_HIP(hipMemcpyAsync(c.pack_in + q * N + ov, r2 + q * oovv, oovv * sizeof(double),
                                 hipMemcpyDeviceToDevice, c.stream));
        }
        pnoeom::sigma_apply(c, PNOEOM_CANONICAL, nvec, c.pack_in, c.pack_out, N, precision);
        for (int q = 0; q < nvec; ++q) {
          PNO_HIP(hipMemcpyAsync(s1 + q * ov, c.pack_out + q * N, ov * sizeof(double), hipMemcpyDeviceToDevice,
                                 c.stream));
          PNO_HIP(hipMemcpyAsync(s2 + q * oovv, c.pack_out + q * N + ov, oovv * sizeof(double),
                                 hipMemcpyDeviceToDevice, c.stream));
        }
      } else {
        pnoeom::sigma_block(c, nvec, r1, r2, s1, s2, c.ov(), c.oovv(), precision);
      }
    } else {
      PNO_CHECK(c.pno.built, PNOEOM_ESTATE, "apply_sigma(PNO) before build_sapno");
      PNO_CHECK(r1 && s1, PNOEOM_EINVAL, "apply_sigma: null vector pointer");
      pnoeom::sigma_apply(c, PNOEOM_PNO, nvec, r1, s1, c.pno.len, precision);
    }
    t.stop();
  });
}

int pnoeom_set_ring_mode(pnoeom_ctx* ctx, int mode) {
  return guarded(ctx, [&](pnoeom::Context& c) {
    PNO_CHECK(mode >= 0 && mode <= 2, PNOEOM_EINVAL, "set_ring_mode: unknown mode");
    c.ring_mode = mode;
  });
}

int pnoeom_davidson_phase(const pnoeom_ctx* ctx, int phase, int cap, double* omega_out, double* resnorm_out,
                          int* iters_out, int* nsigma_out, double* seconds_out) {
  if (!ctx || phase < 0 || phase > 1 || cap < 0) return PNOEOM_EINVAL;
  const pnoeom::Context::PhaseRecord& pr = ctx->c.dav_phase[phase];
  if (pr.n == 0) return PNOEOM_ESTATE;
  for (int k = 0; k < cap && k < pr.n; ++k) {
    if (omega_out) omega_out[k] = pr.omega[k];
    if (resnorm_out) resnorm_out[k] = k < (int)pr.resnorm.size() ? pr.resnorm[k] : 0.0;
  }
  if (iters_out) *iters_out = pr.iters;
  if (nsigma_out) *nsigma_out = pr.nsigma;
  if (seconds_out) *seconds_out = pr.seconds;
  return PNOEOM_OK;
}

int pnoeom_set_bf16_passes(pnoeom_ctx* ctx, int passes) {
  return guarded(ctx, [&](pnoeom::Context& c) {
    PNO_CHECK(passes == 1 || passes == 3, PNOEOM_EINVAL, "set_bf16_passes: 1 or 3");
    c.ring_passes = passes;
  });
}

int pnoeom_set_bf16_scope(pnoeom_ctx* ctx, int scope) {
  return guarded(ctx, [&](pnoeom::Context& c) {
    PNO_CHECK(scope == 0 || scope == 1, PNOEOM_EINVAL, "set_bf16_scope: 0 or 1");
    c.bf16_scope = scope;
  });
}

int pnoeom_ring_mode_used(const pnoeom_ctx* ctx) {
  if (!ctx) return PNOEOM_EINVAL;
  if (!ctx->c.have_df) return PNOEOM_ESTATE;
  return ctx->c.ring_y ? 2 : 1;
}

int pnoeom_set_ladder_mode(pnoeom_ctx* ctx, int mode, int max_slab) {
  return guarded(ctx, [&](pnoeom::Context& c) {
    PNO_CHECK(mode == PNOEOM_LADDER_AUTO || mode == PNOEOM_LADDER_CACHED || mode == PNOEOM_LADDER_STREAMED,
              PNOEOM_EINVAL, "set_ladder_mode: unknown mode");
    PNO_CHECK(max_slab >= 0, PNOEOM_EINVAL, "set_ladder_mode: max_slab < 0");
    c.lad_mode = mode;
    c.lad_max_slab = max_slab;
  });
}

int pnoeom_build_ladder(pnoeom_ctx* ctx, const double* B, const double* t1, int precision) {
  return guarded(ctx, [&](pnoeom::Context& c) {
    pnoeom::TraceRange tr_("pnoeom_build_ladder");
    PNO_CHECK(B, PNOEOM_EINVAL, "build_ladder: B is required");
    PNO_CHECK(precision == PNOEOM_FP64 || precision == PNOEOM_FP32 || precision == PNOEOM_BF16, PNOEOM_EINVAL,
              "build_ladder: precision must be PNOEOM_FP64, PNOEOM_FP32 or PNOEOM_BF16");
    pnoeom::build_ladder(c, B, t1, precision, pnoeom::ladder_budget());
  });
}

int pnoeom_ladder_apply(pnoeom_ctx* ctx, int nmat, const double* X, double* Y, int precision) {
  return guarded(ctx, [&](pnoeom::Context& c) {
    pnoeom::TraceRange tr_("pnoeom_ladder_apply");
    PNO_CHECK(nmat >= 0, PNOEOM_EINVAL, "ladder_apply: nmat < 0");
    if (nmat == 0) return;
    PNO_CHECK(X && Y, PNOEOM_EINVAL, "ladder_apply: null matrix pointer");
    const int64_t vv = (int64_t)c.v * c.v;
    PNO_CHECK(X + nmat * vv <= Y || Y + nmat * vv <= X, PNOEOM_EINVAL, "ladder_apply: X and Y overlap");
    Timer t(c);
    pnoeom::ladder_apply(c, nmat, X, Y, precision);
    t.stop();
  });
}

int pnoeom_ladder_apply_noalloc(pnoeom_ctx* ctx, int nmat, const double* X, double* Y, int precision) {
  return guarded(ctx, [&](pnoeom::Context& c) {
    pnoeom::TraceRange tr_("pnoeom_ladder_apply_noalloc");
    PNO_CHECK(nmat >= 0, PNOEOM_EINVAL, "ladder_apply_noalloc: nmat < 0");
    if (nmat == 0) return;
    PNO_CHECK(X && Y, PNOEOM_EINVAL, "ladder_apply_noalloc: null matrix pointer");
    const int64_t vv = (int64_t)c.v * c.v;
    PNO_CHECK(X + nmat * vv <= Y || Y + nmat * vv <= X, PNOEOM_EINVAL, "ladder_apply_noalloc: X and Y overlap");
    pnoeom::ladder_apply_noalloc(c, nmat, X, Y, precision);
  });
}

long long pnoeom_ladder_noalloc_limit(const pnoeom_ctx* ctx, int precision) {
  if (!ctx || precision < PNOEOM_FP64 || precision > PNOEOM_BF16) return -1;
  // the staging size grows with nmat: bisection for the largest count that fits
  int64_t lo = 0, hi = 1 << 30;
  while (lo < hi) {
    const int64_t mid = lo + (hi - lo + 1) / 2;
    if (pnoeom::ladder_noalloc_bytes(ctx->c, (int)mid, precision) <= pnoeom::kNoAllocScratchBytes)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

int pnoeom_set_pno_states(pnoeom_ctx* ctx, int n, const int* states) {
  return guarded(ctx, [&](pnoeom::Context& c) {
    PNO_CHECK(n >= 0 && (n == 0 || states), PNOEOM_EINVAL, "set_pno_states: bad list");
    std::vector<int> l(states, states + n);
    std::vector<int> sorted = l;
    std::sort(sorted.begin(), sorted.end());
    PNO_CHECK(n == 0 || (sorted.front() >= 0 && std::adjacent_find(sorted.begin(), sorted.end()) == sorted.end()),
              PNOEOM_EINVAL, "set_pno_states: indices must be distinct and >= 0");
    c.pno.states = l;
  });
}

int pnoeom_set_pno_ladder(pnoeom_ctx* ctx, int max_native) {
  return guarded(ctx, [&](pnoeom::Context& c) {
    PNO_CHECK(max_native >= -1, PNOEOM_EINVAL, "set_pno_ladder: max_native < -1");
    c.pno.nat_max = max_native;
  });
}

int pnoeom_pno_ladder_stats(const pnoeom_ctx* ctx, int* cut, int* native_pairs, int* canonical_pairs,
                            double* native_flops) {
  if (!ctx) return PNOEOM_EINVAL;
  if (!ctx->c.pno.built) return PNOEOM_ESTATE;
  if (cut) *cut = ctx->c.pno.nat_cut;
  if (native_pairs) *native_pairs = ctx->c.pno.nat_pairs;
  if (canonical_pairs) *canonical_pairs = ctx->c.pno.canon_pairs;
  if (native_flops) *native_flops = ctx->c.pno.nat_flops;
  return PNOEOM_OK;
}

int pnoeom_set_graph_mode(pnoeom_ctx* ctx, int enable) {
  return guarded(ctx, [&](pnoeom::Context& c) {
    c.graph_mode = enable != 0;
    if (!c.graph_mode) c.drop_graphs();
  });
}

int pnoeom_graph_stats(const pnoeom_ctx* ctx, int* captures, int* launches, int* cached) {
  if (!ctx) return PNOEOM_EINVAL;
  if (captures) *captures = ctx->c.graph_captures;
  if (launches) *launches = ctx->c.graph_launches;
  if (cached) *cached = (int)ctx->c.graphs.size();
  return PNOEOM_OK;
}

void pnoeom_davidson_defaults(pnoeom_davidson_opts* opts) {
  if (!opts) return;
  opts->space = PNOEOM_CANONICAL;
  opts->precision = PNOEOM_FP64;
  opts->tol_e = 1e-8;
  opts->tol_r = 1e-5;
  opts->max_sub = 60;
  opts->max_iter = 200;
  opts->refine_fp64 = 0;
  opts->verbose = 0;
  opts->nextra = 0;
  opts->mixed_tol_e = 0.0;
  opts->mixed_tol_r = 0.0;
  opts->ckpt_every = 0;
  opts->abort_after_iter = 0;
  opts->ckpt_path = nullptr;
  opts->resume_path = nullptr;
  opts->log_path = nullptr;
}

void pnoeom_ccsd_defaults(pnoeom_ccsd_opts* opts) {
  if (!opts) return;
  opts->max_iter = 100;
  opts->tol_e = 1e-10;
  opts->tol_r = 1e-8;
  opts->diis_size = 8;
  opts->precision = PNOEOM_FP64;
  opts->gs_tcut_pno = -1.0;
  opts->gs_tcut_osv = -1.0;
}

int pnoeom_ccsd_residual(pnoeom_ctx* ctx, const double* B, const double* eps, const double* t1, const double* t2,
                         double* r1_out, double* r2_out, double* e_corr_out) {
  return guarded(ctx, [&](pnoeom::Context& c) {
    pnoeom::TraceRange tr_("pnoeom_ccsd_residual");
    PNO_CHECK(B && eps && t1 && t2 && r1_out && r2_out && e_corr_out, PNOEOM_EINVAL,
              "ccsd_residual: null pointer");
    *e_corr_out = pnoeom::ccsd_residual(c, B, eps, t1, t2, r1_out, r2_out);
  });
}

int pnoeom_ccsd(pnoeom_ctx* ctx, const double* B, const double* eps, double* t1, double* t2, int start,
                const pnoeom_ccsd_opts* opts, double* e_corr_out, double* resmax_out, int* iters_out) {
  bool converged = false;
  const int st = guarded(ctx, [&](pnoeom::Context& c) {
    pnoeom::TraceRange tr_("pnoeom_ccsd");
    pnoeom_ccsd_opts o;
    pnoeom_ccsd_defaults(&o);
    if (opts) o = *opts;
    PNO_CHECK(B && eps && t1 && t2 && e_corr_out, PNOEOM_EINVAL, "ccsd: null pointer");
    PNO_CHECK(start == 0 || start == 1, PNOEOM_EINVAL, "ccsd: start must be 0 (MP1) or 1 (given amplitudes)");
    PNO_CHECK(o.max_iter >= 0 && o.tol_e > 0.0 && o.tol_r > 0.0 && o.diis_size >= 0 && o.diis_size <= 64,
              PNOEOM_EINVAL, "ccsd: bad options");
    PNO_CHECK(o.precision == PNOEOM_FP64 || o.precision == PNOEOM_FP32 || o.precision == PNOEOM_BF16,
              PNOEOM_EINVAL, "ccsd: bad precision");
    const pnoeom::CcsdResult r = pnoeom::ccsd_solve(c, B, eps, t1, t2, start == 0, o);
    *e_corr_out = r.e_corr;
    if (resmax_out) *resmax_out = r.rmax;
    if (iters_out) *iters_out = r.iters;
    c.ccsd_energies = r.energies;
    c.ccsd_resmax = r.resmax;
    converged = r.converged;
    if (!converged) c.err = "ccsd: not converged";
  });
  if (st != PNOEOM_OK) return st;
  return converged ? PNOEOM_OK : PNOEOM_ENOTCONV;
}

int pnoeom_ccsd_gs_counts(const pnoeom_ctx* ctx, int* npno_out, int* nosv_out) {
  if (!ctx) return PNOEOM_EINVAL;
  const pnoeom::Context& c = ctx->c;
  if (!c.gs.built) return PNOEOM_ESTATE;
  if (npno_out)
    for (size_t p = 0; p < c.gs.npno.size(); ++p) npno_out[p] = c.gs.npno[p];
  if (nosv_out)
    for (size_t i = 0; i < c.gs.nosv.size(); ++i) nosv_out[i] = c.gs.nosv[i];
  return PNOEOM_OK;
}

int pnoeom_ccsd_history(const pnoeom_ctx* ctx, int cap, double* energies, double* resmax, int* n_out) {
  if (!ctx || !n_out || cap < 0 || (cap > 0 && (!energies || !resmax))) return PNOEOM_EINVAL;
  const pnoeom::Context& c = ctx->c;
  const int n = (int)c.ccsd_energies.size();
  *n_out = n;
  for (int k = 0; k < std::min(n, cap); ++k) {
    energies[k] = c.ccsd_energies[k];
    resmax[k] = c.ccsd_resmax[k];
  }
  return PNOEOM_OK;
}

int pnoeom_davidson(pnoeom_ctx* ctx, int nroots, const pnoeom_davidson_opts* opts, double* omega_out,
                    double* resnorm_out, int* iters_out, int* nsigma_out) {
  int complex_pair = 0;
  int converged = 1;
  int aborted = 0;
  int st = guarded(ctx, [&](pnoeom::Context& c) {
    pnoeom::TraceRange tr_("pnoeom_davidson");
    PNO_CHECK(opts && omega_out, PNOEOM_EINVAL, "davidson: opts and omega_out are required");
    Timer t(c);
    pnoeom::DavidsonResult r = pnoeom::davidson(c, nroots, *opts);
    t.stop();
    for (int k = 0; k < nroots; ++k) {
      omega_out[k] = k < (int)r.omega.size() ? r.omega[k] : 0.0;
      if (resnorm_out) resnorm_out[k] = k < (int)r.resnorm.size() ? r.resnorm[k] : 0.0;
    }
    if (iters_out) *iters_out = r.iters;
    if (nsigma_out) *nsigma_out = r.nsigma;
    complex_pair = r.complex_pair;
    converged = r.converged;
    aborted = r.aborted;
    if (aborted)
      c.err = "Davidson stopped at abort_after_iter";
    else if (!converged)
      c.err = "Davidson did not converge within max_iter";
  });
  if (st != PNOEOM_OK) return st;
  if (aborted) return PNOEOM_EABORTED;
  if (!converged) return PNOEOM_ENOTCONV;
  if (complex_pair) return PNOEOM_ECOMPLEX;
  return PNOEOM_OK;
}

int pnoeom_probe_peaks(pnoeom_ctx* ctx, double* fp64_tflops, double* fp32_tflops, double* bf16_tflops,
                       double* copy_gbs) {
  return guarded(ctx, [&](pnoeom::Context& c) {
    pnoeom::probe_peaks(c.stream, fp64_tflops, fp32_tflops, bf16_tflops, copy_gbs);
  });
}

int pnoeom_gemm_record(int enable) {
  pnoeom::gemm_tune_record(enable != 0);
  return PNOEOM_OK;
}

int pnoeom_gemm_recorded(long long* keys, int cap) {
  const std::vector<pnoeom::GemmKey> k = pnoeom::gemm_tune_recorded();
  if (keys)
    for (int i = 0; i < (int)k.size() && i < cap; ++i)
      for (int j = 0; j < 8; ++j) keys[(size_t)i * 8 + j] = (long long)k[i][j];
  return (int)k.size();
}

int pnoeom_gemm_time(void* hip_stream, const long long* key, int variant, int reps, double* ms) {
  if (!key || !ms || reps < 1) return PNOEOM_EINVAL;
  try {
    pnoeom::GemmKey k;
    for (int j = 0; j < 8; ++j) k[j] = key[j];
    *ms = pnoeom::gemm_tune_time((hipStream_t)hip_stream, k, variant, reps);
    return PNOEOM_OK;
  } catch (const pnoeom::Error& e) {
    (void)hipGetLastError();
    return e.code;
  } catch (...) {
    (void)hipGetLastError();
    return PNOEOM_EHIP;
  }
}

int pnoeom_gemm_bf16(void* hip_stream, long long M, long long N, long long K, float alpha, const void* A,
                     long long lda, const void* B, long long ldb, float beta, float* C, long long ldc, int variant) {
  try {
    pnoeom::GemmBf16Desc d;
    d.M = M; d.N = N; d.K = K; d.alpha = alpha; d.beta = beta;
    d.A = (const uint16_t*)A; d.lda = lda; d.B = (const uint16_t*)B; d.ldb = ldb; d.C = C; d.ldc = ldc;
    d.variant = variant;
    PNO_CHECK(M >= 0 && N >= 0 && K >= 0 && ldc >= N, PNOEOM_EINVAL, "gemm_bf16: bad shape");
    pnoeom::gemm_bf16(d, (hipStream_t)hip_stream);
    return PNOEOM_OK;
  } catch (const pnoeom::Error& e) {
    (void)hipGetLastError();
    return e.code;
  } catch (...) {
    (void)hipGetLastError();
    return PNOEOM_EHIP;
  }
}

int pnoeom_gemm_bf16_time(void* hip_stream, long long M, long long N, long long K, int variant, int reps,
                          double* ms) {
  if (!ms) return PNOEOM_EINVAL;
  try {
    *ms = pnoeom::gemm_bf16_time((hipStream_t)hip_stream, M, N, K, variant, reps);
    return PNOEOM_OK;
  } catch (const pnoeom::Error& e) {
    (void)hipGetLastError();
    return e.code;
  } catch (...) {
    (void)hipGetLastError();
    return PNOEOM_EHIP;
  }
}

int pnoeom_gemm_set_table(int n, const long long* keys, const int* variants) {
  if (n < 0 || (n > 0 && (!keys || !variants))) return PNOEOM_EINVAL;
  std::vector<pnoeom::GemmKey> k(n);
  std::vector<int> v(n);
  for (int i = 0; i < n; ++i) {
    if (variants[i] < 0 || variants[i] >= pnoeom::kGemmVariants) return PNOEOM_EINVAL;
    for (int j = 0; j < 8; ++j) k[i][j] = keys[(size_t)i * 8 + j];
    v[i] = variants[i];
  }
  pnoeom::gemm_tune_set(k, v);
  return PNOEOM_OK;
}

int pnoeom_sigma_memory(pnoeom_ctx* ctx, int space, int precision, long long* per_vector, long long* avail,
                        int* chunk) {
  return guarded(ctx, [&](pnoeom::Context& c) {
    PNO_CHECK(c.have_df, PNOEOM_ESTATE, "sigma_memory before build_df");
    PNO_CHECK(precision == PNOEOM_FP64 || precision == PNOEOM_FP32 || precision == PNOEOM_BF16, PNOEOM_EINVAL,
              "sigma_memory: bad precision");
    PNO_CHECK(space == PNOEOM_CANONICAL || space == PNOEOM_PNO, PNOEOM_EINVAL, "sigma_memory: bad space");
    PNO_CHECK(space == PNOEOM_CANONICAL || c.pno.built, PNOEOM_ESTATE, "sigma_memory: PNO space before build_sapno");
    const int64_t per = pnoeom::sigma_bytes_per_vector(c, precision, space == PNOEOM_PNO);
    size_t freeb = 0, totalb = 0;
    PNO_HIP(hipMemGetInfo(&freeb, &totalb));
    const int64_t av = (int64_t)freeb + pnoeom::sigma_held_bytes(c) - pnoeom::sigma_headroom((int64_t)totalb);
    if (per_vector) *per_vector = per;
    if (avail) *avail = av;
    if (chunk) *chunk = (int)std::max<int64_t>(1, av > 0 ? av / per : 0);
  });
}

int pnoeom_set_eig_backend(pnoeom_ctx* ctx, int backend) {
  return guarded(ctx, [&](pnoeom::Context& c) {
    PNO_CHECK(backend == 0 || backend == 1, PNOEOM_EINVAL, "set_eig_backend: backend must be 0 or 1");
    c.eig_backend = backend;
  });
}

int pnoeom_syev_batched(pnoeom_ctx* ctx, int nmat, int n, double* a, double cut, double* ev, double* vt) {
  return guarded(ctx, [&](pnoeom::Context& c) {
    PNO_CHECK(nmat >= 0 && n >= 1, PNOEOM_EINVAL, "syev_batched: nmat < 0 or n < 1");
    if (nmat == 0) return;
    PNO_CHECK(a && ev && vt, PNOEOM_EINVAL, "syev_batched: null pointer");
    std::vector<int> nsz(nmat, n);
    pnoeom::DBuf<int> dn;
    dn.alloc(nmat);
    pnoeom::batched_syev(c.stream, c.eig_backend, nmat, nsz, n, a, vt, ev, dn, cut);
  });
}

int pnoeom_host_syev(int n, const double* a, double* w, double* v) {
  try {
    return pnoeom::host_syev(n, a, w, v);
  } catch (...) {
    return PNOEOM_EINVAL;
  }
}

int pnoeom_host_eig(int n, const double* a, double* wr, double* wi, double* vr) {
  try {
    return pnoeom::host_eig(n, a, wr, wi, vr);
  } catch (...) {
    return PNOEOM_EHIP;
  }
}

int pnoeom_last_timing(const pnoeom_ctx* ctx, double* total_ms, double* ladder_ms, int* ladder_launches,
                       double* ladder_flops) {
  if (!ctx) return PNOEOM_EINVAL;
  if (ladder_flops) *ladder_flops = ctx->c.last_ladder_flops;
  if (total_ms) *total_ms = ctx->c.last_total_ms;
  if (ladder_ms) *ladder_ms = ctx->c.last_ladder_ms;
  if (ladder_launches) *ladder_launches = ctx->c.last_ladder_launches;
  return PNOEOM_OK;
}

int pnoeom_last_region_timing(const pnoeom_ctx* ctx, int region, double* ms, int* launches, double* flops,
                              double* bytes) {
  if (!ctx) return PNOEOM_EINVAL;
  if (region < 0 || region >= pnoeom::Context::kRegions) return PNOEOM_EINVAL;
  if (ms) *ms = ctx->c.last_reg_ms[region];
  if (launches) *launches = ctx->c.last_reg_launches[region];
  if (flops) *flops = ctx->c.last_reg_flops[region];
  if (bytes) *bytes = ctx->c.last_reg_bytes[region];
  return PNOEOM_OK;
}

int pnoeom_last_ladder_timing(const pnoeom_ctx* ctx, int precision, double* ladder_ms, int* ladder_launches,
                              double* ladder_flops) {
  if (!ctx) return PNOEOM_EINVAL;
  if (precision < PNOEOM_FP64 || precision > PNOEOM_BF16) return PNOEOM_EINVAL;
  if (ladder_ms) *ladder_ms = ctx->c.last_ladder_ms_p[precision];
  if (ladder_launches) *ladder_launches = ctx->c.last_ladder_launches_p[precision];
  if (ladder_flops) *ladder_flops = ctx->c.last_ladder_flops_p[precision];
  return PNOEOM_OK;
}

}  // extern "C"
