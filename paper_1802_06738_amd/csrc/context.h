// The library context: inputs, T-dependent intermediates, PNO data and workspaces.
#pragma once

#include "common.h"

namespace pnoeom {

// Per-vector workspace of the canonical sigma (all FP64, sized once).
struct SigmaWork {
  DBuf<double> Bp, Bc, hp, Jp, Kp, fp, dp, fp_ov, fp_vv, fp_oo;  // (Bc: occupied columns of B')
  DBuf<double> BvopT, BoopT, BvvpT;
  DBuf<double> R2c, Ria, UiaR, UR;  // (R2c: R2 compacted, only for strided input)
  DBuf<double> S1p;                  // partial sums of sigma1's U(R)_ia f' term (fused BF16 mode)
  // ZZ[(q,i,a)][Ziajb row | Z3 row]; RE[(q,i,a)][R^s row | E_X row] (the stacked left operand
  // of the fused ring product; R^s rows only when the E_X products go through Yr / Zr)
  DBuf<double> ZZ, RE, Zp, Xh, O4p, OOVVp, M1;
  DBuf<double> R1c;  // the block's R1 compacted as [(q,j)][c] (ring terms through Yr / Zr)
  DBuf<double> Ftv, Fto;
  DBuf<double> LadAll, Sp, Am, SigP, SigM;  // batched packed ladder
  DBuf<float> Spf, Amf, SigPf, SigMf;
  DBuf<uint16_t> Spb, Amb;  // bfloat16 bits, rows padded to the W+/- column padding
  // BF16 fused ring product: left operand rows [-R^s | R_ia | B'_vo | M1/2] (kfold values)
  DBuf<uint16_t> RAb;
  // FP32 staging for the mixed-precision contractions
  DBuf<float> fa, fc;
  DBuf<float> fz;  // FP32 sum of the Zp terms (fused BF16 ring mode)
  DBuf<float> Sdf;  // FP32 direct block: hole ladder, X_klij T and the ladder (fused BF16 ring mode)
  void release() {
    for (DBuf<double>* b : {&Bp, &Bc, &hp, &Jp, &Kp, &fp, &dp, &fp_ov, &fp_vv, &fp_oo, &BvopT, &BoopT, &BvvpT, &R2c, &Ria,
                            &UiaR, &UR, &ZZ, &RE, &Zp, &Xh, &O4p,
                            &OOVVp, &M1, &R1c, &Ftv, &Fto, &LadAll, &Sp, &Am, &SigP, &SigM, &S1p})
      b->release();
    for (DBuf<float>* b : {&Spf, &Amf, &SigPf, &SigMf, &fa, &fc, &fz, &Sdf}) b->release();
    Spb.release();
    RAb.release();
    Amb.release();
  }
};

struct PNOData {
  bool built = false;
  int nstates = 0;
  double tcut_pno = 0, tcut_osv = 0;
  std::vector<int> npno;        // [P_o] pairs i <= j, row-major
  std::vector<int> nosv;        // [o]
  std::vector<int64_t> off;     // [o + P_o + 1] block offsets in a compressed vector
  int64_t len = 0;
  int nmax = 0;                 // largest block size
  std::vector<int64_t> uoff;    // offsets of the v x n blocks in U (pairs, then OSVs)
  std::vector<int64_t> toff;    // offsets of the per-pair v x n_p work blocks
  DBuf<double> U;               // semicanonical PNO / OSV bases, [v][n] row-major blocks
  DBuf<double> denom_base;      // per compressed element: F_ii (+ F_jj) - fbar_a (- fbar_b)
  DBuf<int64_t> d_off;          // diagonal pair blocks: offsets
  DBuf<int> d_n;                //                       sizes
  GroupTable t_c1, t_c3, t_c2d, t_c2o, t_e1, t_e3;  // compress / expand (first stage)
  DBuf<int64_t> d_xpair;        // per pair: i, j, n_p, offset of its v x n_p block in Tw, in U
  DBuf<double> Tw, r1, r2, s1, s2;
  double xf_flops = 0;          // flops of one compress (or expand) of one vector
  // ladder of the pairs with n_p <= nat_cut evaluated in the PNO space with per-pair
  // factors Bbar_p[a][Q][c] = (U_p^T B~^Q U_p)[a][c]; the other pairs keep the canonical
  // ladder (rows listed by prow: slot in the packed ladder, -1 for a native pair)
  int nat_max = -1;             // requested bound (-1 auto, 0 none)
  std::vector<int> states;      // CIS states averaged by build_sapno (empty: the lowest nstates)
  int nat_cut = 0, nat_pairs = 0, canon_pairs = 0;
  std::vector<int> prow;
  DBuf<int> d_prow;
  DBuf<int> d_slot;             // per slot of the packed ladder: i o + j of its pair (i <= j)
  DBuf<double> Bbar, Y1, Ypart;  // Ypart: split-K partial blocks of the second product
  GroupTable t_na, t_nb;
  DBuf<int> d_nn, d_nch;         // per native pair: n_p, K chunks
  DBuf<int64_t> d_poff, d_yoff;  // per native pair: first partial block, block in the compressed vector
  DBuf<int64_t> d_small;        // native pairs with n_p <= 16 (fused kernel): n, Bbar, vector, partial offsets
  int nsmall = 0;
  double nat_flops = 0;         // flops of the native ladder of one vector
  void reset() {
    built = false;
    npno.clear(); nosv.clear(); off.clear(); uoff.clear(); toff.clear();
    len = 0; nmax = 0;
    U.release(); denom_base.release(); d_off.release(); d_n.release(); d_xpair.release();
    Tw.release(); r1.release(); r2.release(); s1.release(); s2.release();
    nat_cut = nat_pairs = canon_pairs = 0;
    prow.clear(); d_prow.release(); d_slot.release(); Bbar.release(); Y1.release(); Ypart.release(); nat_flops = 0;
    d_nn.release(); d_nch.release(); d_poff.release(); d_yoff.release(); d_small.release(); nsmall = 0;
  }
};

struct Context {
  int o = 0, v = 0, naux = 0, nmo = 0;
  hipStream_t stream = nullptr;
  std::string err;
  bool have_df = false;
  int precision = PNOEOM_FP64;

  // inputs
  DBuf<double> B, eps, t1;
  // dressed Hamiltonian
  DBuf<double> Bt, h, hd, fd, dt, dtmp, J, K;
  DBuf<double> BovT, BvoT, BooT, BvvT, Bvv2;
  // amplitudes
  DBuf<double> T, U, Tia, Tsia, UiaT;
  // integrals / intermediates
  DBuf<double> G, GX, g2, Gq, OVVO, OOVVx, Wh, OOOVp;
  DBuf<double> Fqvv, Fqoo, Fvv, Foo, fd_ov;
  DBuf<double> Dr, Xr, DX2, Wvo2, YU;
  DBuf<double> BYU;  // [Q][(j,b)] = B~^Q_bj + YU[Q][(j,b)]: the right factor of the DF ring terms of B'_vo
  // ring operands, rows of 2 ov: [Dr | Xr] (rows 0..ov-1) stacked on [Tia | Tsia] (rows
  // ov..2ov-1), the right operand of the fused product [R^s | E_X] DXTT
  DBuf<double> DXTT;
  // R1-driven three-body ring terms through T-only intermediates (ring_y): with
  // TT = [T_ia | T^s_ia] (rows of 2 ov),
  //   Yr[(a,c)][2 ov] = sum_(i,b) (ic|ab)~ TT[(i,b)],   Zr[(j,l)][2 ov] = sum_(i,b) (ij|lb)~ TT[(i,b)]
  // (then DXTT holds only its [Dr | Xr] rows).  ring_mode: 0 when Yr fits, 1 never, 2 always.
  DBuf<double> Yr, Zr;
  bool ring_y = false;
  int ring_mode = 0;
  // symmetric eigenproblems above 128: 0 on the GPU (tridiagonal solver), 1 on host threads
  int eig_backend = 0;
  // BF16 ring products (precision BF16 with ring_y): right operands [Dr | Xr]^T and DX2^T as
  // bfloat16 rows of ring_passes blocks of ldr (= ov padded to 64) values: one pass takes
  // bf16(x), three passes the split x = hi + lo as [hi | lo | hi] (left operands [hi | hi | lo]),
  // so that the products sum to hi hi + hi lo + lo hi
  DBuf<uint16_t> DXb, DX2b;
  int64_t ldr = 0;
  // BF16 scope 1, one pass: right operand of the ring product fused with the DF ring terms,
  // row n = [Dr^T | DX2^T | BYU^T | YU^T] of kfold = 2 ldr + 2 ldq bfloat16 values
  DBuf<uint16_t> RBb;
  int64_t kfold = 0;
  int ring_passes = 1;
  // BF16 scope (next build_df): 0 = the ladder and the ring products on bfloat16 MFMA, the
  // other contractions FP32; 1 = also the hole ladder, X_klij, M1 and the DF and R1 ring terms
  int bf16_scope = 1;
  // packed ladder: W+[(a<=b),(c<=d)] = W_abcd + W_abdc, W-[(a<b),(c<d)] = W_abcd - W_abdc
  DBuf<double> Wp, Wm;          // FP64 (always: the FP64 sigma and the refinement of mixed runs)
  DBuf<float> Wpf, Wmf;         // FP32 (precision FP32)
  DBuf<uint16_t> Wpb, Wmb;      // bfloat16 bits (precision BF16), rows padded to ldpb / ldmb columns
  int64_t ldpb = 0, ldmb = 0;
  DBuf<float> DX2f, DXTTf;
  // FP32 copies of the T-only right factors of the hole-ladder and three-body products and of
  // B~_ov (precision FP32 / BF16: those products then run on FP32 MFMA)
  DBuf<float> Whf, g2f, T32, BovTf;
  DBuf<float> BYUf, YUf;  // FP32 copies of the DF ring factors (precision FP32 / BF16)
  // BF16 scope 1: FP32 copies of Foo, Wvo2 and Zr (Fock-type, Wvo and Zr ring terms)
  DBuf<float> Foof, Wvo2f, Zrf;
  // bfloat16 operands of the other large products in BF16 mode (rows padded to 64 values):
  // Wh [(ij)][(kl)], g2 [(kl)][(cd)], T^T [(ab)][(kl)] (hole ladder and X_klij), B~_ov as
  // [Q][(jb)] (M1), BYU^T and YU^T as [(kc)][Q] (DF ring terms, rows of ldq), and Yr with
  // its last two indices swapped, [(a, n)][c] (R1 term of the ring)
  DBuf<uint16_t> Whb, g2b, TTb, BovQb, BYUb, YUb, Yrb;
  DBuf<uint16_t> Whbs;  // the rows (i <= j) of Whb, pairs in row-major order (fused BF16 mode)
  DBuf<uint16_t> Gqb;  // Gq^T as [b][(k,l,d)] (Ftv), rows of ldg
  // T as rows [(i,j,a)][c] and Fvv without its diagonal as rows [b][c] (rows of ldv; the
  // Fock-type products T Ftv^T and R (Fvv - diag)^T), and the diagonal of Fvv
  DBuf<uint16_t> Tvb, Fvob;
  DBuf<double> Fvvd;
  DBuf<double> Food;  // diagonal of Foo (BF16 scope 1: its off-diagonal part rides in Whb)
  int64_t ldoo = 0, ldvv = 0, ldov = 0, ldv = 0, ldg = 0;
  bool bf_rest = false;
  // build-time temporaries of build_df, by slot (each slot's uses follow one another on the
  // stream); kept between builds while keep_build_tmp is set (the repeated builds of the
  // CCSD solver then allocate nothing), else released at the end of each build
  DBuf<double> btmp[4];
  bool keep_build_tmp = false;
  double* build_tmp(int slot, int64_t n) {
    if ((int64_t)btmp[slot].n < n) btmp[slot].alloc(n);
    return btmp[slot];
  }

  // ladder storage (pnoeom_set_ladder_mode): 0 auto, 1 cached W+/-, 2 streamed from B~_vv
  int lad_mode = 0, lad_max_slab = 0;
  // restricted canonical ladder (PNO sigma with native pairs): slot per pair or -1, slots per vector
  const int* lad_prow = nullptr;
  const int* lad_slot = nullptr;  // and the pair (i o + j) of each slot
  int64_t lad_nsub = -1;
  DBuf<int> slot_all;             // i o + j of every pair i <= j in ladder-slot order
  bool lad_streamed = false;    // W+/- not stored: rebuilt slab by slab in every sigma
  bool have_lad = false;        // the ladder can be applied (build_df or build_ladder done)
  DBuf<float> BvvTf;            // FP32 copy of BvvT (streamed, precision FP32)
  DBuf<uint16_t> BvvTb;         // bfloat16 copy of BvvT, rows padded to ldq columns (streamed, BF16)
  int64_t ldq = 0;
  DBuf<double> lad_tmp, lad_wp, lad_wm;  // slab workspace (raw storage, element type per precision)

  SigmaWork sw;
  PNOData pno;
  // the phases of the last Davidson call: [0] the main run (FP32 / BF16 before a refinement,
  // or the whole FP64 run), [1] the FP64 refinement; n = 0 when the phase did not run
  struct PhaseRecord {
    std::vector<double> omega, resnorm;
    int iters = 0, nsigma = 0, n = 0;
    double seconds = 0;
  } dav_phase[2];
  PNOData gs;   // ground-state PNOs / OSVs of the PNO-CCSD simulation (build_gs_pnos; build_df keeps them)

  // E_CC - E_ref and largest |Omega| of every amplitude set of the last pnoeom_ccsd
  std::vector<double> ccsd_energies, ccsd_resmax;
  // timing of the last sigma / Davidson call
  double last_total_ms = 0, last_ladder_ms = 0, last_ladder_flops = 0;
  int last_ladder_launches = 0;
  double ladder_flops = 0;          // algorithmic flops of the timed ladder launches
  int ladder_kernel_launches = 0;   // GEMM launches inside the timed ladder regions
  // the same split by contraction precision (FP64, FP32, BF16)
  double ladder_flops_p[3] = {0, 0, 0};
  int ladder_launches_p[3] = {0, 0, 0};
  double last_ladder_ms_p[3] = {0, 0, 0}, last_ladder_flops_p[3] = {0, 0, 0};
  int last_ladder_launches_p[3] = {0, 0, 0};
  std::vector<int> ev_prec;         // per start/stop event pair: ladder precision (0..2) or 3 + region
  // other timed regions: 0 = Davidson inner products, 1 = PNO back-transform / projection,
  // 2 = W slab builds of the streamed ladder (factor GEMM + pack), 3 = ring (ov)^3 products,
  // 4 = ladder of the native PNO pairs
  static constexpr int kRegions = 5;
  double reg_flops[kRegions] = {}, reg_bytes[kRegions] = {};
  int reg_launches[kRegions] = {};
  double last_reg_ms[kRegions] = {}, last_reg_flops[kRegions] = {}, last_reg_bytes[kRegions] = {};
  int last_reg_launches[kRegions] = {};
  // events around a timed region (returns the stop event to record, or nullptr when not timing)
  hipEvent_t region_begin(int region, hipStream_t s) {
    if (!timing) return nullptr;
    hipEvent_t a = next_event(), b = next_event();
    ev_prec.push_back(3 + region);
    if (hipEventRecord(a, s) != hipSuccess) return nullptr;
    return b;
  }
  void region_end(hipEvent_t b, int region, hipStream_t s, int launches, double flops, double bytes) {
    if (!b) return;
    (void)hipEventRecord(b, s);
    reg_launches[region] += launches;
    reg_flops[region] += flops;
    reg_bytes[region] += bytes;
  }
  bool timing = false;
  std::vector<hipEvent_t> ev_pool;  // start/stop pairs around ladder launches
  size_t ev_used = 0;
  hipEvent_t next_event() {
    if (ev_used == ev_pool.size()) {
      hipEvent_t e;
      PNO_HIP(hipEventCreate(&e));
      ev_pool.push_back(e);
    }
    return ev_pool[ev_used++];
  }

  // replay of sigma blocks from captured HIP graphs (pnoeom_set_graph_mode)
  struct SigmaGraph {
    int nv = 0, prec = 0, space = 0;
    int64_t N = 0;
    uint64_t sig = 0;                 // buffer signature at capture
    hipGraphExec_t exec = nullptr;
  };
  bool graph_mode = false;
  std::vector<SigmaGraph> graphs;
  hipStream_t gstream = nullptr;      // stream the graphs are captured on and launched on
  hipEvent_t gev[2] = {nullptr, nullptr};
  DBuf<double> gin, gout;             // fixed input / output of the captured blocks
  DBuf<double> pack_in, pack_out;     // packed canonical vectors of apply_sigma in graph mode
  int fixed_chunk = 0;                // > 0: vectors per sigma chunk (set while capturing)
  int last_chunk = 0;
  int sw_precision = -1;              // precision the sigma workspaces were last sized for
  int graph_launches = 0, graph_captures = 0;
  void drop_graphs() {
    for (SigmaGraph& g : graphs)
      if (g.exec) (void)hipGraphExecDestroy(g.exec);
    graphs.clear();
  }
  ~Context() {
    drop_graphs();
    for (hipEvent_t& e : gev)
      if (e) (void)hipEventDestroy(e);
    if (gstream) (void)hipStreamDestroy(gstream);
    for (hipEvent_t e : ev_pool) (void)hipEventDestroy(e);
  }

  int64_t ov() const { return (int64_t)o * v; }
  int64_t oovv() const { return (int64_t)o * o * v * v; }
  int64_t vlen() const { return ov() + oovv(); }  // canonical vector length
};

void build_df(Context& c, const double* B, const double* eps, const double* t1, const double* t2,
              int precision);
// streamed ladder (ladder.hip)
int64_t ladder_budget();
int64_t streamed_ladder_bytes(const Context& c, int64_t na0, int precision);
void prepare_streamed_ladder(Context& c, int precision, int64_t budget_bytes);
void ladder_streamed(Context& c, int precision, int64_t rows, const void* S, int64_t ldS, const void* A,
                     int64_t ldA, void* SigP, void* SigM);
void build_ladder(Context& c, const double* B, const double* t1, int precision, int64_t budget_bytes);
// Y_m = sum_cd W_abcd X_m[c][d] for nmat v x v matrices (cached or streamed W)
void ladder_apply(Context& c, int nmat, const double* X, double* Y, int precision);
// the same without any device allocation: staging in a fixed per-GPU scratch array
constexpr int64_t kNoAllocScratchBytes = 128ll << 20;
int64_t ladder_noalloc_bytes(const Context& c, int nmat, int precision);
void ladder_apply_noalloc(Context& c, int nmat, const double* X, double* Y, int precision);
void sigma_canonical(Context& c, const double* r1, const double* r2, double* s1, double* s2, int precision);
// nvec vectors; r1/s1 of vector q at offset q*stride1, r2/s2 at q*stride2
void sigma_block(Context& c, int nvec, const double* r1, const double* r2, double* s1, double* s2, int64_t stride1,
                 int64_t stride2, int precision);
void symmetrize_r2(hipStream_t s, int o, int v, double* r2);
// CIS lowest roots; vec (device [n][o][v]) may be null
void cis_roots(Context& c, int n, double* omega, double* vec);
void build_sapno(Context& c, int nstates, double tcut_pno, double tcut_osv);
// PNO compress / expand of nvec vectors (canonical full arrays <-> compressed)
void pno_compress(Context& c, int nvec, const double* r1, const double* r2, double* x);
void pno_expand(Context& c, int nvec, const double* x, double* r1, double* r2);
// the same with another set of PNOs (the ground-state ones)
void pno_compress(Context& c, PNOData& P, int nvec, const double* r1, const double* r2, double* x);
void pno_expand(Context& c, PNOData& P, int nvec, const double* x, double* r1, double* r2);
void project_pno(Context& c, PNOData& P, double* x);
void precond_pno(Context& c, PNOData& P, double* x, double theta);
void build_gs_pnos(Context& c, const double* t2, double tcut_pno, double tcut_osv);
void sigma_pno(Context& c, int nvec, const double* x, double* y, int precision);
// vectors per sigma chunk that fit the free device memory (pno: with the canonical
// expansions of the PNO-space sigma)
int sigma_chunk(Context& c, int nvec, int precision, bool pno);
int64_t sigma_bytes_per_vector(const Context& c, int precision, bool pno);
int64_t sigma_held_bytes(const Context& c);
int64_t sigma_headroom(int64_t total);
// sigma of nv packed vectors X[q] = x + q*N (canonical: [r1 | r2], PNO: compressed)
// into S; through captured graphs when c.graph_mode
void sigma_apply(Context& c, int space, int nv, const double* X, double* S, int64_t N, int precision);

struct DavidsonResult {
  std::vector<double> omega, resnorm;
  int iters = 0;
  int nsigma = 0;
  bool converged = false;
  bool complex_pair = false;
  bool aborted = false;   // stopped at abort_after_iter
};
DavidsonResult davidson(Context& c, int nroots, const pnoeom_davidson_opts& opt);

// CCSD ground state (ccsd.hip)
struct CcsdResult {
  std::vector<double> energies, resmax;  // per evaluated amplitude set
  double e_corr = 0, rmax = 0;
  int iters = 0;
  bool converged = false;
};
double ccsd_residual(Context& c, const double* B, const double* eps, const double* t1, const double* t2,
                     double* r1, double* r2);
CcsdResult ccsd_solve(Context& c, const double* B, const double* eps, double* t1, double* t2, bool start_mp1,
                      const pnoeom_ccsd_opts& opt);

// host eigen-solver (eig.cpp); returns 0 or a negative status
// vectors of the first nvec eigenvalues in sorted order (nvec < 0: all); the others are zero
int host_eig(int n, const double* a, double* wr, double* wi, double* vr, int nvec = -1);
int host_syev(int n, const double* a, double* w, double* v);
void probe_peaks(hipStream_t s, double* fp64_tflops, double* fp32_tflops, double* bf16_tflops, double* copy_gbs);
int host_syev_batched(int nmat, const int* nsz, int ld, double* A, double* ev, double* Vt, int nthreads);

// GPU batched symmetric eigensolver through tridiagonal form (syev.hip) for matrices of up to
// kSyevMaxN: A[m] (nsz[m] x nsz[m], device sizes dn, leading dimension and row stride ld, matrix
// stride ld*ld) is overwritten; ev[m*ld + k] gets every eigenvalue in ascending order and row k of
// Vt[m] the unit eigenvector of eigenvalue k when |ev| >= cut (zero rows otherwise).
constexpr int kSyevMaxN = 1024;
void syev_tridiag(hipStream_t s, int nmat, const int* dn, int nmax, int ld, double* A, double* Vt, double* ev,
                  double cut);
// batched_syev (sapno.hip): Jacobi up to 128, else syev_tridiag (eig_backend 0, n <= kSyevMaxN)
// or the host solver; eigenvector rows of eigenvalues below cut may be left zero
void batched_syev(hipStream_t s, int backend, int nmat, const std::vector<int>& nsz, int ld, double* A, double* Vt,
                  double* ev, int* dn, double cut);

}  // namespace pnoeom
