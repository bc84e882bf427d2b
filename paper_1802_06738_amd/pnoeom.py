"""ctypes binding of libpnoeom.so (argument marshalling only).

Every computation runs in the HIP library; this module checks tensor shapes,
dtypes and devices, passes raw device pointers and the current HIP stream, and
turns status codes into exceptions.  It raises if the library is missing: there
is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))

FP64, FP32, BF16 = 0, 1, 2
CANONICAL, PNO = 0, 1
LADDER_AUTO, LADDER_CACHED, LADDER_STREAMED = 0, 1, 2
STATUS = {0: "OK", -1: "EINVAL", -2: "ENOMEM", -3: "EHIP", -4: "ENOTCONV", -5: "ESTATE", -6: "ECOMPLEX",
          -7: "EABORTED"}
EXPORTED_SYMBOLS = ["pnoeom_create", "pnoeom_destroy", "pnoeom_last_error", "pnoeom_build_df", "pnoeom_cis",
                    "pnoeom_build_sapno", "pnoeom_pno_layout", "pnoeom_pno_transform", "pnoeom_apply_sigma", "pnoeom_davidson_defaults",
                    "pnoeom_davidson", "pnoeom_host_eig", "pnoeom_last_timing", "pnoeom_last_ladder_timing",
                    "pnoeom_last_region_timing", "pnoeom_host_syev", "pnoeom_probe_peaks",
                    "pnoeom_gemm_record", "pnoeom_gemm_recorded", "pnoeom_gemm_time", "pnoeom_gemm_set_table",
                    "pnoeom_gemm_bf16", "pnoeom_gemm_bf16_time",
                    "pnoeom_set_graph_mode", "pnoeom_graph_stats", "pnoeom_set_ladder_mode",
                    "pnoeom_set_ring_mode", "pnoeom_ring_mode_used", "pnoeom_set_bf16_passes",
                    "pnoeom_set_bf16_scope",
                    "pnoeom_davidson_phase",
                    "pnoeom_build_ladder", "pnoeom_ladder_apply", "pnoeom_ladder_apply_noalloc",
                    "pnoeom_ladder_noalloc_limit", "pnoeom_set_pno_ladder",
                    "pnoeom_pno_ladder_stats", "pnoeom_set_pno_states", "pnoeom_ccsd_defaults",
                    "pnoeom_ccsd_residual", "pnoeom_ccsd", "pnoeom_ccsd_history", "pnoeom_ccsd_gs_counts",
                    "pnoeom_set_eig_backend", "pnoeom_syev_batched", "pnoeom_sigma_memory"]


class PnoEomError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code


class DavidsonOpts(C.Structure):
    _fields_ = [("space", C.c_int), ("precision", C.c_int), ("tol_e", C.c_double), ("tol_r", C.c_double),
                ("max_sub", C.c_int), ("max_iter", C.c_int), ("refine_fp64", C.c_int), ("verbose", C.c_int),
                ("nextra", C.c_int), ("mixed_tol_e", C.c_double), ("mixed_tol_r", C.c_double),
                ("ckpt_every", C.c_int), ("abort_after_iter", C.c_int), ("ckpt_path", C.c_char_p),
                ("resume_path", C.c_char_p), ("log_path", C.c_char_p)]


class CcsdOpts(C.Structure):
    _fields_ = [("max_iter", C.c_int), ("tol_e", C.c_double), ("tol_r", C.c_double), ("diis_size", C.c_int),
                ("precision", C.c_int), ("gs_tcut_pno", C.c_double), ("gs_tcut_osv", C.c_double)]


_LIB = None


def library_path() -> str:
    return os.path.join(HERE, "libpnoeom.so")


def load_library():
    global _LIB
    if _LIB is not None:
        return _LIB
    path = library_path()
    if not os.path.exists(path):
        raise FileNotFoundError(f"{path} is missing: build it with __graft_entry__.build()")
    # torch first: the library then binds to the HIP runtime torch already loaded (the
    # one whose memory and streams it is handed), not to a second copy
    import torch  # noqa: F401
    lib = C.CDLL(path)
    vp, dp, ip = C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_int)
    lib.pnoeom_create.argtypes = [C.c_int, C.c_int, C.c_int, vp, C.POINTER(vp)]
    lib.pnoeom_destroy.argtypes = [vp]
    lib.pnoeom_destroy.restype = None
    lib.pnoeom_last_error.argtypes = [vp]
    lib.pnoeom_last_error.restype = C.c_char_p
    lib.pnoeom_build_df.argtypes = [vp, vp, vp, vp, vp, C.c_int]
    lib.pnoeom_cis.argtypes = [vp, C.c_int, dp, vp]
    lib.pnoeom_build_sapno.argtypes = [vp, C.c_int, C.c_double, C.c_double, ip, ip]
    lib.pnoeom_pno_layout.argtypes = [vp, C.POINTER(C.c_longlong), C.POINTER(C.c_longlong)]
    lib.pnoeom_apply_sigma.argtypes = [vp, C.c_int, vp, vp, vp, vp, C.c_int, C.c_int]
    lib.pnoeom_pno_transform.argtypes = [vp, C.c_int, C.c_int, vp, vp, vp]
    lib.pnoeom_davidson_defaults.argtypes = [C.POINTER(DavidsonOpts)]
    lib.pnoeom_davidson_defaults.restype = None
    lib.pnoeom_davidson.argtypes = [vp, C.c_int, C.POINTER(DavidsonOpts), dp, dp, ip, ip]
    lib.pnoeom_host_eig.argtypes = [C.c_int, dp, dp, dp, dp]
    lib.pnoeom_last_timing.argtypes = [vp, dp, dp, ip, dp]
    lib.pnoeom_last_ladder_timing.argtypes = [vp, C.c_int, dp, ip, dp]
    lib.pnoeom_last_region_timing.argtypes = [vp, C.c_int, dp, ip, dp, dp]
    lib.pnoeom_host_syev.argtypes = [C.c_int, dp, dp, dp]
    lib.pnoeom_probe_peaks.argtypes = [vp, dp, dp, dp, dp]
    lib.pnoeom_gemm_record.argtypes = [C.c_int]
    lib.pnoeom_gemm_recorded.argtypes = [C.POINTER(C.c_longlong), C.c_int]
    lib.pnoeom_gemm_time.argtypes = [vp, C.POINTER(C.c_longlong), C.c_int, C.c_int, dp]
    lib.pnoeom_gemm_set_table.argtypes = [C.c_int, C.POINTER(C.c_longlong), C.POINTER(C.c_int)]
    ll = C.c_longlong
    lib.pnoeom_gemm_bf16.argtypes = [vp, ll, ll, ll, C.c_float, vp, ll, vp, ll, C.c_float, vp, ll, C.c_int]
    lib.pnoeom_gemm_bf16_time.argtypes = [vp, ll, ll, ll, C.c_int, C.c_int, dp]
    lib.pnoeom_set_graph_mode.argtypes = [vp, C.c_int]
    lib.pnoeom_graph_stats.argtypes = [vp, ip, ip, ip]
    lib.pnoeom_set_ladder_mode.argtypes = [vp, C.c_int, C.c_int]
    lib.pnoeom_set_ring_mode.argtypes = [vp, C.c_int]
    lib.pnoeom_ring_mode_used.argtypes = [vp]
    lib.pnoeom_set_bf16_passes.argtypes = [vp, C.c_int]
    lib.pnoeom_set_bf16_scope.argtypes = [vp, C.c_int]
    lib.pnoeom_davidson_phase.argtypes = [vp, C.c_int, C.c_int, dp, dp, ip, ip, dp]
    lib.pnoeom_build_ladder.argtypes = [vp, vp, vp, C.c_int]
    lib.pnoeom_ladder_apply.argtypes = [vp, C.c_int, vp, vp, C.c_int]
    lib.pnoeom_ladder_apply_noalloc.argtypes = [vp, C.c_int, vp, vp, C.c_int]
    lib.pnoeom_ladder_noalloc_limit.argtypes = [vp, C.c_int]
    lib.pnoeom_ladder_noalloc_limit.restype = C.c_longlong
    lib.pnoeom_set_pno_ladder.argtypes = [vp, C.c_int]
    lib.pnoeom_set_eig_backend.argtypes = [vp, C.c_int]
    lib.pnoeom_sigma_memory.argtypes = [vp, C.c_int, C.c_int, C.POINTER(C.c_longlong), C.POINTER(C.c_longlong), ip]
    lib.pnoeom_syev_batched.argtypes = [vp, C.c_int, C.c_int, vp, C.c_double, vp, vp]
    lib.pnoeom_set_pno_states.argtypes = [vp, C.c_int, ip]
    lib.pnoeom_pno_ladder_stats.argtypes = [vp, ip, ip, ip, dp]
    lib.pnoeom_ccsd_defaults.argtypes = [C.POINTER(CcsdOpts)]
    lib.pnoeom_ccsd_defaults.restype = None
    lib.pnoeom_ccsd_residual.argtypes = [vp, vp, vp, vp, vp, vp, vp, dp]
    lib.pnoeom_ccsd.argtypes = [vp, vp, vp, vp, vp, C.c_int, C.POINTER(CcsdOpts), dp, dp, ip]
    lib.pnoeom_ccsd_history.argtypes = [vp, C.c_int, dp, dp, ip]
    lib.pnoeom_ccsd_gs_counts.argtypes = [vp, ip, ip]
    _LIB = lib
    # the autotuner's table of GEMM tile choices for this device, when present
    from .autotune import DEFAULT_TABLE, load_table
    if os.path.exists(DEFAULT_TABLE):
        load_table(DEFAULT_TABLE, lib)
    return lib


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def host_eig(a: np.ndarray, vectors: bool = True):
    """Eigenvalues (sorted by real part) and right eigenvectors of a small dense matrix."""
    lib = load_library()
    a = np.ascontiguousarray(a, dtype=np.float64)
    n = a.shape[0]
    wr = np.zeros(n)
    wi = np.zeros(n)
    vr = np.zeros((n, n)) if vectors else None
    st = lib.pnoeom_host_eig(n, _dptr(a), _dptr(wr), _dptr(wi), _dptr(vr) if vectors else None)
    if st != 0:
        raise PnoEomError(st, "host_eig failed")
    return wr + 1j * wi, vr


def host_syev(a: np.ndarray):
    """Eigenvalues (unordered) and unit eigenvectors (columns) of a symmetric matrix,
    by the library's host solver (the one the PNO build uses for large blocks)."""
    lib = load_library()
    a = np.ascontiguousarray(a, dtype=np.float64)
    n = a.shape[0]
    w = np.zeros(n)
    v = np.zeros((n, n))
    st = lib.pnoeom_host_syev(n, _dptr(a), _dptr(w), _dptr(v))
    if st != 0:
        raise PnoEomError(st, "host_syev failed")
    return w, v


def _dev(t, shape=None, name="tensor"):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a torch tensor on a HIP device")
    if t.dtype != torch.float64:
        raise TypeError(f"{name} must be float64")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
    return C.c_void_p(t.data_ptr())


def gemm_bf16(A, B, C_out, alpha=1.0, beta=0.0, variant=0):
    """C_out = alpha A B^T + beta C_out on the library's bfloat16 MFMA kernels.  A [M, K] and
    B [N, K] torch.bfloat16 on the device (contiguous, K a multiple of 64), C_out [M, N]
    torch.float32 (contiguous)."""
    import torch
    lib = load_library()
    for t, dt, nm in ((A, torch.bfloat16, "A"), (B, torch.bfloat16, "B"), (C_out, torch.float32, "C")):
        if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != dt or not t.is_contiguous():
            raise TypeError(f"{nm} must be a contiguous {dt} tensor on a HIP device")
    M, K = A.shape
    N = B.shape[0]
    if B.shape[1] != K or tuple(C_out.shape) != (M, N):
        raise ValueError("gemm_bf16: shapes do not match")
    st = lib.pnoeom_gemm_bf16(C.c_void_p(torch.cuda.current_stream().cuda_stream), M, N, K, float(alpha),
                              C.c_void_p(A.data_ptr()), K, C.c_void_p(B.data_ptr()), K, float(beta),
                              C.c_void_p(C_out.data_ptr()), N, int(variant))
    if st != 0:
        raise PnoEomError(st, "gemm_bf16 failed")
    return C_out


def gemm_bf16_time(M, N, K, variant=0, reps=10):
    """Mean milliseconds of one bfloat16 GEMM launch of shape M x N x K (scratch operands)."""
    import torch
    lib = load_library()
    ms = C.c_double()
    st = lib.pnoeom_gemm_bf16_time(C.c_void_p(torch.cuda.current_stream().cuda_stream), M, N, K, int(variant),
                                   int(reps), C.byref(ms))
    if st != 0:
        raise PnoEomError(st, "gemm_bf16_time failed")
    return ms.value


class PnoEom:
    """One library context (o occupied, v virtual, naux fitting functions) on the current device."""

    def __init__(self, o: int, v: int, naux: int, stream=None):
        import torch
        self.lib = load_library()
        self.o, self.v, self.naux = o, v, naux
        self.nmo = o + v
        if stream is None:
            stream = torch.cuda.current_stream()
        self.stream = stream
        h = C.c_void_p()
        st = self.lib.pnoeom_create(o, v, naux, C.c_void_p(stream.cuda_stream), C.byref(h))
        if st != 0:
            raise PnoEomError(st, "pnoeom_create failed")
        self.h = h
        self._pno_len = None

    def close(self):
        if getattr(self, "h", None):
            self.lib.pnoeom_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, st):
        if st != 0:
            raise PnoEomError(st, self.lib.pnoeom_last_error(self.h).decode())

    def build_df(self, B, eps, t1=None, t2=None, precision=FP64):
        o, v, n = self.o, self.v, self.nmo
        args = [_dev(B, (self.naux, n, n), "B"), _dev(eps, (n,), "eps"),
                _dev(t1, (o, v), "t1") if t1 is not None else None,
                _dev(t2, (o, o, v, v), "t2") if t2 is not None else None]
        self._check(self.lib.pnoeom_build_df(self.h, *args, precision))

    def cis(self, nroots, vectors=True):
        import torch
        om = np.zeros(nroots)
        vec = torch.empty((nroots, self.o, self.v), dtype=torch.float64, device="cuda") if vectors else None
        self._check(self.lib.pnoeom_cis(self.h, nroots, _dptr(om), _dev(vec) if vectors else None))
        return om, vec

    def build_sapno(self, nstates, tcut_pno, tcut_osv=-1.0):
        npair = self.o * (self.o + 1) // 2
        npno = np.zeros(npair, dtype=np.int32)
        nosv = np.zeros(self.o, dtype=np.int32)
        self._check(self.lib.pnoeom_build_sapno(self.h, nstates, tcut_pno, tcut_osv,
                                                npno.ctypes.data_as(C.POINTER(C.c_int)),
                                                nosv.ctypes.data_as(C.POINTER(C.c_int))))
        self._pno_len = None
        return npno, nosv

    def pno_layout(self):
        n = self.o + self.o * (self.o + 1) // 2 + 1
        off = np.zeros(n, dtype=np.int64)
        ln = C.c_longlong()
        self._check(self.lib.pnoeom_pno_layout(self.h, off.ctypes.data_as(C.POINTER(C.c_longlong)), C.byref(ln)))
        return off, int(ln.value)

    def pno_compress(self, r1, r2):
        import torch
        nvec = r1.shape[0]
        _, ln = self.pno_layout()
        x = torch.zeros((nvec, ln), dtype=torch.float64, device=r1.device)
        self._check(self.lib.pnoeom_pno_transform(self.h, nvec, 0, _dev(r1, (nvec, self.o, self.v), "r1"),
                                                  _dev(r2, (nvec, self.o, self.o, self.v, self.v), "r2"), _dev(x)))
        return x

    def pno_expand(self, x):
        import torch
        nvec = x.shape[0]
        r1 = torch.empty((nvec, self.o, self.v), dtype=torch.float64, device=x.device)
        r2 = torch.empty((nvec, self.o, self.o, self.v, self.v), dtype=torch.float64, device=x.device)
        self._check(self.lib.pnoeom_pno_transform(self.h, nvec, 1, _dev(r1), _dev(r2), _dev(x, None, "x")))
        return r1, r2

    def sigma(self, r1, r2, precision=FP64):
        """Canonical sigma for r1 [nvec, o, v], r2 [nvec, o, o, v, v] (torch float64 on device)."""
        import torch
        nvec = r1.shape[0]
        o, v = self.o, self.v
        s1 = torch.empty_like(r1)
        s2 = torch.empty_like(r2)
        self._check(self.lib.pnoeom_apply_sigma(self.h, nvec, _dev(r1, (nvec, o, v), "r1"),
                                                _dev(r2, (nvec, o, o, v, v), "r2"), _dev(s1), _dev(s2),
                                                CANONICAL, precision))
        return s1, s2

    def sigma_pno(self, x, precision=FP64):
        import torch
        nvec, n = x.shape
        y = torch.empty_like(x)
        self._check(self.lib.pnoeom_apply_sigma(self.h, nvec, _dev(x, (nvec, n), "x"), None, _dev(y), None, PNO,
                                                precision))
        return y

    def davidson(self, nroots, space=CANONICAL, precision=FP64, tol_e=1e-8, tol_r=-1.0, max_sub=60,
                 max_iter=200, refine_fp64=False, verbose=False, nextra=0, mixed_tol_e=0.0, mixed_tol_r=0.0,
                 ckpt_every=0, abort_after_iter=0, ckpt_path=None, resume_path=None, log_path=None):
        opts = DavidsonOpts()
        self.lib.pnoeom_davidson_defaults(C.byref(opts))
        opts.space, opts.precision, opts.tol_e, opts.tol_r = space, precision, tol_e, tol_r
        opts.max_sub, opts.max_iter = max_sub, max_iter
        opts.refine_fp64, opts.verbose, opts.nextra = int(refine_fp64), int(verbose), int(nextra)
        opts.mixed_tol_e, opts.mixed_tol_r = float(mixed_tol_e), float(mixed_tol_r)
        opts.ckpt_every, opts.abort_after_iter = int(ckpt_every), int(abort_after_iter)
        opts.ckpt_path = os.fsencode(ckpt_path) if ckpt_path else None
        opts.resume_path = os.fsencode(resume_path) if resume_path else None
        opts.log_path = os.fsencode(log_path) if log_path else None
        om = np.zeros(nroots)
        rn = np.zeros(nroots)
        it = C.c_int()
        ns = C.c_int()
        st = self.lib.pnoeom_davidson(self.h, nroots, C.byref(opts), _dptr(om), _dptr(rn), C.byref(it),
                                      C.byref(ns))
        if st not in (0, -6):
            self._check(st)
        out = dict(omega=om, resnorm=rn, iters=it.value, nsigma=ns.value, complex=(st == -6))
        for ph, name in ((0, "main_phase"), (1, "refine_phase")):
            pom = np.zeros(nroots)
            prn = np.zeros(nroots)
            pit, pns, psec = C.c_int(), C.c_int(), C.c_double()
            if self.lib.pnoeom_davidson_phase(self.h, ph, nroots, _dptr(pom), _dptr(prn), C.byref(pit),
                                              C.byref(pns), C.byref(psec)) == 0:
                out[name] = dict(omega=pom, resnorm=prn, iters=pit.value, nsigma=pns.value, seconds=psec.value)
        return out

    def ccsd_residual(self, B, eps, t1, t2):
        """CCSD residual (Omega1 [o][v], Omega2 [o][o][v][v]) and E_CC - E_ref of given amplitudes.
        Leaves no intermediates behind (build_df again before sigma / davidson)."""
        import torch
        o, v, n = self.o, self.v, self.nmo
        r1 = torch.empty((o, v), dtype=torch.float64, device="cuda")
        r2 = torch.empty((o, o, v, v), dtype=torch.float64, device="cuda")
        e = C.c_double()
        self._check(self.lib.pnoeom_ccsd_residual(self.h, _dev(B, (self.naux, n, n), "B"), _dev(eps, (n,), "eps"),
                                                  _dev(t1, (o, v), "t1"), _dev(t2, (o, o, v, v), "t2"),
                                                  _dev(r1), _dev(r2), C.byref(e)))
        return r1, r2, e.value

    def ccsd(self, B, eps, t1=None, t2=None, max_iter=100, tol_e=1e-10, tol_r=1e-8, diis_size=8,
             precision=FP64, raise_on_notconv=True, gs_tcut_pno=-1.0, gs_tcut_osv=-1.0):
        """Solve the CCSD equations (Jacobi + DIIS) from T1 = 0 and first-order T2, or from the
        given t1 and t2 (both or neither).  Returns dict(t1, t2, e_corr, resmax, iters, converged);
        the context then holds the intermediates at those amplitudes (contraction precision
        `precision`), ready for sigma / davidson.  gs_tcut_pno >= 0: the ground-state PNO
        simulation (then also npno / nosv, the ground-state PNO and OSV counts)."""
        import torch
        o, v, n = self.o, self.v, self.nmo
        if (t1 is None) != (t2 is None):
            raise ValueError("give both t1 and t2, or neither")
        start = 0 if t1 is None else 1
        t1 = torch.zeros((o, v), dtype=torch.float64, device="cuda") if t1 is None else t1.clone()
        t2 = torch.zeros((o, o, v, v), dtype=torch.float64, device="cuda") if t2 is None else t2.clone()
        opts = CcsdOpts()
        self.lib.pnoeom_ccsd_defaults(C.byref(opts))
        opts.max_iter, opts.tol_e, opts.tol_r = int(max_iter), float(tol_e), float(tol_r)
        opts.diis_size, opts.precision = int(diis_size), int(precision)
        opts.gs_tcut_pno, opts.gs_tcut_osv = float(gs_tcut_pno), float(gs_tcut_osv)
        e = C.c_double()
        rm = C.c_double()
        it = C.c_int()
        st = self.lib.pnoeom_ccsd(self.h, _dev(B, (self.naux, n, n), "B"), _dev(eps, (n,), "eps"),
                                  _dev(t1, (o, v), "t1"), _dev(t2, (o, o, v, v), "t2"), start, C.byref(opts),
                                  C.byref(e), C.byref(rm), C.byref(it))
        if st != 0 and (st != -4 or raise_on_notconv):
            self._check(st)
        self._pno_len = None
        n = C.c_int()
        self._check(self.lib.pnoeom_ccsd_history(self.h, 0, None, None, C.byref(n)))
        he = np.zeros(n.value)
        hr = np.zeros(n.value)
        self._check(self.lib.pnoeom_ccsd_history(self.h, n.value, _dptr(he), _dptr(hr), C.byref(n)))
        out = dict(t1=t1, t2=t2, e_corr=e.value, resmax=rm.value, iters=it.value, converged=(st == 0),
                   energies=he, resmax_history=hr)
        if gs_tcut_pno >= 0:
            npno = np.zeros(self.o * (self.o + 1) // 2, dtype=np.int32)
            nosv = np.zeros(self.o, dtype=np.int32)
            st = self.lib.pnoeom_ccsd_gs_counts(self.h, npno.ctypes.data_as(C.POINTER(C.c_int)),
                                                nosv.ctypes.data_as(C.POINTER(C.c_int)))
            if st == -5 and not out["converged"]:
                npno = nosv = None   # a diverged simulation keeps no ground-state PNOs
            else:
                self._check(st)
            out["npno"], out["nosv"] = npno, nosv
        return out

    def set_ring_mode(self, mode=0):
        """R1-driven ring terms for the next build_df: 0 auto, 1 through (ij|ab)', 2 through the
        T-only intermediates."""
        self._check(self.lib.pnoeom_set_ring_mode(self.h, int(mode)))

    def set_bf16_passes(self, passes=1):
        """bfloat16 ring products of BF16 contractions for the next build_df: 1 or 3 passes."""
        self._check(self.lib.pnoeom_set_bf16_passes(self.h, int(passes)))

    def set_bf16_scope(self, scope=1):
        """Contractions of BF16 mode on bfloat16 MFMA for the next build_df: 0 the ladder and the
        ring products, 1 also the hole ladder, X_klij, M1, the DF and R1 ring terms."""
        self._check(self.lib.pnoeom_set_bf16_scope(self.h, int(scope)))

    def ring_mode_used(self):
        st = self.lib.pnoeom_ring_mode_used(self.h)
        if st < 0:
            self._check(st)
        return st

    def set_ladder_mode(self, mode=LADDER_AUTO, max_slab=0):
        """Cached or streamed W+/- for the next build_df (LADDER_AUTO / _CACHED / _STREAMED)."""
        self._check(self.lib.pnoeom_set_ladder_mode(self.h, int(mode), int(max_slab)))

    def build_ladder(self, B, t1=None, precision=FP64):
        """Dressed virtual factors and the streamed-ladder workspace only (no other intermediates)."""
        o, v, n = self.o, self.v, self.nmo
        self._check(self.lib.pnoeom_build_ladder(self.h, _dev(B, (self.naux, n, n), "B"),
                                                 _dev(t1, (o, v), "t1") if t1 is not None else None, precision))

    def ladder_apply(self, X, precision=FP64, out=None):
        """Y[m] = sum_cd W_ab^cd X[m][c][d] for X [nmat, v, v] (torch float64 on device)."""
        import torch
        nmat = X.shape[0]
        v = self.v
        Y = torch.empty_like(X) if out is None else out
        self._check(self.lib.pnoeom_ladder_apply(self.h, nmat, _dev(X, (nmat, v, v), "X"),
                                                 _dev(Y, (nmat, v, v), "Y"), precision))
        return Y

    def ladder_apply_noalloc(self, X, out, precision=FP64):
        """ladder_apply into the caller's `out` with no device allocation in the library
        (staging in its fixed per-GPU scratch array; see pnoeom_ladder_apply_noalloc)."""
        nmat = X.shape[0]
        v = self.v
        self._check(self.lib.pnoeom_ladder_apply_noalloc(self.h, nmat, _dev(X, (nmat, v, v), "X"),
                                                         _dev(out, (nmat, v, v), "Y"), precision))
        return out

    def ladder_noalloc_limit(self, precision=FP64):
        """Largest batch ladder_apply_noalloc accepts at this context's v."""
        return int(self.lib.pnoeom_ladder_noalloc_limit(self.h, precision))

    def set_pno_states(self, states=()):
        """CIS states averaged by the next build_sapno (one state: state-specific PNOs; () = default)."""
        arr = (C.c_int * max(len(states), 1))(*[int(k) for k in states])
        self._check(self.lib.pnoeom_set_pno_states(self.h, len(states), arr if len(states) else None))

    def set_pno_ladder(self, max_native=-1):
        """PNO-space ladder for pairs with n_p <= max_native at the next build_sapno (-1 auto, 0 none)."""
        self._check(self.lib.pnoeom_set_pno_ladder(self.h, int(max_native)))

    def sigma_memory(self, space, precision):
        """(bytes per trial vector of a sigma chunk, bytes available to chunks, vectors per chunk)."""
        per, av, ch = C.c_longlong(), C.c_longlong(), C.c_int()
        self._check(self.lib.pnoeom_sigma_memory(self.h, int(space), int(precision), C.byref(per), C.byref(av),
                                                 C.byref(ch)))
        return per.value, av.value, ch.value

    def set_eig_backend(self, backend=0):
        """Symmetric eigenproblems above 128 in build_sapno / syev_batched: 0 GPU, 1 host threads."""
        self._check(self.lib.pnoeom_set_eig_backend(self.h, int(backend)))

    def syev_batched(self, a, cut=0.0):
        """Eigenpairs of the symmetric matrices a [nmat, n, n] (float64 on the device, overwritten):
        (ev [nmat, n], vt [nmat, n, n]) with row k of vt[m] the eigenvector of ev[m, k] wherever
        |ev[m, k]| >= cut (other rows may be zero)."""
        import torch
        nmat, n = int(a.shape[0]), int(a.shape[1])
        pa = _dev(a, (nmat, n, n), "a")
        ev = torch.empty((nmat, n), dtype=torch.float64, device=a.device)
        vt = torch.empty((nmat, n, n), dtype=torch.float64, device=a.device)
        self._check(self.lib.pnoeom_syev_batched(self.h, nmat, n, pa, float(cut), _dev(ev), _dev(vt)))
        return ev, vt

    def pno_ladder_stats(self):
        v = [C.c_int() for _ in range(3)]
        f = C.c_double()
        self._check(self.lib.pnoeom_pno_ladder_stats(self.h, *[C.byref(x) for x in v], C.byref(f)))
        return dict(cut=v[0].value, native_pairs=v[1].value, canonical_pairs=v[2].value, native_flops=f.value)

    def set_graph_mode(self, enable=True):
        self._check(self.lib.pnoeom_set_graph_mode(self.h, int(bool(enable))))

    def graph_stats(self):
        v = [C.c_int() for _ in range(3)]
        self._check(self.lib.pnoeom_graph_stats(self.h, *[C.byref(x) for x in v]))
        return dict(captures=v[0].value, launches=v[1].value, cached=v[2].value)

    def probe_peaks(self):
        """Measured MFMA TFLOP/s (fp64, fp32, bf16) and device-copy HBM GB/s."""
        v = [C.c_double() for _ in range(4)]
        self._check(self.lib.pnoeom_probe_peaks(self.h, *[C.byref(x) for x in v]))
        return dict(fp64_tflops=v[0].value, fp32_tflops=v[1].value, bf16_tflops=v[2].value, copy_gbs=v[3].value)

    def last_timing(self):
        t = C.c_double()
        lad = C.c_double()
        n = C.c_int()
        fl = C.c_double()
        self._check(self.lib.pnoeom_last_timing(self.h, C.byref(t), C.byref(lad), C.byref(n), C.byref(fl)))
        out = dict(total_ms=t.value, ladder_ms=lad.value, ladder_launches=n.value, ladder_flops=fl.value)
        for p, name in ((FP64, "fp64"), (FP32, "fp32"), (BF16, "bf16")):
            self._check(self.lib.pnoeom_last_ladder_timing(self.h, p, C.byref(lad), C.byref(n), C.byref(fl)))
            out[name] = dict(ladder_ms=lad.value, ladder_launches=n.value, ladder_flops=fl.value)
        by = C.c_double()
        for r, name in ((0, "dots"), (1, "pno_transform"), (2, "ladder_w_build"), (3, "ring"),
                        (4, "pno_native_ladder")):
            self._check(self.lib.pnoeom_last_region_timing(self.h, r, C.byref(lad), C.byref(n), C.byref(fl),
                                                           C.byref(by)))
            out[name] = dict(ms=lad.value, launches=n.value, flops=fl.value, bytes=by.value)
        return out
