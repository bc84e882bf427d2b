"""GPU CCSD ground state against the oracle and against exact two-electron energies.

Residual: elementwise |gpu - oracle| <= 1e-11 * max|oracle| (FP64 contractions in another
summation order; the quadratic terms pass through one more intermediate than sigma's).
Solver: both sides iterate to max|Omega| < 1e-11 with the same Jacobi + DIIS algorithm; at
config 1 the oracle's amplitudes at that bound differ from its 1e-14 solution by < 1e-13,
so 1e-9 on the amplitudes and 1e-10 Eh on the energy leave a wide margin.
Two electrons: CCSD and EOM-CCSD are exact, so the GPU energies equal the eigenvalues of the
two-electron singlet Hamiltonian to the convergence bounds (1e-9 Eh).
"""
import numpy as np
import pytest

from synthgen import make_system, config_system, random_r

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return torch


def _dev(s):
    torch = _torch()
    return torch.from_numpy(s.B).cuda(), torch.from_numpy(s.eps).cuda()


def _sym(x):
    return 0.5 * (x + x.transpose(1, 0, 3, 2))


@pytest.mark.parametrize("o,v,naux,seed", [(4, 20, 60, 1), (3, 17, 41, 2), (1, 9, 20, 3), (6, 33, 70, 4)])
def test_residual_matches_oracle(o, v, naux, seed):
    print(f"[ccsd residual] o={o} v={v} naux={naux} seed={seed}", flush=True)
    torch = _torch()
    from paper_1802_06738_amd import PnoEom
    from oracle.residual import ccsd_residual
    from oracle.ccsd import ccsd_energy
    s = make_system(o, v, naux, seed)
    rng = np.random.default_rng(seed + 100)
    t1 = rng.standard_normal((o, v)) * 0.03
    t2 = _sym(rng.standard_normal((o, o, v, v)) * 0.03)
    ctx = PnoEom(o, v, naux)
    B, eps = _dev(s)
    g1, g2, ge = ctx.ccsd_residual(B, eps, torch.from_numpy(t1).cuda(), torch.from_numpy(t2).cuda())
    w1, w2 = ccsd_residual(s.eps, s.B, o, t1, t2)
    assert np.max(np.abs(g1.cpu().numpy() - w1)) <= 1e-11 * np.max(np.abs(w1))
    assert np.max(np.abs(g2.cpu().numpy() - w2)) <= 1e-11 * np.max(np.abs(w2))
    e = ccsd_energy(s.eps, s.B, o, t1, t2)
    assert abs(ge - e) <= 1e-12 * abs(e)
    # the context keeps no intermediates of T2 / 2: sigma is refused until build_df
    from paper_1802_06738_amd.pnoeom import PnoEomError
    with pytest.raises(PnoEomError):
        ctx.sigma(torch.zeros((1, o, v), dtype=torch.float64, device="cuda"),
                  torch.zeros((1, o, o, v, v), dtype=torch.float64, device="cuda"))


def test_solver_matches_oracle_config1():
    print("[ccsd solve] config 1", flush=True)
    torch = _torch()
    from paper_1802_06738_amd import PnoEom
    from oracle.ccsd import solve_ccsd
    from oracle.sigma import SigmaOracle
    s = config_system(1)
    o, v = s.o, s.v
    a1, a2, ae, ait, ar = solve_ccsd(s.eps, s.B, o, tol_r=1e-11, tol_e=1e-12)
    assert ar < 1e-11
    ctx = PnoEom(o, v, s.naux)
    B, eps = _dev(s)
    r = ctx.ccsd(B, eps, tol_r=1e-11, tol_e=1e-12, raise_on_notconv=False)
    print("max|Omega| per step:", " ".join(f"{x:.2e}" for x in r["resmax_history"]), flush=True)
    assert r["converged"] and r["resmax"] < 1e-11
    assert len(r["energies"]) == r["iters"] + 1 and r["energies"][-1] == r["e_corr"]
    assert abs(r["e_corr"] - ae) < 1e-10
    assert abs(r["iters"] - ait) <= 2
    assert np.max(np.abs(r["t1"].cpu().numpy() - a1)) < 1e-9
    assert np.max(np.abs(r["t2"].cpu().numpy() - a2)) < 1e-9
    # the context now holds the intermediates at the converged amplitudes
    r1, r2 = random_r(o, v, 77, nvec=1)
    g1, g2 = ctx.sigma(torch.from_numpy(r1).cuda(), torch.from_numpy(r2).cuda())
    so = SigmaOracle(s.eps, s.B, o, a1, a2)
    x1, x2 = so.sigma(r1[0], r2[0])
    assert np.max(np.abs(g1.cpu().numpy()[0] - x1)) <= 1e-9 * np.max(np.abs(x1))
    assert np.max(np.abs(g2.cpu().numpy()[0] - x2)) <= 1e-9 * np.max(np.abs(x2))


def test_solver_restart_from_given_amplitudes():
    print("[ccsd restart] o=3 v=17", flush=True)
    torch = _torch()
    from paper_1802_06738_amd import PnoEom
    s = make_system(3, 17, 41, 5)
    ctx = PnoEom(3, 17, 41)
    B, eps = _dev(s)
    a = ctx.ccsd(B, eps, max_iter=4, raise_on_notconv=False)
    assert not a["converged"] and a["iters"] == 4
    b = ctx.ccsd(B, eps, t1=a["t1"], t2=a["t2"], tol_r=1e-10)
    c = ctx.ccsd(B, eps, tol_r=1e-10)
    assert b["converged"] and c["converged"]
    assert abs(b["e_corr"] - c["e_corr"]) < 1e-10
    assert torch.max(torch.abs(b["t2"] - c["t2"])).item() < 1e-8


@pytest.mark.parametrize("v,naux,seed", [(24, 60, 11), (60, 140, 12)])
def test_two_electron_ccsd_and_eom_equal_fci(v, naux, seed):
    print(f"[ccsd fci] o=1 v={v} naux={naux}", flush=True)
    torch = _torch()
    from paper_1802_06738_amd import PnoEom
    from oracle.ham import bare
    from oracle.fci import full_eri
    from oracle.ccsd import two_electron_singlet_energies
    o = 1
    s = make_system(o, v, naux, seed)
    _, h, eref = bare(s.eps, s.B, o)
    ef = two_electron_singlet_energies(h, full_eri(s.B))
    ctx = PnoEom(o, v, naux)
    B, eps = _dev(s)
    r = ctx.ccsd(B, eps, tol_r=1e-11, tol_e=1e-12)
    assert r["converged"]
    assert abs(eref + r["e_corr"] - ef[0]) < 1e-9
    nroots = 4
    d = ctx.davidson(nroots, tol_e=1e-10, tol_r=1e-7, max_sub=40, verbose=True)
    exc = ef[1:nroots + 1] - ef[0]
    assert np.max(np.abs(np.sort(d["omega"]) - exc)) < 1e-9


@pytest.mark.parametrize("tcut", [0.0, 1e-6, 1e-5])
def test_gs_pno_ccsd_matches_oracle(tcut):
    """Ground-state PNO-CCSD simulation: PNO / OSV counts exact, energy and amplitudes of the
    projected equations as the oracle's (both to max|Omega-bar| < 1e-11), sigma afterwards at
    those amplitudes; T_cut = 0 is the canonical solution."""
    print(f"[gs-pno ccsd] o=4 v=20 kappa=1 tcut={tcut}", flush=True)
    torch = _torch()
    from paper_1802_06738_amd import PnoEom
    from oracle.ccsd import solve_ccsd, gs_pno_basis
    from oracle.sigma import SigmaOracle
    o, v, naux = 4, 20, 60
    s = make_system(o, v, naux, 3, kappa=1.0)
    basis = gs_pno_basis(s.eps, s.B, o, tcut)
    a1, a2, ae, ait, ar = solve_ccsd(s.eps, s.B, o, tol_r=1e-11, tol_e=1e-12, basis=basis)
    assert ar < 1e-11
    ctx = PnoEom(o, v, naux)
    B, eps = _dev(s)
    r = ctx.ccsd(B, eps, tol_r=1e-11, tol_e=1e-12, gs_tcut_pno=tcut, raise_on_notconv=False)
    print("max|Omega-bar| per step:", " ".join(f"{x:.2e}" for x in r["resmax_history"]), flush=True)
    assert r["converged"]
    assert np.array_equal(r["npno"], basis.npno()) and np.array_equal(r["nosv"], basis.nosv())
    assert abs(r["e_corr"] - ae) < 1e-10
    assert np.max(np.abs(r["t1"].cpu().numpy() - a1)) < 1e-9
    assert np.max(np.abs(r["t2"].cpu().numpy() - a2)) < 1e-9
    if tcut == 0.0:
        c1, c2, ce, _, _ = solve_ccsd(s.eps, s.B, o, tol_r=1e-11, tol_e=1e-12)
        assert abs(r["e_corr"] - ce) < 1e-10
    r1, r2 = random_r(o, v, 78, nvec=1)
    g1, g2 = ctx.sigma(torch.from_numpy(r1).cuda(), torch.from_numpy(r2).cuda())
    x1, x2 = SigmaOracle(s.eps, s.B, o, a1, a2).sigma(r1[0], r2[0])
    # a canonical solve afterwards discards the ground-state PNOs
    if tcut > 0.0:
        ctx2 = PnoEom(o, v, naux)
        ctx2.ccsd(B, eps, gs_tcut_pno=tcut, max_iter=2, raise_on_notconv=False)
        assert ctx2.lib.pnoeom_ccsd_gs_counts(ctx2.h, None, None) == 0
        ctx2.ccsd(B, eps, max_iter=2, raise_on_notconv=False)
        assert ctx2.lib.pnoeom_ccsd_gs_counts(ctx2.h, None, None) == -5   # ESTATE
    assert np.max(np.abs(g1.cpu().numpy()[0] - x1)) <= 1e-9 * np.max(np.abs(x1))
    assert np.max(np.abs(g2.cpu().numpy()[0] - x2)) <= 1e-9 * np.max(np.abs(x2))


def test_ccsd_error_paths():
    """Bad options and missing buffers are refused with EINVAL before any work."""
    print("[ccsd errors]", flush=True)
    import ctypes as C
    import torch
    from paper_1802_06738_amd import PnoEom
    from paper_1802_06738_amd.pnoeom import PnoEomError, CcsdOpts, _dev
    s = make_system(2, 6, 12, 5)
    ctx = PnoEom(2, 6, 12)
    B, eps = torch.from_numpy(s.B).cuda(), torch.from_numpy(s.eps).cuda()
    for kw in (dict(max_iter=-1), dict(tol_r=0.0), dict(tol_e=-1.0), dict(diis_size=65), dict(precision=7)):
        with pytest.raises(PnoEomError) as e:
            ctx.ccsd(B, eps, **kw)
        assert e.value.code == -1, kw
    with pytest.raises(ValueError):
        ctx.ccsd(B, eps, t1=torch.zeros((2, 6), dtype=torch.float64, device="cuda"))   # t2 missing
    t1 = torch.zeros((2, 6), dtype=torch.float64, device="cuda")
    t2 = torch.zeros((2, 2, 6, 6), dtype=torch.float64, device="cuda")
    opts = CcsdOpts()
    ctx.lib.pnoeom_ccsd_defaults(C.byref(opts))
    e_out = C.c_double()
    st = ctx.lib.pnoeom_ccsd(ctx.h, _dev(B), None, _dev(t1), _dev(t2), 0, C.byref(opts), C.byref(e_out), None, None)
    assert st == -1                                                   # null eps
    st = ctx.lib.pnoeom_ccsd(ctx.h, _dev(B), _dev(eps), _dev(t1), _dev(t2), 2, C.byref(opts), C.byref(e_out),
                             None, None)
    assert st == -1                                                   # start must be 0 or 1
    r1 = torch.empty_like(t1)
    r2 = torch.empty_like(t2)
    st = ctx.lib.pnoeom_ccsd_residual(ctx.h, _dev(B), _dev(eps), _dev(t1), _dev(t2), _dev(r1), _dev(r2), None)
    assert st == -1                                                   # null energy output
    # the context is still usable afterwards
    r = ctx.ccsd(B, eps, tol_r=1e-10)
    assert r["converged"]


def test_ccsd_divergence_leaves_no_intermediates():
    """A non-finite iteration (forced from the host by a NaN orbital energy) ends with ENOTCONV,
    returns its amplitudes and leaves the context without intermediates: sigma is refused
    with ESTATE until a finite solve builds them again."""
    print("[ccsd divergence] o=2 v=8", flush=True)
    torch = _torch()
    from paper_1802_06738_amd import PnoEom
    from paper_1802_06738_amd.pnoeom import PnoEomError
    s = make_system(2, 8, 20, 6)
    ctx = PnoEom(2, 8, 20)
    B, eps = _dev(s)
    bad = eps.clone()
    bad[3] = float("nan")
    a = ctx.ccsd(B, bad, raise_on_notconv=False)
    assert not a["converged"] and a["iters"] == 0 and not np.isfinite(a["e_corr"])
    r1, r2 = random_r(2, 8, 79, nvec=1)
    R1, R2 = torch.from_numpy(r1).cuda(), torch.from_numpy(r2).cuda()
    with pytest.raises(PnoEomError) as e:
        ctx.sigma(R1, R2)
    assert e.value.code == -5
    b = ctx.ccsd(B, eps, tol_r=1e-10)
    assert b["converged"] and np.isfinite(b["e_corr"])
    g1, g2 = ctx.sigma(R1, R2)
    assert torch.isfinite(g1).all() and torch.isfinite(g2).all()
    # ground-state PNO simulation: PNOs from finite first-order densities, then NaN start
    # amplitudes (set on the host) make the first step non-finite; the PNOs built in that call
    # are dropped with the intermediates
    print("[ccsd divergence] ground-state PNO simulation", flush=True)
    g = ctx.ccsd(B, eps, tol_r=1e-10, gs_tcut_pno=1e-6)
    assert g["converged"] and g["npno"] is not None
    t2n = torch.full((2, 2, 8, 8), float("nan"), dtype=torch.float64, device="cuda")
    t1n = torch.zeros((2, 8), dtype=torch.float64, device="cuda")
    d = ctx.ccsd(B, eps, t1=t1n, t2=t2n, gs_tcut_pno=1e-6, raise_on_notconv=False)
    assert not d["converged"] and d["npno"] is None and d["nosv"] is None
    assert ctx.lib.pnoeom_ccsd_gs_counts(ctx.h, None, None) == -5   # ESTATE
    with pytest.raises(PnoEomError) as e:
        ctx.sigma(R1, R2)
    assert e.value.code == -5
