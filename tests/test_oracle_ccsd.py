"""Pins of the CCSD ground-state oracle (CPU only).

The energy formula is tied to the brute-force projection <0|exp(-T) H exp(T)|0> of
the determinant engine; the closed form of the two-electron singlet Hamiltonian to
the determinant engine's Hamiltonian; the solver to the exactness of CCSD for two
electrons (its energy is the lowest singlet FCI energy, and EOM-CCSD on its
amplitudes gives the singlet FCI excitation energies) and to a zero residual.
"""
import numpy as np
import pytest

from synthgen import make_system
from oracle.ham import bare, mp2_amplitudes, mp2_energy
from oracle.fci import FCI, full_eri, _expm_apply
from oracle.residual import ccsd_residual
from oracle.sigma import SigmaOracle
from oracle.davidson import dense_eom
from oracle.ccsd import ccsd_energy, solve_ccsd, two_electron_singlet_energies


def _sym(x):
    return 0.5 * (x + x.transpose(1, 0, 3, 2))


@pytest.mark.parametrize("o,v,seed", [(1, 4, 3), (2, 3, 4), (3, 4, 5)])
def test_energy_formula_vs_brute_force(o, v, seed):
    s = make_system(o, v, 10, seed, sigma_b=0.12)
    _, h, eref = bare(s.eps, s.B, o)
    f = FCI(h, full_eri(s.B), o)
    rng = np.random.default_rng(seed)
    t1 = rng.standard_normal((o, v)) * 0.2
    t2 = _sym(rng.standard_normal((o, o, v, v)) * 0.2)
    S = f.space
    T = S.excitation_op(t1, t2)
    ref = S.ref()
    x = _expm_apply(T, ref, 1.0)
    y = _expm_apply(T, f.H(x), -1.0)
    e_brute = float(ref @ y) - eref
    assert abs(ccsd_energy(s.eps, s.B, o, t1, t2) - e_brute) < 1e-12 * max(1.0, abs(e_brute))
    # T1 = 0 and first-order T2: the MP2 energy
    t2m = mp2_amplitudes(s.eps, s.B, o)
    assert abs(ccsd_energy(s.eps, s.B, o, np.zeros((o, v)), t2m) - mp2_energy(s.eps, s.B, o)) < 1e-13


def test_two_electron_closed_form_vs_determinants():
    o, v = 1, 4
    s = make_system(o, v, 8, 31, sigma_b=0.15)
    _, h, _ = bare(s.eps, s.B, o)
    f = FCI(h, full_eri(s.B), o)
    n = f.nmo
    Hm = f.h_matrix_dense()
    cols = []
    for p in range(n):
        for q in range(p, n):
            x = np.zeros(n * n)
            x[f.space.index[1 << p] * n + f.space.index[1 << q]] += 1.0
            x[f.space.index[1 << q] * n + f.space.index[1 << p]] += 1.0
            cols.append(x / np.linalg.norm(x))
    Q = np.array(cols).T
    ref = np.sort(np.linalg.eigvalsh(Q.T @ Hm @ Q))
    got = two_electron_singlet_energies(h, full_eri(s.B))
    assert np.max(np.abs(got - ref)) < 1e-12


@pytest.mark.parametrize("v,naux,seed", [(4, 8, 31), (9, 20, 7)])
def test_two_electron_ccsd_is_exact(v, naux, seed):
    o = 1
    s = make_system(o, v, naux, seed, sigma_b=0.15)
    _, h, eref = bare(s.eps, s.B, o)
    t1, t2, e, it, rmax = solve_ccsd(s.eps, s.B, o, tol_r=1e-12, tol_e=1e-14)
    assert rmax < 1e-12 and it < 100
    ef = two_electron_singlet_energies(h, full_eri(s.B))
    assert abs(eref + e - ef[0]) < 1e-10
    so = SigmaOracle(s.eps, s.B, o, t1, t2)
    wd, _ = dense_eom(so.sigma, o, v)
    assert np.max(np.abs(np.sort(wd.real) - (ef[1:] - ef[0]))) < 1e-9
    assert np.max(np.abs(wd.imag)) < 1e-9


def test_solver_zero_residual_and_symmetry():
    o, v = 3, 7
    s = make_system(o, v, 20, 5)
    t1, t2, e, it, rmax = solve_ccsd(s.eps, s.B, o, tol_r=1e-11)
    w1, w2 = ccsd_residual(s.eps, s.B, o, t1, t2)
    assert max(np.abs(w1).max(), np.abs(w2).max()) < 1e-11
    assert np.max(np.abs(t2 - t2.transpose(1, 0, 3, 2))) < 1e-11 * np.abs(t2).max()
    assert abs(e - ccsd_energy(s.eps, s.B, o, t1, t2)) < 1e-15 and e < 0
    # a shorter DIIS history takes another path to the same fixed point
    u1, u2, e2, it2, r2 = solve_ccsd(s.eps, s.B, o, tol_r=1e-11, diis=4, max_iter=400)
    assert r2 < 1e-11 and abs(e2 - e) < 1e-10 and np.max(np.abs(u2 - t2)) < 1e-9


def test_gs_pno_simulation():
    """Ground-state PNO-CCSD simulation: T_cut = 0 is canonical CCSD; at T_cut > 0 the
    amplitudes stay in the OSV / PNO space and solve P Omega(T) = 0 (checked with the
    full-array projector, not the compressed residual the solver stops on), and the energy
    error grows as the cut is raised."""
    from oracle.ccsd import gs_pno_basis
    o = 4
    s = make_system(o, 20, 60, 3, kappa=1.0)
    a1, a2, ae, _, _ = solve_ccsd(s.eps, s.B, o, tol_r=1e-11, tol_e=1e-12)
    b0 = gs_pno_basis(s.eps, s.B, o, 0.0)
    assert b0.npno().min() == 20
    z1, z2, ze, _, _ = solve_ccsd(s.eps, s.B, o, tol_r=1e-11, tol_e=1e-12, basis=b0)
    assert abs(ze - ae) < 1e-12 and np.max(np.abs(z2 - a2)) < 1e-10 and np.max(np.abs(z1 - a1)) < 1e-10
    errs = []
    for tc in (1e-8, 1e-6, 1e-5, 1e-4):
        b = gs_pno_basis(s.eps, s.B, o, tc)
        t1, t2, e, it, rmax = solve_ccsd(s.eps, s.B, o, tol_r=1e-11, tol_e=1e-12, basis=b)
        assert rmax < 1e-11 and it < 60
        w1, w2 = ccsd_residual(s.eps, s.B, o, t1, t2)
        p1, p2 = b.project(w1, w2)
        assert max(np.abs(p1).max(), np.abs(p2).max()) < 1e-10
        q1, q2 = b.project(t1, t2)
        assert np.max(np.abs(q2 - t2)) < 1e-13 and np.max(np.abs(q1 - t1)) < 1e-13
        errs.append(abs(e - ae))
    assert all(x < y for x, y in zip(errs, errs[1:])) and errs[0] < 1e-5
