"""Closed-shell CCSD ground state (oracle).

Test infrastructure: see oracle/__init__.py.

The Methods section defines the CC ground state by the energy
E_CC = <0| exp(-T) H exp(T) |0> and the projected amplitude equations
<mu| exp(-T) H exp(T) |0> = 0 for all singles and doubles mu; the residual of
those equations is residual.ccsd_residual.  The paper gives no solver, so the
one here is the usual one (a reading): Jacobi steps with orbital-energy
denominators,
    t_i^a    <- t_i^a    + Omega_i^a    / (eps_i - eps_a)
    t_ij^ab  <- t_ij^ab  + Omega_ij^ab  / (eps_i + eps_j - eps_a - eps_b),
accelerated by Pulay's DIIS over the last few (amplitude, step) pairs.

Energy.  With closed-shell T = sum t_i^a E_ai + 1/2 sum t_ij^ab E_ai E_bj the
projection onto the reference ends at second order in T:
    E_CC - E_ref = sum_ia 2 f_ia t_i^a
                 + sum_ijab [2 (ia|jb) - (ib|ja)] (t_ij^ab + t_i^a t_j^b).
"""
from __future__ import annotations

import numpy as np

from .residual import ccsd_residual


def ccsd_energy(eps, B, o, t1, t2):
    """E_CC - E_ref of the formula above (f_ia = 0: the synthetic Fock matrix is diagonal)."""
    B = np.asarray(B, dtype=np.float64)
    Bov = B[:, :o, o:]
    g = np.einsum("Qia,Qjb->iajb", Bov, Bov, optimize=True)
    tau = np.asarray(t2) + np.einsum("ia,jb->ijab", t1, t1)
    L = 2.0 * g - g.transpose(0, 3, 2, 1)             # [i,a,j,b]: 2(ia|jb) - (ib|ja)
    return float(np.einsum("iajb,ijab->", L, tau, optimize=True))


def denominators(eps, o):
    eps = np.asarray(eps, dtype=np.float64)
    eo, ev = eps[:o], eps[o:]
    d1 = eo[:, None] - ev[None, :]
    d2 = eo[:, None, None, None] + eo[None, :, None, None] - ev[None, None, :, None] - ev[None, None, None, :]
    return d1, d2


def gs_densities(t2):
    """Ground-state pair densities D_(0)^ij = 2/(1 + d_ij) (T T~^T + T^T T~), T~ = 2T - T^T,
    of the guess amplitudes (Methods, ground-state PNOs), for all pairs [i, j, v, v]."""
    from .sapno import pair_density
    o, v = t2.shape[0], t2.shape[2]
    D = np.zeros((o, o, v, v))
    for i in range(o):
        for j in range(o):
            D[i, j] = pair_density(t2[i, j], i == j)
    return D


def gs_pno_basis(eps, B, o, tcut_pno, tcut_osv=None):
    """GS-PNOs / OSVs from the MP1 pair densities, semicanonical in the Fock matrix diag(eps)."""
    from .ham import mp2_amplitudes
    from .sapno import PNOBasis
    return PNOBasis(gs_densities(mp2_amplitudes(eps, B, o)), np.asarray(eps, dtype=np.float64), o, tcut_pno,
                    tcut_osv)


def compressed_max(basis, w1, w2):
    """Largest element of the residual in the OSV / PNO basis (U^i^T w^i, U^ij^T w^ij U^ij for
    pairs i <= j, off-diagonal pairs weighted by sqrt 2, the weight that makes the compressed
    inner product the full-array one)."""
    m = 0.0
    for i in range(basis.o):
        if basis.osv[i].shape[1]:
            m = max(m, float(np.abs(basis.osv[i].T @ w1[i]).max()))
    for (i, j), U in basis.pno.items():
        if U.shape[1]:
            m = max(m, float(np.abs(U.T @ w2[i, j] @ U).max()) * (1.0 if i == j else np.sqrt(2.0)))
    return m


def solve_ccsd(eps, B, o, t1=None, t2=None, tol_r=1e-10, tol_e=1e-12, max_iter=200, diis=8, basis=None):
    """Jacobi + DIIS solution of the CCSD equations.

    Starts from (t1, t2), default T1 = 0 and the first-order T2 (MP1).  Converged when
    the largest |Omega| is below tol_r and the last step changed the energy by less than
    tol_e.  Returns (t1, t2, e_corr, steps taken, max|Omega|).

    basis (a sapno.PNOBasis, e.g. gs_pno_basis): the ground-state PNO simulation of the
    Methods section.  The start is projected onto the OSV / PNO space; every step takes the
    residual into the semicanonical OSV / PNO basis, divides it by f_ii (+ f_jj) - fbar_a
    (- fbar_b) there and transforms it back (basis.precondition at omega = 0), so the
    amplitudes stay in the space and the fixed point is P Omega = 0; max|Omega| is then
    measured in that basis (compressed_max).
    """
    from .ham import mp2_amplitudes
    eps = np.asarray(eps, dtype=np.float64)
    B = np.asarray(B, dtype=np.float64)
    v = B.shape[1] - o
    t1 = np.zeros((o, v)) if t1 is None else np.array(t1, dtype=np.float64)
    t2 = mp2_amplitudes(eps, B, o) if t2 is None else np.array(t2, dtype=np.float64)
    if basis is not None:
        t1, t2 = basis.project(t1, t2)
    d1, d2 = denominators(eps, o)
    xs, es = [], []
    e, e_prev = ccsd_energy(eps, B, o, t1, t2), np.inf
    for it in range(max_iter + 1):
        w1, w2 = ccsd_residual(eps, B, o, t1, t2)
        if basis is None:
            rmax = max(float(np.abs(w1).max()), float(np.abs(w2).max()))
        else:
            rmax = compressed_max(basis, w1, w2)
        if (rmax < tol_r and abs(e - e_prev) < tol_e) or it == max_iter:
            return t1, t2, e, it, rmax
        if basis is None:
            s = np.concatenate([(w1 / d1).ravel(), (w2 / d2).ravel()])
        else:
            p1, p2 = basis.precondition(w1, w2, 0.0)
            s = np.concatenate([p1.ravel(), p2.ravel()])
        x = np.concatenate([t1.ravel(), t2.ravel()]) + s
        xs.append(x)
        es.append(s)
        if len(xs) > diis:
            xs.pop(0)
            es.pop(0)
        if len(xs) > 1:
            m = len(xs)
            A = np.zeros((m + 1, m + 1))
            for k in range(m):
                for l in range(m):
                    A[k, l] = es[k] @ es[l]
            A[m, :m] = A[:m, m] = -1.0
            rhs = np.zeros(m + 1)
            rhs[m] = -1.0
            c = np.linalg.solve(A, rhs)[:m]
            x = sum(ck * xk for ck, xk in zip(c, xs))
        t1 = x[:o * v].reshape(o, v).copy()
        t2 = x[o * v:].reshape(o, o, v, v).copy()
        e_prev, e = e, ccsd_energy(eps, B, o, t1, t2)


def two_electron_singlet_energies(h, eri):
    """Eigenvalues of H on the singlet states of two electrons (the closed-shell o = 1 case).

    A two-electron state sum_pq C_pq a+_{p alpha} a+_{q beta}|vac> is a singlet when C is
    symmetric.  On the coefficient matrix the Hamiltonian of ham.py acts as
        (H C)_pq = sum_r h_pr C_rq + sum_s h_qs C_ps + sum_rs (pr|qs) C_rs
    (one-body part on each electron, Coulomb interaction between the alpha and the beta
    electron).  The matrix is restricted to an orthonormal basis of symmetric C.
    """
    h = np.asarray(h, dtype=np.float64)
    n = h.shape[0]
    eri = np.asarray(eri, dtype=np.float64).reshape(n, n, n, n)
    one = np.eye(n)
    Hm = np.kron(h, one) + np.kron(one, h) + eri.transpose(0, 2, 1, 3).reshape(n * n, n * n)
    iu = np.triu_indices(n)
    Q = np.zeros((n * n, len(iu[0])))
    for k, (p, q) in enumerate(zip(*iu)):
        if p == q:
            Q[p * n + p, k] = 1.0
        else:
            Q[p * n + q, k] = Q[q * n + p, k] = np.sqrt(0.5)
    return np.linalg.eigvalsh(Q.T @ Hm @ Q)
