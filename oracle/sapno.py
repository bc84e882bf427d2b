"""CIS, CIS(D) doubles, state-averaged pair densities and PNO/OSV bases (oracle).

Test infrastructure: see oracle/__init__.py.

Follows the Methods section:
  * CIS roots: lowest eigenpairs of A_{ia,jb} = d_ij d_ab (f_aa - f_ii) + 2(ia|jb) - (ij|ab),
    normalised so that sum_ia (b_i^a)^2 = 1.
  * CIS(D) doubles of state k (the state-specific doubles equation and the K
    intermediate that follows it), with G^{pq}_{rs} = <pq|rs> = (pr|qs) for real orbitals.
  * Pair density of state k (same form as the ground-state pair density with
    T replaced by the CIS(D) doubles), averaged over the N states (the
    state-averaged density equation).
  * PNOs: eigenvectors of the averaged density per pair i <= j, kept when the
    magnitude of the occupation number is >= T_CutPNO; OSVs: the same for the
    diagonal pairs with T_CutOSV (T_CutOSV = T_CutPNO/10 in Computational Details).
  * Both are rotated to the semicanonical basis, in which the virtual Fock block
    is diagonal (eigenvalues f-bar used by the preconditioner).
Zero denominators are clamped to magnitude 1e-4 Eh keeping their sign.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

ES = dict(optimize=True)
DEN_CLAMP = 1e-4


def clamp(d):
    s = np.where(d >= 0.0, 1.0, -1.0)
    return np.where(np.abs(d) < DEN_CLAMP, s * DEN_CLAMP, d)


def symmetrize(r2):
    """Orthogonal projection onto R2[i,j,a,b] = R2[j,i,b,a] (the singlet space)."""
    return 0.5 * (r2 + r2.transpose(1, 0, 3, 2))


def cis_matrix(eps, B, o):
    nmo = B.shape[1]
    v = nmo - o
    Bov = B[:, :o, o:]
    Boo = B[:, :o, :o]
    Bvv = B[:, o:, o:]
    iajb = np.einsum("Qia,Qjb->iajb", Bov, Bov, **ES)
    ijab = np.einsum("Qij,Qab->iajb", Boo, Bvv, **ES)
    A = 2.0 * iajb - ijab
    d = (eps[o:][None, :] - eps[:o][:, None])
    A = A.reshape(o * v, o * v)
    A[np.diag_indices(o * v)] += d.ravel()
    return A


def cis_roots(eps, B, o, n):
    """Lowest n CIS excitation energies and unit-norm singles vectors [k, i, a]."""
    A = cis_matrix(eps, B, o)
    w, U = sla.eigh(A)
    v = B.shape[1] - o
    b = U[:, :n].T.reshape(n, o, v)
    return w[:n], b


def cisd_k(eps, B, o, b):
    """K^{ij}_{ab} = b_i^c (ac|bj) + b_j^c (ai|bc) - b_l^a (li|bj) - b_l^b (ai|lj)."""
    Bov = B[:, :o, o:]
    Boo = B[:, :o, :o]
    Bvv = B[:, o:, o:]
    Bvo = B[:, o:, :o]
    acbj = np.einsum("Qac,Qbj->acbj", Bvv, Bvo, **ES)
    K = np.einsum("ic,acbj->ijab", b, acbj, **ES)
    K += np.einsum("jc,bcai->ijab", b, acbj, **ES)            # (ai|bc) = (bc|ai)
    libj = np.einsum("Qli,Qbj->libj", Boo, Bvo, **ES)
    K -= np.einsum("la,libj->ijab", b, libj, **ES)
    K -= np.einsum("lb,ljai->ijab", b, libj, **ES)            # (ai|lj) = (lj|ai)
    return K


def cisd_doubles(eps, B, o, omega, b):
    """B^{ij}_{ab(k)} = K^{ij}_{ab(k)} / (omega_k + f_ii + f_jj - f_aa - f_bb)."""
    eo = eps[:o]
    ev = eps[o:]
    d = omega + eo[:, None, None, None] + eo[None, :, None, None] \
        - ev[None, None, :, None] - ev[None, None, None, :]
    return cisd_k(eps, B, o, b) / clamp(d)


def pair_density(bij, diag):
    """D = 2/(1+d_ij) (B Bt^T + B^T Bt), Bt = 2B - B^T, for one pair block B (v x v)."""
    bt = 2.0 * bij - bij.T
    return (2.0 / (2.0 if diag else 1.0)) * (bij @ bt.T + bij.T @ bt)


def sa_densities(eps, B, o, nstates, states=None):
    """Average of the CIS(D) pair densities over the lowest nstates CIS roots, or over
    the listed CIS states (one state: the state-specific density of that state).

    Returns (D [i, j, v, v] for all i, j with D[j,i] = D[i,j], omegas, cis vectors).
    """
    states = list(range(nstates)) if states is None else [int(k) for k in states]
    w, b = cis_roots(eps, B, o, max(states) + 1)
    v = B.shape[1] - o
    D = np.zeros((o, o, v, v))
    for k in states:
        bk = cisd_doubles(eps, B, o, w[k], b[k])
        for i in range(o):
            for j in range(i, o):
                d = pair_density(bk[i, j], i == j)
                D[i, j] += d
                if j != i:
                    D[j, i] += d
    D /= len(states)
    return D, w, b


def truncated_basis(d, cut, fvv):
    """Eigenvectors of a symmetric density with |n| >= cut, in the semicanonical basis.

    Returns (U [v, n], fbar [n], occupations [n] of the kept vectors before rotation).
    """
    n, U = sla.eigh(d)
    keep = np.abs(n) >= cut
    U = U[:, keep]
    if U.shape[1] == 0:
        return U, np.zeros(0), n[keep]
    fb, W = sla.eigh(U.T @ fvv @ U)
    return U @ W, fb, n[keep]


class PNOBasis:
    """Per-pair PNOs U^{ij} (i <= j) and per-occupied OSVs U^i, semicanonical.

    fvv (virtual one-particle matrix, default diag(eps_v)) defines the semicanonical
    rotation through its symmetric part; eo (default eps_occ) the occupied energies
    of the preconditioner.  Neither changes the projector P, only convergence.
    """

    def __init__(self, D, eps, o, tcut_pno, tcut_osv=None, fvv=None, eo=None):
        if tcut_osv is None or tcut_osv < 0:
            tcut_osv = tcut_pno / 10.0
        self.o = o
        self.v = D.shape[2]
        self.eps = eps
        self.eo = eps[:o] if eo is None else eo
        fvv = np.diag(eps[o:]) if fvv is None else 0.5 * (fvv + fvv.T)
        self.pno = {}
        self.fbar = {}
        for i in range(o):
            for j in range(i, o):
                U, fb, _ = truncated_basis(D[i, j], tcut_pno, fvv)
                self.pno[(i, j)] = U
                self.fbar[(i, j)] = fb
        self.osv = []
        self.fosv = []
        for i in range(o):
            U, fb, _ = truncated_basis(D[i, i], tcut_osv, fvv)
            self.osv.append(U)
            self.fosv.append(fb)

    def npno(self):
        return np.array([self.pno[(i, j)].shape[1] for i in range(self.o) for j in range(i, self.o)])

    def nosv(self):
        return np.array([u.shape[1] for u in self.osv])

    def project(self, r1, r2):
        """P: r^i -> U^i U^i^T r^i, r^{ij} -> U^{ij} U^{ij}^T r^{ij} U^{ij} U^{ij}^T.

        The input is first symmetrised to the singlet space (r^{ji} = r^{ij}^T), so
        round-off can never grow components outside it.
        """
        r2 = symmetrize(r2)
        p1 = np.zeros_like(r1)
        p2 = np.zeros_like(r2)
        for i in range(self.o):
            U = self.osv[i]
            p1[i] = U @ (U.T @ r1[i])
        for (i, j), U in self.pno.items():
            blk = U @ (U.T @ r2[i, j] @ U) @ U.T
            p2[i, j] = blk
            p2[j, i] = blk.T
        return p1, p2

    def precondition(self, r1, r2, omega):
        """Residual -> OSV/PNO basis -> divide by semicanonical denominators -> back."""
        eo = self.eo
        p1 = np.zeros_like(r1)
        p2 = np.zeros_like(r2)
        for i in range(self.o):
            U = self.osv[i]
            rb = U.T @ r1[i]
            p1[i] = U @ (rb / clamp(omega + eo[i] - self.fosv[i]))
        for (i, j), U in self.pno.items():
            fb = self.fbar[(i, j)]
            rb = U.T @ r2[i, j] @ U
            d = omega + eo[i] + eo[j] - fb[:, None] - fb[None, :]
            blk = U @ (rb / clamp(d)) @ U.T
            p2[i, j] = blk
            p2[j, i] = blk.T
        return p1, p2


class CanonicalBasis:
    """P = identity (on the singlet space); diagonal preconditioner.

    The denominators use the occupied / virtual one-particle energies eo, ev
    (default: the orbital energies; the Davidson drivers pass the diagonal of the
    one-particle part of H-bar).
    """

    def __init__(self, eps, o, eo=None, ev=None):
        self.eps = eps
        self.o = o
        self.eo = eps[:o] if eo is None else eo
        self.ev = eps[o:] if ev is None else ev

    def project(self, r1, r2):
        return r1.copy(), symmetrize(r2)

    def precondition(self, r1, r2, omega):
        eo = self.eo
        ev = self.ev
        d1 = omega + eo[:, None] - ev[None, :]
        d2 = omega + eo[:, None, None, None] + eo[None, :, None, None] \
            - ev[None, None, :, None] - ev[None, None, None, :]
        return r1 / clamp(d1), r2 / clamp(d2)
