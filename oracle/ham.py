"""Closed-shell Hamiltonian built from density-fitting factors (oracle).

Test infrastructure: see oracle/__init__.py.

The Hamiltonian is H = sum_pq h_pq E_pq + 1/2 sum_pqrs (pq|rs)(E_pq E_rs - d_qr E_ps)
with the spin-summed excitation operators E_pq of the Methods section (the
operators in which T and R are parameterised).  Density fitting (Computational
Details) gives (pq|rs) = sum_Q B^Q_pq B^Q_rs.  The Fock matrix of the synthetic
reference is diag(eps), which fixes the core operator h = f - sum_k [2(pq|kk) - (pk|kq)].

A *general* Hamiltonian in this module is stored as
  f      : its Fock matrix with respect to the closed-shell reference |0>
  pairs  : list of (L, R) DF factor pairs, (pq|rs) = sum_t sum_Q L_t^Q_pq R_t^Q_rs
so that similarity-dressed (non-Hermitian) and one-index-transformed operators
fit the same container.  Every container used here keeps (pq|rs) = (rs|pq).
"""
from __future__ import annotations

import numpy as np


class DFHam:
    """General closed-shell two-body Hamiltonian (Fock matrix + DF factor pairs)."""

    def __init__(self, f, pairs, o, h=None):
        self.f = np.asarray(f)
        self.pairs = list(pairs)
        self.o = o
        self.nmo = self.f.shape[0]
        self.h = h
        self._cache = {}

    def sl(self, c):
        return slice(0, self.o) if c == "o" else slice(self.o, self.nmo)

    def eri(self, spec):
        """Block of (pq|rs); spec is a 4-letter string over {o, v}, e.g. 'vvvv'."""
        if spec in self._cache:
            return self._cache[spec]
        p, q, r, s = (self.sl(c) for c in spec)
        out = None
        for L, R in self.pairs:
            a = L[:, p, q]
            b = R[:, r, s]
            n1 = a.shape[1] * a.shape[2]
            n2 = b.shape[1] * b.shape[2]
            blk = (a.reshape(a.shape[0], n1).T @ b.reshape(b.shape[0], n2)).reshape(
                a.shape[1], a.shape[2], b.shape[1], b.shape[2])
            out = blk if out is None else out + blk
        self._cache[spec] = out
        return out

    def ladder_matrix(self):
        """W[(a,b),(c,d)] = (ac|bd) as a (v^2 x v^2) matrix (particle-particle ladder)."""
        if "ladder" in self._cache:
            return self._cache["ladder"]
        o, n = self.o, self.nmo
        v = n - o
        W = None
        for L, R in self.pairs:
            m = L[:, o:, o:].reshape(-1, v * v).T @ R[:, o:, o:].reshape(-1, v * v)
            m = m.reshape(v, v, v, v).transpose(0, 2, 1, 3)
            W = m.copy() if W is None else W + m
        W = W.reshape(v * v, v * v)
        self._cache["ladder"] = W
        return W

    def fo(self, spec):
        p, q = (self.sl(c) for c in spec)
        return self.f[p, q]


def coulomb_exchange(L, R, o):
    """J_pq = sum_Q L^Q_pq sum_k R^Q_kk and K_pq = sum_Q sum_k L^Q_pk R^Q_kq."""
    dR = np.einsum("Qkk->Q", R[:, :o, :o])
    J = np.einsum("Qpq,Q->pq", L, dR)
    K = np.einsum("Qpk,Qkq->pq", L[:, :, :o], R[:, :o, :])
    return J, K


def fock_of(h, pairs, o):
    """f_pq = h_pq + sum_k [2 (pq|kk) - (pk|kq)] for a general DF Hamiltonian."""
    f = np.array(h, dtype=np.float64, copy=True)
    for L, R in pairs:
        J, K = coulomb_exchange(L, R, o)
        f += 2.0 * J - K
    return f


def bare(eps, B, o):
    """Bare Hamiltonian of the synthetic system: Fock = diag(eps), (pq|rs) = B.B.

    Returns (DFHam, h_core, E_ref).  E_ref = sum_i (h_ii + f_ii) is the closed-shell
    reference energy <0|H|0>.
    """
    f = np.diag(eps)
    J, K = coulomb_exchange(B, B, o)
    h = f - (2.0 * J - K)
    e_ref = float(np.trace(h[:o, :o]) + np.trace(f[:o, :o]))
    return DFHam(f, [(B, B)], o, h=h), h, e_ref


def t1_matrix(t1, nmo):
    """Embed t_i^a into an (nmo x nmo) matrix with entries at [i, o + a]."""
    o, v = t1.shape
    m = np.zeros((nmo, nmo))
    m[:o, o:] = t1
    return m


def dress(h, B, t1):
    """T1 similarity transformation H~ = exp(-T1) H exp(T1) (Methods, H-bar definition).

    exp(-T1) a+_p exp(T1) and exp(-T1) a_q exp(T1) are linear in the bare operators,
    so H~ keeps the two-body form with integrals x~ = X^T x Y, X = 1 - t, Y = 1 + t^T,
    where t holds t_i^a at [i, o+a].  Returns the dressed DFHam.
    """
    o = t1.shape[0]
    nmo = h.shape[0]
    t = t1_matrix(t1, nmo)
    X = np.eye(nmo) - t
    Y = np.eye(nmo) + t.T
    hd = X.T @ h @ Y
    Bd = np.einsum("rp,Qrs,sq->Qpq", X, B, Y, optimize=True)
    f = fock_of(hd, [(Bd, Bd)], o)
    return DFHam(f, [(Bd, Bd)], o, h=hd), Bd


def one_index(hd, Bd, r1):
    """Derivative of the T1-dressed Hamiltonian along R1: H' = [H~, R1].

    Dressing with t + e r factorises as (1 - e r)^T H~ (1 + e r^T) because products
    of two occupied-to-virtual matrices vanish, so d/de gives the one-index
    transformation x' = -r^T x~ + x~ r^T for h and for each DF factor.  Two-electron
    integrals of H' follow the product rule: (pq|rs)' = B'.B~ + B~.B'.
    """
    o = r1.shape[0]
    nmo = hd.shape[0]
    r = t1_matrix(r1, nmo)
    hp = -r.T @ hd + hd @ r.T
    Bp = -np.matmul(r.T[None, :, :], Bd) + np.matmul(Bd, r.T[None, :, :])
    pairs = [(Bp, Bd), (Bd, Bp)]
    f = fock_of(hp, pairs, o)
    return DFHam(f, pairs, o, h=hp)


def mp2_amplitudes(eps, B, o):
    """First-order amplitudes t_ij^ab = (ia|jb) / (f_ii + f_jj - f_aa - f_bb) (eq. T1).

    For real orbitals the integral G^{ij}_{ab} of the paper is (ia|jb).  Layout [i,j,a,b].
    """
    Bov = B[:, :o, o:]
    g = np.einsum("Qia,Qjb->ijab", Bov, Bov, optimize=True)
    eo = eps[:o]
    ev = eps[o:]
    d = eo[:, None, None, None] + eo[None, :, None, None] - ev[None, None, :, None] - ev[None, None, None, :]
    return g / d


def mp2_energy(eps, B, o, t2=None):
    """Closed-shell second-order energy sum (ia|jb)(2 t_ij^ab - t_ij^ba)."""
    if t2 is None:
        t2 = mp2_amplitudes(eps, B, o)
    Bov = B[:, :o, o:]
    g = np.einsum("Qia,Qjb->ijab", Bov, Bov, optimize=True)
    return float(np.sum(g * (2.0 * t2 - t2.transpose(0, 1, 3, 2))))
