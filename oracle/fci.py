"""Brute-force determinant engine: the plain definition on tiny cases (oracle).

Test infrastructure: see oracle/__init__.py.

Slater determinants of o alpha and o beta electrons in nmo spatial orbitals are
pairs of occupation bit strings; a determinant is |alpha string>|beta string>
with creators in ascending orbital order, alpha before beta.  The spin-summed
excitation operator E_pq = sum_s a+_{ps} a_{qs} is kron(e_pq, 1) + kron(1, e_pq)
with e_pq its matrix on one spin's strings.  H, T and R are assembled from E_pq
exactly as written in the Methods section, and
  Omega_mu = <mu| exp(-T) H exp(T) |0>,   sigma_mu = <mu| exp(-T) [H, R] exp(T) |0>
are evaluated with sparse matrix-vector products (T is nilpotent, so the
exponential series ends).  Read-off: singles from a+_{a alpha} a_{i alpha}|0>,
doubles from a+_{a alpha} a_{i alpha} a+_{b beta} a_{j beta}|0>.
"""
from __future__ import annotations

import itertools
import math

import numpy as np
import scipy.sparse as sp


def _strings(nmo, nel):
    out = []
    for occ in itertools.combinations(range(nmo), nel):
        m = 0
        for p in occ:
            m |= 1 << p
        out.append(m)
    return out


def _popcount_below(s, p):
    return bin(s & ((1 << p) - 1)).count("1")


class FCISpace:
    def __init__(self, nmo, o):
        self.nmo = nmo
        self.o = o
        self.strs = _strings(nmo, o)
        self.index = {s: k for k, s in enumerate(self.strs)}
        self.ns = len(self.strs)
        self.dim = self.ns * self.ns
        self._e = {}
        self._E = {}
        hf = (1 << o) - 1
        self.hf = self.index[hf] * self.ns + self.index[hf]

    def e_str(self, p, q):
        """a+_p a_q on one spin's strings (sparse ns x ns)."""
        key = (p, q)
        if key in self._e:
            return self._e[key]
        rows, cols, vals = [], [], []
        for k, s in enumerate(self.strs):
            if not (s >> q) & 1:
                continue
            sign = (-1) ** _popcount_below(s, q)
            s1 = s & ~(1 << q)
            if (s1 >> p) & 1:
                continue
            sign *= (-1) ** _popcount_below(s1, p)
            s2 = s1 | (1 << p)
            rows.append(self.index[s2])
            cols.append(k)
            vals.append(float(sign))
        m = sp.csr_matrix((vals, (rows, cols)), shape=(self.ns, self.ns))
        self._e[key] = m
        return m

    def E(self, p, q):
        key = (p, q)
        if key not in self._E:
            e = self.e_str(p, q)
            one = sp.identity(self.ns, format="csr")
            self._E[key] = (sp.kron(e, one) + sp.kron(one, e)).tocsr()
        return self._E[key]

    def ham_apply(self, h, eri):
        """Return a function x -> H x with H from core h and (pq|rs) (full nmo^4)."""
        n = self.nmo

        def apply(x):
            y = np.zeros_like(x)
            Ex = {}
            for r in range(n):
                for s in range(n):
                    Ex[(r, s)] = self.E(r, s) @ x
            for p in range(n):
                for q in range(n):
                    if h[p, q] != 0.0:
                        y += h[p, q] * Ex[(p, q)]
                    acc = np.zeros_like(x)
                    for r in range(n):
                        for s in range(n):
                            c = eri[p, q, r, s]
                            if c != 0.0:
                                acc += c * Ex[(r, s)]
                    y += 0.5 * (self.E(p, q) @ acc)
                    # - 1/2 sum_s (pq|qs)-type term: - d_qr E_ps
                    for s in range(n):
                        c = eri[p, q, q, s]
                        if c != 0.0:
                            y -= 0.5 * c * Ex[(p, s)]
            return y
        return apply

    def excitation_op(self, r1, r2):
        """R = sum_ia r_i^a E_ai + 1/2 sum_ijab r_ij^ab E_ai E_bj as a sparse matrix."""
        o = self.o
        op = sp.csr_matrix((self.dim, self.dim))
        v = r1.shape[1]
        for i in range(o):
            for a in range(v):
                if r1[i, a] != 0.0:
                    op = op + r1[i, a] * self.E(o + a, i)
        for i in range(o):
            for j in range(o):
                for a in range(v):
                    for b in range(v):
                        c = r2[i, j, a, b]
                        if c != 0.0:
                            op = op + (0.5 * c) * (self.E(o + a, i) @ self.E(o + b, j))
        return op.tocsr()

    def ref(self):
        x = np.zeros(self.dim)
        x[self.hf] = 1.0
        return x

    def readoff(self, vec, v):
        """Singles [i,a] and doubles [i,j,a,b] coefficients of a state vector."""
        o = self.o
        one = sp.identity(self.ns, format="csr")
        ref = self.ref()
        s1 = np.zeros((o, v))
        s2 = np.zeros((o, o, v, v))
        for i in range(o):
            for a in range(v):
                u = sp.kron(self.e_str(o + a, i), one) @ ref
                s1[i, a] = u @ vec
        for i in range(o):
            for a in range(v):
                ua = self.e_str(o + a, i)
                for j in range(o):
                    for b in range(v):
                        u = sp.kron(ua, self.e_str(o + b, j)) @ ref
                        s2[i, j, a, b] = u @ vec
        return s1, s2


def _expm_apply(op, x, sign=1.0):
    out = x.copy()
    term = x.copy()
    for n in range(1, 64):
        term = (sign / n) * (op @ term)
        if not np.any(term):
            break
        out += term
    return out


class FCI:
    """Brute-force H, H-bar, Omega and sigma for a tiny closed-shell system."""

    def __init__(self, h, eri, o):
        self.nmo = h.shape[0]
        self.o = o
        self.v = self.nmo - o
        self.space = FCISpace(self.nmo, o)
        self.h = h
        self.eri = eri
        self.H = self.space.ham_apply(h, eri)

    def energy_ref(self):
        x = self.space.ref()
        return float(x @ self.H(x))

    def omega(self, t1, t2):
        T = self.space.excitation_op(t1, t2)
        x = _expm_apply(T, self.space.ref(), 1.0)
        x = self.H(x)
        x = _expm_apply(T, x, -1.0)
        return self.space.readoff(x, self.v)

    def sigma(self, t1, t2, r1, r2):
        S = self.space
        T = S.excitation_op(t1, t2)
        R = S.excitation_op(r1, r2)
        x = _expm_apply(T, S.ref(), 1.0)
        y = self.H(R @ x) - R @ self.H(x)
        y = _expm_apply(T, y, -1.0)
        return S.readoff(y, self.v)

    def apply_R(self, r1, r2):
        R = self.space.excitation_op(r1, r2)
        return self.space.readoff(R @ self.space.ref(), self.v)

    def h_matrix_dense(self):
        n = self.space.dim
        cols = []
        for k in range(n):
            e = np.zeros(n)
            e[k] = 1.0
            cols.append(self.H(e))
        return np.array(cols).T

    def excitation_level(self):
        """Number of alpha+beta electrons outside the reference orbitals, per determinant."""
        S = self.space
        occ_mask = (1 << self.o) - 1
        lev = np.zeros(S.dim, dtype=int)
        for ka, sa in enumerate(S.strs):
            la = bin(sa & ~occ_mask).count("1")
            for kb, sb in enumerate(S.strs):
                lev[ka * S.ns + kb] = la + bin(sb & ~occ_mask).count("1")
        return lev

    def orbital_energy_sum(self, eps):
        """sum of eps over occupied orbitals of each determinant (MP zeroth order)."""
        S = self.space
        e = np.zeros(S.dim)
        es = np.zeros(S.ns)
        for k, s in enumerate(S.strs):
            es[k] = sum(eps[p] for p in range(self.nmo) if (s >> p) & 1)
        for ka in range(S.ns):
            e[ka * S.ns:(ka + 1) * S.ns] = es[ka] + es
        return e


def full_eri(B):
    n = B.shape[1]
    return np.einsum("Qpq,Qrs->pqrs", B, B).reshape(n, n, n, n)


def n_determinants(nmo, o):
    return math.comb(nmo, o) ** 2
