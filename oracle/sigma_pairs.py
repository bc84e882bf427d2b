"""EOM-CCSD sigma at selected outputs, for systems too large for the full oracle (oracle).

Test infrastructure: see oracle/__init__.py.

The full oracle (sigma.py) forms the dense v^2 x v^2 ladder matrix and every
integral block at once (at o = 40, v = 400 the ladder matrix alone takes 205 GB).
This module evaluates the same closed-shell equations -- sigma as the directional
derivative of the CC residual along R (sigma.py), with the terms of residual.py --
only at the outputs asked for:
  * sigma2 blocks [a, b] of listed pairs (i, j);
  * sigma1 columns [i, a] of listed virtual orbitals a.
Each term is the term of residual.c2 / l2 / q2 / c1 / l1 with its output indices
fixed; integral blocks are formed from the DF factors, (pq|rs) = sum_t sum_Q
L_t^Q_pq R_t^Q_rs, only over the index ranges those outputs touch, and the particle
ladder of one pair block X is sum_t sum_Q L_t^Q X (R_t^Q)^T.  The P_ij^ab
symmetrisation of the ring-type terms needs their (j, i) block next to (i, j).
"""
from __future__ import annotations

import numpy as np

from .ham import bare, dress, one_index, mp2_amplitudes
from .residual import u_of

ES = dict(optimize=True)


def _orb(H, c, sel):
    """Absolute orbital indices of class c ('o' / 'v'), all or the listed ones."""
    base = np.arange(H.o) if c == "o" else H.o + np.arange(H.nmo - H.o)
    return base if sel is None else base[np.asarray(sel, dtype=np.int64)]


def eri_sel(H, spec, sel=(None, None, None, None)):
    """(pq|rs) of H for p, q, r, s of the classes in spec (e.g. 'ovvo'), each index all or listed."""
    ip, iq, ir, i_s = (_orb(H, c, x) for c, x in zip(spec, sel))
    out = 0.0
    for L, R in H.pairs:
        a = L[:, ip][:, :, iq]
        b = R[:, ir][:, :, i_s]
        out = out + np.tensordot(a, b, axes=([0], [0]))
    return out


def ladder_block(H, x):
    """sum_cd (ac|bd) x_cd of H for one v x v block x."""
    o = H.o
    y = 0.0
    for L, R in H.pairs:
        lx = np.matmul(L[:, o:, o:], x)                   # [Q, a, d] = sum_c L_ac x_cd
        y = y + np.tensordot(lx, R[:, o:, o:], axes=([0, 2], [0, 2]))   # sum_Qd lx_Qad R_Qbd
    return y


class _Blocks:
    """Integral blocks of one Hamiltonian shared by the terms of one sigma evaluation."""

    def __init__(self, H):
        self.H = H
        self._c = {}

    def get(self, key, fn):
        if key not in self._c:
            self._c[key] = fn()
        return self._c[key]

    def ovov(self):
        return self.get("ovov", lambda: eri_sel(self.H, "ovov"))

    def ovvo_col(self, y):   # (kc|by) as [k, c, b]
        return self.get(("ovvo", y), lambda: eri_sel(self.H, "ovvo", (None, None, None, [y]))[:, :, :, 0])

    def oovv_row(self, y):   # (ky|bc) as [k, b, c]
        return self.get(("oovv", y), lambda: eri_sel(self.H, "oovv", (None, [y], None, None))[:, 0])


def _l2_pair(Hb, t, U, i, j):
    """residual.l2 at the block (i, j)."""
    H = Hb.H

    def z(x, y):
        r = t[x, y] @ H.fo("vv").T                                   # sum_c f_bc t_xy^ac
        r -= np.einsum("k,kab->ab", H.fo("oo")[:, y], t[x], **ES)    # sum_k f_ky t_xk^ab
        r += np.einsum("kcb,kac->ab", Hb.ovvo_col(y), U[x], **ES)    # (kc|by) U_xk^ac
        r -= np.einsum("kbc,kac->ab", Hb.oovv_row(y), t[x], **ES)    # (ky|bc) t_xk^ac
        r -= np.einsum("kbc,kac->ab", Hb.oovv_row(x), t[:, y], **ES)  # (kx|bc) t_ky^ac
        return r

    out = ladder_block(H, t[i, j])
    g = eri_sel(H, "oooo", (None, [i], None, [j]))[:, 0, :, 0]       # (ki|lj)
    out += np.einsum("kl,klab->ab", g, t, **ES)
    return out + z(i, j) + z(j, i).T


class _Q2:
    """residual.q2(H; X, Y) at selected pairs; the Y-intermediates are formed on demand."""

    def __init__(self, Hb, X, Y):
        self.g = Hb.ovov()                         # (kc|ld) as [k, c, l, d]
        self.X, self.Y = X, Y
        self.UX, self.UY = u_of(X), u_of(Y)
        self.fvv = -np.einsum("klbd,kcld->bc", self.UY, self.g, **ES)
        self.foo = np.einsum("jlcd,kcld->kj", self.UY, self.g, **ES)
        self._dq, self._eq = {}, {}

    def dq(self, y):   # dq_kbcy as [k, b, c]
        if y not in self._dq:
            g, UY, Y = self.g, self.UY, self.Y
            self._dq[y] = 0.5 * np.einsum("kcnf,nbf->kbc", g, UY[y], **ES) \
                - 0.5 * np.einsum("kfnc,nbf->kbc", g, Y[y], **ES)
        return self._dq[y]

    def eq(self, y):   # eq_kbcy as [k, b, c]
        if y not in self._eq:
            self._eq[y] = -0.5 * np.einsum("kfnc,nfb->kbc", self.g, self.Y[y], **ES)
        return self._eq[y]

    def pair(self, i, j):
        X, UX = self.X, self.UX
        xh = np.einsum("kcld,cd->kl", self.g, self.Y[i, j], **ES)
        out = np.einsum("klab,kl->ab", X, xh, **ES)

        def z(x, y):
            r = X[x, y] @ self.fvv.T
            r -= np.einsum("k,kab->ab", self.foo[:, y], X[x], **ES)
            r += np.einsum("kbc,kac->ab", self.dq(y), UX[x], **ES)
            r -= np.einsum("kbc,kac->ab", self.eq(y), X[x], **ES)
            r -= np.einsum("kbc,kac->ab", self.eq(x), X[:, y], **ES)
            return r

        return out + z(i, j) + z(j, i).T


def _l1_cols(H, t, cols):
    """residual.l1 at the virtual orbitals listed in cols: [i, a]."""
    U = u_of(t)
    cols = np.asarray(cols, dtype=np.int64)
    r = np.einsum("me,imae->ia", H.fo("ov"), U[:, :, cols], **ES)
    r += np.einsum("aemf,imef->ia", eri_sel(H, "vvov", (cols, None, None, None)), U, **ES)
    r -= np.einsum("mine,mnae->ia", eri_sel(H, "ooov"), U[:, :, cols], **ES)
    return r


class PairSigmaOracle:
    """sigma of one trial vector at selected outputs, for fixed (eps, B, T1, T2)."""

    def __init__(self, eps, B, o, t1=None, t2=None):
        self.o = o
        self.v = B.shape[1] - o
        self.eps = np.asarray(eps, dtype=np.float64)
        _, h, self.e_ref = bare(self.eps, B, o)
        if t1 is None:
            t1 = np.zeros((o, self.v))
        if t2 is None:
            t2 = mp2_amplitudes(self.eps, B, o)
        self.t1, self.t2 = t1, t2
        self.Hd, self.Bd = dress(h, B, t1)

    def prepare(self, r1, r2):
        """The parts of one trial vector's sigma that every output shares: the R1-transformed
        Hamiltonian H', the U combinations of T2 and R2, and the three q2 evaluators."""
        t2 = self.t2
        Hp = one_index(self.Hd.h, self.Bd, r1)
        bp, bd = _Blocks(Hp), _Blocks(self.Hd)
        return dict(r1=r1, r2=r2, Hp=Hp, bp=bp, bd=bd, ut=u_of(t2), ur=u_of(r2), q_ptt=_Q2(bp, t2, t2),
                    q_dtr=_Q2(bd, t2, r2), q_drt=_Q2(bd, r2, t2))

    def pair(self, st, i, j):
        """sigma2 block [a, b] of pair (i, j) for a prepared trial vector."""
        t2, r2 = self.t2, st["r2"]
        blk = eri_sel(st["Hp"], "vovo", (None, [i], None, [j]))[:, 0, :, 0]     # c2(H') = (ai|bj)'
        blk = blk + _l2_pair(st["bp"], t2, st["ut"], i, j) + st["q_ptt"].pair(i, j)
        blk += _l2_pair(st["bd"], r2, st["ur"], i, j) + st["q_dtr"].pair(i, j) + st["q_drt"].pair(i, j)
        return blk

    def cols(self, st, cols):
        """sigma1 [i, len(cols)] at the listed virtual orbitals for a prepared trial vector."""
        cols = np.asarray(cols, dtype=np.int64)
        Hp = st["Hp"]
        return Hp.fo("vo")[cols].T.copy() + _l1_cols(Hp, self.t2, cols) + _l1_cols(self.Hd, st["r2"], cols)

    def sigma(self, r1, r2, pairs, cols=()):
        """(sigma1[:, cols] as [i, len(cols)], {(i, j): sigma2 block [a, b]}) of (r1, r2),
        the same equations as SigmaOracle.sigma:
          sigma1 = c1(H') + l1(H'; T2) + l1(H~; R2)
          sigma2 = c2(H') + l2(H'; T2) + q2(H'; T2, T2) + l2(H~; R2) + q2(H~; T2, R2) + q2(H~; R2, T2)."""
        st = self.prepare(r1, r2)
        s2 = {(i, j): self.pair(st, i, j) for (i, j) in pairs}
        s1 = self.cols(st, cols) if len(cols) else None
        return s1, s2
