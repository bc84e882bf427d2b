"""Closed-shell projected coupled-cluster equations of a general Hamiltonian (oracle).

Test infrastructure: see oracle/__init__.py.

For a two-body Hamiltonian H (any Fock matrix f, any DF integrals with
(pq|rs) = (rs|pq); it need not be Hermitian) and doubles amplitudes T2 only,
the projections of exp(-T2) H exp(T2)|0> onto singles and doubles
(Methods, the projected CC equations) are polynomials in T2:

  Omega1 = c1(H) + l1(H; T2)                       (linear in T2)
  Omega2 = c2(H) + l2(H; T2) + q2(H; T2, T2)        (quadratic in T2)

Singles are read off as the coefficient of a+_{a alpha} a_{i alpha}|0>, doubles as
the coefficient of a+_{a alpha} a_{i alpha} a+_{b beta} a_{j beta}|0>; with the
operator parameterisation of the Methods section that read-off returns t_ij^ab
from T2|0>.  The expressions below are the spin integration of the textbook
spin-orbital CCD equations (Bartlett/Stanton form, T1 = 0) to closed-shell
amplitudes; T1 enters only through the similarity dressing of H (ham.dress).
In q2(X, Y), X is the amplitude outside the intermediate and Y the one inside.

Layouts: T2 and results are [i, j, a, b]; singles are [i, a].
"""
from __future__ import annotations

import numpy as np

ES = dict(optimize=True)


def u_of(t):
    """U_ij^ab = 2 t_ij^ab - t_ij^ba."""
    return 2.0 * t - t.transpose(0, 1, 3, 2)


def psym(z):
    """P_ij^ab z_ij^ab = z_ij^ab + z_ji^ba."""
    return z + z.transpose(1, 0, 3, 2)


def c1(H):
    """<S| H |0> : f_ai, returned as [i, a]."""
    return H.fo("vo").T.copy()


def l1(H, t):
    """Singles projection of [H, T2]: Fock, three-external and three-internal terms."""
    U = u_of(t)
    r = np.einsum("me,imae->ia", H.fo("ov"), U, **ES)
    r += np.einsum("aemf,imef->ia", H.eri("vvov"), U, **ES)
    r -= np.einsum("mine,mnae->ia", H.eri("ooov"), U, **ES)
    return r


def c2(H):
    """<D| H |0> : (ai|bj), returned as [i, j, a, b]."""
    return H.eri("vovo").transpose(1, 3, 0, 2).copy()


def l2(H, t):
    """Doubles projection of [H, T2] (terms linear in T2)."""
    U = u_of(t)
    # particle-particle ladder: sum_cd (ac|bd) t_ij^cd
    o, v = t.shape[1], t.shape[2]
    out = (t.reshape(o * o, v * v) @ H.ladder_matrix().T).reshape(o, o, v, v)
    # hole-hole ladder: sum_kl (ki|lj) t_kl^ab
    out += np.einsum("kilj,klab->ijab", H.eri("oooo"), t, **ES)
    # Fock terms and the particle-hole (ring) terms, symmetrised by P_ij^ab
    z = np.einsum("bc,ijac->ijab", H.fo("vv"), t, **ES)
    z -= np.einsum("kj,ikab->ijab", H.fo("oo"), t, **ES)
    z += np.einsum("kcbj,ikac->ijab", H.eri("ovvo"), U, **ES)
    z -= np.einsum("kjbc,ikac->ijab", H.eri("oovv"), t, **ES)
    z -= np.einsum("kibc,kjac->ijab", H.eri("oovv"), t, **ES)
    return out + psym(z)


def q2(H, X, Y):
    """Doubles projection of 1/2 [[H, T2], T2] written as a bilinear form q2(X, Y)."""
    g = H.eri("ovov")                # (kc|ld) as [k, c, l, d]
    UX = u_of(X)
    UY = u_of(Y)
    # sum_klcd (kc|ld) Y_ij^cd X_kl^ab
    xh = np.einsum("kcld,ijcd->klij", g, Y, **ES)
    out = np.einsum("klab,klij->ijab", X, xh, **ES)
    # Fock-like intermediates built from Y
    fvv = -np.einsum("klbd,kcld->bc", UY, g, **ES)
    foo = np.einsum("jlcd,kcld->kj", UY, g, **ES)
    # ring intermediates built from Y: direct (D) and exchange (E) spin parts
    dq = 0.5 * np.einsum("kcnf,jnbf->kbcj", g, UY, **ES) \
        - 0.5 * np.einsum("kfnc,jnbf->kbcj", g, Y, **ES)
    eq = -0.5 * np.einsum("kfnc,jnfb->kbcj", g, Y, **ES)
    z = np.einsum("bc,ijac->ijab", fvv, X, **ES)
    z -= np.einsum("kj,ikab->ijab", foo, X, **ES)
    z += np.einsum("kbcj,ikac->ijab", dq, UX, **ES)
    z -= np.einsum("kbcj,ikac->ijab", eq, X, **ES)
    z -= np.einsum("kbci,kjac->ijab", eq, X, **ES)
    return out + psym(z)


def residual(H, t2):
    """(Omega1, Omega2) of exp(-T2) H exp(T2)|0> for a (possibly dressed) Hamiltonian."""
    return c1(H) + l1(H, t2), c2(H) + l2(H, t2) + q2(H, t2, t2)


def ccsd_residual(eps, B, o, t1, t2):
    """CCSD residual <mu| exp(-T) H exp(T) |0> of the bare synthetic Hamiltonian.

    T1 is absorbed into the similarity dressing of H (ham.dress); the remaining
    T2 part is the polynomial of this module.
    """
    from .ham import bare, dress
    _, h, _ = bare(eps, B, o)
    Hd, _ = dress(h, B, t1)
    return residual(Hd, t2)
