"""EOM-CCSD sigma vector sigma = <mu| [H-bar, R] |0> (oracle).

Test infrastructure: see oracle/__init__.py.

With H-bar = exp(-T) H exp(T) (Methods) and R an excitation operator of the same
form as T (R1 amplitudes B^i_a, R2 amplitudes B^ij_ab in the paper's notation),
R commutes with T, so
    [H-bar, R] = d/de exp(-(T + eR)) H exp(T + eR) |_{e=0}.
The sigma vector is therefore the directional derivative of the CCSD residual of
the residual module along R:
  * the R1 part differentiates the T1 dressing, giving the Hamiltonian H' of
    ham.one_index, which enters the T2-polynomial linearly;
  * the R2 part differentiates the T2-polynomial at the dressed Hamiltonian.
    sigma1 = c1(H') + l1(H'; T2) + l1(H~; R2)
    sigma2 = c2(H') + l2(H'; T2) + q2(H'; T2, T2)
           + l2(H~; R2) + q2(H~; T2, R2) + q2(H~; R2, T2)
This commutator (connected) form is the definition used for any T, including
the MP2 amplitudes of the synthetic workloads that do not solve the CCSD
equations (for a CCSD solution it equals <mu|(H-bar - E_CC) R|0>).
R2 must satisfy R2[i,j,a,b] = R2[j,i,b,a]; the result has the same symmetry.
"""
from __future__ import annotations

import numpy as np

from .ham import bare, dress, one_index, mp2_amplitudes
from .residual import c1, c2, l1, l2, q2


class SigmaOracle:
    """Holds the dressed Hamiltonian for fixed (eps, B, T1, T2) and evaluates sigma."""

    def __init__(self, eps, B, o, t1=None, t2=None):
        self.o = o
        self.v = B.shape[1] - o
        self.eps = np.asarray(eps, dtype=np.float64)
        _, h, self.e_ref = bare(self.eps, B, o)
        if t1 is None:
            t1 = np.zeros((o, self.v))
        if t2 is None:
            t2 = mp2_amplitudes(self.eps, B, o)
        self.t1 = t1
        self.t2 = t2
        self.Hd, self.Bd = dress(h, B, t1)

    def sigma(self, r1, r2):
        Hp = one_index(self.Hd.h, self.Bd, r1)
        t2 = self.t2
        s1 = c1(Hp) + l1(Hp, t2) + l1(self.Hd, r2)
        s2 = c2(Hp) + l2(Hp, t2) + q2(Hp, t2, t2)
        s2 += l2(self.Hd, r2) + q2(self.Hd, t2, r2) + q2(self.Hd, r2, t2)
        return s1, s2

    def dressed_fock_diagonals(self):
        """Diagonal of the one-particle part of H-bar at fixed T: f~ + the T2 terms.

        F_kj = f~_kj + sum_lcd U_jl^cd (kc|ld),  F_bc = f~_bc - sum_kld U_kl^bd (kc|ld).
        Used only by the Davidson preconditioner (convergence, not results).
        """
        from .residual import u_of
        g = self.Hd.eri("ovov")
        U = u_of(self.t2)
        foo = self.Hd.fo("oo") + np.einsum("jlcd,kcld->kj", U, g, optimize=True)
        fvv = self.Hd.fo("vv") - np.einsum("klbd,kcld->bc", U, g, optimize=True)
        return np.diag(foo).copy(), np.diag(fvv).copy(), fvv

    def sigma_terms(self, r1, r2):
        """The R2-driven doubles pieces one by one (for per-term parity)."""
        Hd = self.Hd
        lad = np.einsum("acbd,ijcd->ijab", Hd.eri("vvvv"), r2, optimize=True)
        return {"ladder": lad}
