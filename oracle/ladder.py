"""Particle-particle ladder term of sigma2 (oracle).

Test infrastructure: see oracle/__init__.py.

The ladder intermediate of the Methods section (the largest one) is the vvvv block
of the two-electron integrals of the T1-dressed Hamiltonian H~ = exp(-T1) H exp(T1),
W_ab^cd = (ac|bd)~.  It acts on each pair's doubles block on its own:
    Y_ij^ab = sum_cd (ac|bd)~ R_ij^cd.
With density fitting (Computational Details) (ac|bd)~ = sum_Q B~^Q_ac B~^Q_bd, so for
one v x v block X
    Y = sum_Q B~^Q X (B~^Q)^T.
"""
from __future__ import annotations

import numpy as np

from .ham import dress


def dressed_virtual_factors(B, o, t1=None):
    """B~^Q_ac for virtual a, c from the T1 similarity transformation of ham.dress
    (the core operator does not enter the factors, so a zero one is passed)."""
    B = np.asarray(B, dtype=np.float64)
    nmo = B.shape[1]
    if t1 is None:
        t1 = np.zeros((o, nmo - o))
    _, Bd = dress(np.zeros((nmo, nmo)), B, t1)
    return np.ascontiguousarray(Bd[:, o:, o:])


def ladder_from_factors(F, X):
    """Y[m] = sum_Q F^Q X[m] (F^Q)^T for factors F [naux, v, v] and blocks X [n, v, v]."""
    F = np.asarray(F, dtype=np.float64)
    X = np.asarray(X, dtype=np.float64)
    return np.einsum("Qac,mcd,Qbd->mab", F, X, F, optimize=True)


def ladder_apply(B, o, t1, X):
    """Ladder term sum_cd (ac|bd)~ X[m][c][d] of the dressed Hamiltonian for blocks X [n, v, v]."""
    return ladder_from_factors(dressed_virtual_factors(B, o, t1), X)


def dressed_rows(B, o, t1, rows):
    """B~^Q_{r,:} of the virtual rows r only, written out from the transformation
    (1 - t)^T B (1 + t^T): the left factor subtracts sum_k t_k^r B^Q_{k,:} from row r,
    the right factor leaves virtual columns unchanged.  Returns [naux, len(rows), v]."""
    B = np.asarray(B)
    rows = np.asarray(rows, dtype=np.int64)
    out = np.array(B[:, o + rows, o:], dtype=np.float64)
    if t1 is not None:
        out -= np.einsum("kr,Qkc->Qrc", np.asarray(t1)[:, rows], B[:, :o, o:], optimize=True)
    return out


def ladder_entries(B, o, t1, X, samples, absolute=False):
    """Y[m][a][b] for the listed (m, a, b) triples, one row a of one block at a time
    (for systems too large for the full W).  absolute=True gives instead
    sum_Q sum_cd |B~^Q_ac| (|X_cd| + |X_dc|) |B~^Q_bd|, the scale of rounding-error bounds."""
    samples = [tuple(int(x) for x in s) for s in samples]
    need = sorted({s[1] for s in samples} | {s[2] for s in samples})
    pos = {r: k for k, r in enumerate(need)}
    F = dressed_rows(B, o, t1, need)          # [naux, nrows, v]
    if absolute:
        F = np.abs(F)
    out = np.empty(len(samples))
    cache = {}
    for k, (m, a, b) in enumerate(samples):
        if (m, a) not in cache:
            x = np.asarray(X[m], dtype=np.float64)
            if absolute:
                x = np.abs(x) + np.abs(x).T
            cache[(m, a)] = F[:, pos[a], :] @ x   # [naux, v]
        out[k] = float(np.sum(cache[(m, a)] * F[:, pos[b], :]))
    return out
