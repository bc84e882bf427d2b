"""Davidson eigensolver with the PNO modification, and dense diagonalisation (oracle).

Test infrastructure: see oracle/__init__.py.

The paper specifies only the PNO modification of the Davidson correction step
(residual -> OSV/PNO basis -> preconditioner -> back-transform); the remaining
steps are the standard non-Hermitian block Davidson method:
  1. guess: the lowest k CIS vectors (singles only), projected by P
  2. orthonormalise (two passes of classical Gram-Schmidt, full-array Frobenius
     inner product over all i, j, a, b plus singles)
  3. sigma of every new vector, then P sigma
  4. G = V^T (P sigma); eigenpairs of G sorted by real part; keep the lowest k
  5. Ritz vectors x = V y, residuals r = (P sigma) y - theta x
  6. converged when ||r_k|| <= tol_r and |theta_k - theta_k(prev)| <= tol_e for all k
  7. correction for every unconverged root: the preconditioner of the basis
     (canonical, or the PNO/OSV one), normalised, orthogonalised, and dropped if
     the norm left after orthogonalisation is < 1e-10
  8. collapse to the tracked Ritz vectors when the subspace would exceed max_sub
nextra Ritz pairs beyond the k target roots are tracked (guessed from the next
CIS vectors and kept at collapse) but need not converge; they speed up the
highest target roots.  A complex pair of Ritz values is handled with its real
parts (reported).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla


def pack(r1, r2):
    return np.concatenate([r1.ravel(), r2.ravel()])


def unpack(x, o, v):
    n1 = o * v
    return x[:n1].reshape(o, v), x[n1:].reshape(o, o, v, v)


def _orth_against(V, x, passes=2):
    """Classical Gram-Schmidt against the orthonormal V; the second pass only when the first
    removed more than half of the squared norm ("twice is enough")."""
    if not V:
        return x
    M = np.array(V)
    n0 = float(x @ x)
    for p in range(passes):
        x = x - M.T @ (M @ x)
        if p == 0 and float(x @ x) >= 0.5 * n0:
            break
    return x


def davidson(sigma, basis, guess, o, v, nroots, tol_e=1e-8, tol_r=None, max_sub=60,
             max_iter=200, verbose=False, nextra=0):
    """Lowest-real-part EOM roots of x -> P sigma(x) on range(P).

    sigma(r1, r2) -> (s1, s2); basis provides project() and precondition().
    guess: list of (r1, r2).  Returns dict(omega, resnorm, iters, vectors, complex).
    """
    if tol_r is None:
        tol_r = 0.1 * np.sqrt(tol_e)

    def psig(x):
        s1, s2 = sigma(*unpack(x, o, v))
        return pack(*basis.project(s1, s2))

    V, S = [], []
    for g in guess:
        x = pack(*basis.project(*g))
        x = _orth_against(V, x)
        nrm = np.linalg.norm(x)
        if nrm > 1e-10:
            V.append(x / nrm)
    S = [psig(x) for x in V]
    theta_old = None
    had_complex = False
    ntarget = nroots
    nk = nroots + nextra
    for it in range(1, max_iter + 1):
        Vm = np.array(V)
        Sm = np.array(S)
        G = Vm @ Sm.T
        w, Y = sla.eig(G)
        order = np.argsort(w.real, kind="stable")
        w = w[order][:nk]
        Y = Y[:, order][:, :nk]
        if np.any(np.abs(w.imag) > 0):
            had_complex = True
        theta = w.real
        Y = Y.real
        Y = Y / np.linalg.norm(Vm.T @ Y, axis=0)[None, :]
        X = Vm.T @ Y
        Rr = Sm.T @ Y - X * theta[None, :]
        rn = np.linalg.norm(Rr, axis=0)
        de = np.abs(theta - theta_old) if theta_old is not None else np.full(nk, np.inf)
        conv = (rn <= tol_r) & (de <= tol_e)
        conv[ntarget:] = True
        if verbose:
            print(f"it {it:3d} m {len(V):3d} theta {theta[:ntarget]} |r| {rn[:ntarget]}")
        if np.all(conv):
            return dict(omega=theta[:ntarget], resnorm=rn[:ntarget], iters=it, vectors=X[:, :ntarget],
                        complex=had_complex)
        theta_old = theta
        new = []
        # preconditioned residuals; if every one of them lies in span(V), the residuals
        # themselves (orthogonal to V by the Galerkin condition V^T r = 0)
        for precondition in (True, False):
            for k in range(ntarget):
                if conv[k]:
                    continue
                if precondition:
                    c1, c2 = basis.precondition(*unpack(Rr[:, k], o, v), theta[k])
                    x = pack(*basis.project(c1, c2))
                else:
                    x = Rr[:, k].copy()
                x = x / np.linalg.norm(x)
                x = _orth_against(V + new, x)
                nrm = np.linalg.norm(x)
                if nrm < 1e-10:
                    continue
                new.append(x / nrm)
            if new:
                break
        if not new:
            # nothing outside span(V) is left: the Ritz values cannot change any more, so
            # residuals within tol_r are final
            if np.all(rn[:ntarget] <= tol_r):
                return dict(omega=theta[:ntarget], resnorm=rn[:ntarget], iters=it, vectors=X[:, :ntarget],
                            complex=had_complex)
            raise RuntimeError("Davidson stalled: no new directions")
        if len(V) + len(new) > max_sub:
            Q, _ = np.linalg.qr(Y)
            V = list((Vm.T @ Q).T)
            S = list((Sm.T @ Q).T)
            new2 = []
            for x in new:
                x = _orth_against(V + new2, x)
                nrm = np.linalg.norm(x)
                if nrm >= 1e-10:
                    new2.append(x / nrm)
            new = new2
        V.extend(new)
        S.extend(psig(x) for x in new)
    raise RuntimeError("Davidson did not converge")


def singlet_basis(o, v):
    """Orthonormal basis (full-array Frobenius) of the space with R2[i,j,a,b] = R2[j,i,b,a].

    Independent parameters: R1[i,a]; R2 for i < j (all a, b); R2 for i == j, a <= b.
    Returns a list of (index tuple list, weight) describing each basis vector.
    """
    n1 = o * v
    out = []
    for i in range(o):
        for a in range(v):
            out.append(([i * v + a], [1.0]))

    def idx(i, j, a, b):
        return n1 + ((i * o + j) * v + a) * v + b

    s = 1.0 / np.sqrt(2.0)
    for i in range(o):
        for j in range(i, o):
            for a in range(v):
                for b in range(v):
                    if i == j and b < a:
                        continue
                    if i == j and a == b:
                        out.append(([idx(i, i, a, a)], [1.0]))
                    else:
                        out.append(([idx(i, j, a, b), idx(j, i, b, a)], [s, s]))
    return out


def dense_eom(sigma, o, v, basis=None):
    """Eigenvalues of the EOM map on the singlet space (or range(P)), sorted by real part.

    The matrix is built column by column from sigma of orthonormal basis vectors.
    With a PNO basis the columns span range(P) (Q^T H-bar Q of the PNO simulation).
    """
    if basis is None:
        cols = singlet_basis(o, v)
        n = o * v + o * o * v * v
        Q = np.zeros((n, len(cols)))
        for k, (ix, wt) in enumerate(cols):
            Q[ix, k] = wt
    else:
        Q = pno_range_basis(basis, o, v)
    M = np.zeros((Q.shape[1], Q.shape[1]))
    for k in range(Q.shape[1]):
        s1, s2 = sigma(*unpack(Q[:, k], o, v))
        M[:, k] = Q.T @ pack(s1, s2)
    w = sla.eigvals(M)
    return w[np.argsort(w.real, kind="stable")], M


def pno_range_basis(basis, o, v):
    """Orthonormal columns spanning range(P) for a PNOBasis."""
    cols = []
    n1 = o * v
    for i in range(o):
        U = basis.osv[i]
        for k in range(U.shape[1]):
            x = np.zeros(n1 + o * o * v * v)
            x[i * v:(i + 1) * v] = U[:, k]
            cols.append(x)
    for (i, j), U in basis.pno.items():
        n = U.shape[1]
        for a in range(n):
            for b in range(n):
                if i == j and b < a:
                    continue
                e = np.zeros((n, n))
                e[a, b] = 1.0
                if i == j:
                    e = e + e.T if a != b else e
                blk = U @ e @ U.T
                r2 = np.zeros((o, o, v, v))
                r2[i, j] = blk
                r2[j, i] = blk.T
                x = np.concatenate([np.zeros(n1), r2.ravel()])
                cols.append(x / np.linalg.norm(x))
    return np.array(cols).T
