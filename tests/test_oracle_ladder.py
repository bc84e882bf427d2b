"""Pins of the oracle's particle-particle ladder (CPU only).

The ladder term sum_cd (ac|bd)~ R_ij^cd of sigma2 is pinned
  * by brute force: for a Hamiltonian whose factors vanish whenever an index is
    occupied (no occupied-orbital integrals, so T2 = 0 and no other term couples
    doubles to doubles), sigma2 of a doubles-only R at T = 0 is
    (e_a + e_b - e_i - e_j) R + ladder(R), read off the determinant engine;
  * against the sigma oracle (itself pinned to the determinant engine) on the same
    kind of Hamiltonian at a larger size;
  * by the row-by-row form used for sampled entries of large systems, with T1 != 0;
  * by the exact symmetries W_ab^cd = W_ba^dc (so ladder(X^T) = ladder(X)^T) and linearity.
"""
import numpy as np
import pytest

from synthgen import make_system, random_r, random_blocks
from oracle.ham import bare
from oracle.fci import FCI, full_eri
from oracle.sigma import SigmaOracle
from oracle.ladder import ladder_apply, ladder_entries, dressed_virtual_factors, ladder_from_factors


def _vv_only(s):
    o = s.o
    B = s.B.copy()
    B[:, :o, :] = 0.0
    B[:, :, :o] = 0.0
    return B


def _denom(eps, o):
    eo, ev = eps[:o], eps[o:]
    return ev[None, None, :, None] + ev[None, None, None, :] - eo[:, None, None, None] - eo[None, :, None, None]


@pytest.mark.parametrize("o,v,seed", [(2, 3, 21), (2, 4, 22)])
def test_ladder_equals_brute_force_doubles_block(o, v, seed):
    s = make_system(o, v, 10, seed, sigma_b=0.12)
    B = _vv_only(s)
    _, h, _ = bare(s.eps, B, o)
    f = FCI(h, full_eri(B), o)
    _, r2 = random_r(o, v, seed + 1)
    r2 = r2[0]
    b1, b2 = f.sigma(np.zeros((o, v)), np.zeros((o, o, v, v)), np.zeros((o, v)), r2)
    lad = ladder_apply(B, o, None, r2.reshape(o * o, v, v)).reshape(o, o, v, v)
    assert np.max(np.abs(b1)) < 1e-13
    ref = b2 - _denom(s.eps, o) * r2
    assert np.max(np.abs(lad - ref)) < 1e-12 * np.max(np.abs(ref))
    assert np.max(np.abs(lad)) > 1e-3  # the term is not trivially zero


def test_ladder_equals_sigma_oracle_doubles_block():
    o, v, seed = 3, 9, 23
    s = make_system(o, v, 20, seed)
    B = _vv_only(s)
    _, r2 = random_r(o, v, seed + 1)
    r2 = r2[0]
    so = SigmaOracle(s.eps, B, o, np.zeros((o, v)), np.zeros((o, o, v, v)))
    _, s2 = so.sigma(np.zeros((o, v)), r2)
    lad = ladder_apply(B, o, None, r2.reshape(o * o, v, v)).reshape(o, o, v, v)
    ref = s2 - _denom(s.eps, o) * r2
    assert np.max(np.abs(lad - ref)) < 1e-12 * np.max(np.abs(ref))


def test_ladder_rows_form_matches_full_with_t1():
    o, v, naux = 4, 11, 17
    s = make_system(o, v, naux, 24, t1_sigma=0.1)
    X = random_blocks(v, 3, 25)
    Y = ladder_apply(s.B, o, s.t1, X)
    rng = np.random.default_rng(26)
    samples = [(int(rng.integers(3)), int(rng.integers(v)), int(rng.integers(v))) for _ in range(40)]
    samples += [(0, 0, 0), (2, v - 1, v - 1), (1, 0, v - 1)]
    got = ladder_entries(s.B, o, s.t1, X, samples)
    want = np.array([Y[m, a, b] for m, a, b in samples])
    assert np.max(np.abs(got - want)) < 1e-13 * np.max(np.abs(Y))
    # the dressing changes the answer (so the test sees T1)
    Y0 = ladder_apply(s.B, o, None, X)
    assert np.max(np.abs(Y - Y0)) > 1e-3 * np.max(np.abs(Y))


def test_ladder_symmetry_and_linearity():
    o, v, naux = 3, 8, 12
    s = make_system(o, v, naux, 27, t1_sigma=0.05)
    X = random_blocks(v, 2, 28)
    Y = ladder_apply(s.B, o, s.t1, X)
    Yt = ladder_apply(s.B, o, s.t1, X.transpose(0, 2, 1))
    assert np.max(np.abs(Yt - Y.transpose(0, 2, 1))) < 1e-13 * np.max(np.abs(Y))
    Z = ladder_apply(s.B, o, s.t1, 2.0 * X[:1] - 0.5 * X[1:])
    assert np.max(np.abs(Z - (2.0 * Y[:1] - 0.5 * Y[1:]))) < 1e-13 * np.max(np.abs(Y))
    F = dressed_virtual_factors(s.B, o, s.t1)
    assert np.array_equal(ladder_from_factors(F, X), Y)
