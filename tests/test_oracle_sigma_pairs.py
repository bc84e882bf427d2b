"""Pins of the sampled-output sigma (oracle/sigma_pairs.py) against the full oracle sigma,
itself pinned to the brute-force determinant engine: the same equations evaluated only at
listed pairs (i, j) and virtual orbitals a, with T1 != 0, given or first-order T2, random R."""
import numpy as np
import pytest

from synthgen import make_system, random_r
from oracle.sigma import SigmaOracle
from oracle.sigma_pairs import PairSigmaOracle, eri_sel, ladder_block


def _sym(x):
    return 0.5 * (x + x.transpose(1, 0, 3, 2))


@pytest.mark.parametrize("o,v,naux,seed,given_t2", [(3, 7, 11, 1, False), (4, 9, 13, 2, True), (5, 6, 9, 3, False)])
def test_pair_sigma_equals_full_sigma(o, v, naux, seed, given_t2):
    s = make_system(o, v, naux, seed, t1_sigma=0.05)
    rng = np.random.default_rng(seed)
    t2 = _sym(rng.standard_normal((o, o, v, v)) * 0.05) if given_t2 else None
    full = SigmaOracle(s.eps, s.B, o, s.t1, t2)
    part = PairSigmaOracle(s.eps, s.B, o, s.t1, t2)
    r1, r2 = random_r(o, v, seed + 7)
    a1, a2 = full.sigma(r1[0], r2[0])
    pairs = [(0, 0), (0, o - 1), (o - 1, 1), (1, 1), (2, 0)]
    cols = [0, v - 1, 2]
    b1, b2 = part.sigma(r1[0], r2[0], pairs, cols)
    for (i, j) in pairs:
        assert np.max(np.abs(b2[(i, j)] - a2[i, j])) <= 1e-12 * np.max(np.abs(a2))
    assert np.max(np.abs(b1 - a1[:, cols])) <= 1e-12 * np.max(np.abs(a1))


def test_pair_sigma_helpers():
    """The restricted integral blocks and the per-block ladder against the full forms."""
    s = make_system(3, 6, 10, 5, t1_sigma=0.05)
    part = PairSigmaOracle(s.eps, s.B, 3, s.t1)
    H = part.Hd
    full = H.eri("ovvo")
    assert np.allclose(eri_sel(H, "ovvo", (None, [1, 2], None, [0])), full[:, [1, 2]][:, :, :, [0]], atol=1e-14)
    x = np.random.default_rng(3).standard_normal((6, 6))
    W = H.ladder_matrix()
    assert np.allclose(ladder_block(H, x).ravel(), W @ x.ravel(), atol=1e-13)
