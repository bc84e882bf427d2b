"""GPU batched symmetric eigensolver (pnoeom_syev_batched, the solver of pnoeom_build_sapno
for pair densities and semicanonical blocks above 128) against LAPACK's (numpy.linalg.eigh),
and the SA-PNO build with it against the oracle.

The eigenvalues are unique and compared directly (2e-14 of the largest).  Eigenvectors are
compared through what is unique about them: each kept vector's residual |A x - lambda x|, the
orthonormality of the kept set, and the projector onto the kept space, which is basis
independent; the kept-space projector moves by about eps |A| / (gap at the cut), so the test
spectra keep that gap at or above 1e-4 |A|.  Counts of kept eigenvalues are exact.
"""
import numpy as np
import pytest

from synthgen import make_system, random_r

pytestmark = pytest.mark.gpu


def _ctx(o=2, v=8, naux=10):
    import torch
    from paper_1802_06738_amd import PnoEom
    assert torch.cuda.is_available()
    return PnoEom(o, v, naux)


def _spectrum_batch(n, seed):
    """Three kinds of symmetric test matrices: a dense random one (all eigenvectors needed),
    a rank-deficient density-like one (eigenvalues 1e-1 .. 1e-12 and exact zeros, kept above
    1e-7 with no eigenvalue in [1e-8, 1e-6]) and one with four-fold degenerate eigenvalues."""
    rng = np.random.default_rng(seed)
    out = []
    a = rng.standard_normal((n, n))
    out.append(a + a.T)
    q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    big = 10.0 ** rng.uniform(-6, -1, n // 3)
    small = 10.0 ** rng.uniform(-12, -8, n // 3)
    w = np.concatenate([big, small, np.zeros(n - 2 * (n // 3))])
    out.append((q * w) @ q.T)
    q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    w = np.resize(np.repeat(rng.uniform(-1.0, 1.0, n // 4 + 1), 4), n)
    out.append((q * w) @ q.T)
    return np.stack([0.5 * (m + m.T) for m in out])


def _check(a, ev, vt, cut):
    for m in range(a.shape[0]):
        wr, vr = np.linalg.eigh(a[m])
        scale = np.max(np.abs(wr))
        assert np.max(np.abs(np.sort(ev[m]) - wr)) <= 2e-14 * scale * np.sqrt(a.shape[1])
        keep = np.abs(ev[m]) >= cut
        keep_r = np.abs(wr) >= cut
        assert keep.sum() == keep_r.sum()
        x = vt[m][keep].T
        assert np.max(np.abs(a[m] @ x - x * ev[m][keep])) <= 1e-12 * scale
        assert np.max(np.abs(x.T @ x - np.eye(x.shape[1]))) <= 1e-12
        p = x @ x.T
        pr = vr[:, keep_r] @ vr[:, keep_r].T
        assert np.max(np.abs(p - pr)) <= 1e-9


@pytest.mark.parametrize("n", [129, 136, 400, 1024])
@pytest.mark.parametrize("backend", [0, 1])
def test_syev_batched_matches_lapack(n, backend):
    import torch
    print(f"[syev n={n} backend={backend}]", flush=True)
    ctx = _ctx()
    ctx.set_eig_backend(backend)
    a = _spectrum_batch(n, 100 + n)
    for cut in (0.0, 1e-7):
        ev, vt = ctx.syev_batched(torch.from_numpy(a).cuda(), cut)
        _check(a, ev.cpu().numpy(), vt.cpu().numpy(), cut)


def test_syev_batched_small_and_split():
    """n = 1 and 2, a diagonal matrix (every off-diagonal zero: T splits everywhere) and a
    zero matrix, through the tridiagonal path's n > 128 dispatch of one batch of 130."""
    import torch
    print("[syev split]", flush=True)
    ctx = _ctx()
    rng = np.random.default_rng(7)
    a = np.zeros((3, 130, 130))
    a[0] = np.diag(rng.uniform(-1, 1, 130))
    b = rng.standard_normal((130, 130))
    a[2] = b + b.T
    ev, vt = ctx.syev_batched(torch.from_numpy(a.copy()).cuda(), 0.0)
    ev, vt = ev.cpu().numpy(), vt.cpu().numpy()
    eps = np.finfo(float).eps
    assert np.max(np.abs(np.sort(ev[0]) - np.sort(np.diag(a[0])))) <= 4 * eps
    assert np.max(np.abs(vt[0] @ vt[0].T - np.eye(130))) <= 1e-13
    assert np.max(np.abs(ev[1])) <= 1e-300
    assert np.max(np.abs(vt[1] @ vt[1].T - np.eye(130))) <= 1e-12
    _check(a[2:], ev[2:], vt[2:], 0.0)
    for n in (1, 2):
        m = rng.standard_normal((4, n, n))
        m = m + m.transpose(0, 2, 1)
        e, v = ctx.syev_batched(torch.from_numpy(m.copy()).cuda(), 0.0)
        _check(m, e.cpu().numpy(), v.cpu().numpy(), 0.0)


@pytest.mark.parametrize("backend", [0, 1])
def test_sapno_v400_counts_and_projector(backend):
    """o = 3, v = 400: pair densities of 400 x 400 (and semicanonical blocks above 128) on
    either backend; PNO/OSV counts exact against the oracle, projector 1e-9."""
    import torch
    from oracle.sapno import sa_densities, PNOBasis
    from oracle.sigma import SigmaOracle
    from paper_1802_06738_amd import PnoEom
    print(f"[sapno v400 backend={backend}]", flush=True)
    o, v, naux, nst, tcut = 3, 400, 120, 2, 1e-6
    s = make_system(o, v, naux, 43, kappa=0.5, t1_sigma=1e-3)
    ctx = PnoEom(o, v, naux)
    ctx.build_df(torch.from_numpy(s.B).cuda(), torch.from_numpy(s.eps).cuda(), torch.from_numpy(s.t1).cuda())
    ctx.set_eig_backend(backend)
    npno, nosv = ctx.build_sapno(nst, tcut)
    so = SigmaOracle(s.eps, s.B, s.o, s.t1)
    eo, _, fvv = so.dressed_fock_diagonals()
    D, _, _ = sa_densities(s.eps, s.B, s.o, nst)
    pb = PNOBasis(D, s.eps, s.o, tcut, fvv=fvv, eo=eo)
    print(f"  PNOs per pair {npno.tolist()}, OSVs {nosv.tolist()}", flush=True)
    assert np.array_equal(npno, pb.npno()) and np.array_equal(nosv, pb.nosv())
    r1, r2 = random_r(o, v, 47, nvec=1)
    x = ctx.pno_compress(torch.from_numpy(r1).cuda(), torch.from_numpy(r2).cuda())
    e1, e2 = ctx.pno_expand(x)
    p1, p2 = pb.project(r1[0], r2[0])
    assert np.max(np.abs(e1.cpu().numpy()[0] - p1)) <= 1e-9 * np.max(np.abs(p1))
    assert np.max(np.abs(e2.cpu().numpy()[0] - p2)) <= 1e-9 * np.max(np.abs(p2))


def test_sigma_memory_and_eig_backend_errors():
    """pnoeom_sigma_memory: ESTATE before build_df (and in the PNO space before build_sapno),
    then bytes per vector at least the vector's own FP64 work arrays, a positive chunk; an
    unknown eigensolver backend is EINVAL."""
    import torch
    from paper_1802_06738_amd import PnoEom, PnoEomError, FP64, BF16, CANONICAL, PNO
    print("[sigma memory]", flush=True)
    o, v, naux = 3, 20, 40
    s = make_system(o, v, naux, 5, kappa=1.0, t1_sigma=1e-3)
    ctx = PnoEom(o, v, naux)
    with pytest.raises(PnoEomError):
        ctx.sigma_memory(CANONICAL, FP64)
    with pytest.raises(PnoEomError):
        ctx.set_eig_backend(2)
    ctx.build_df(torch.from_numpy(s.B).cuda(), torch.from_numpy(s.eps).cuda(), torch.from_numpy(s.t1).cuda())
    per, avail, chunk = ctx.sigma_memory(CANONICAL, FP64)
    assert per >= 8 * o * o * v * v and avail > 0 and chunk >= 1
    assert chunk == max(1, avail // per)
    with pytest.raises(PnoEomError):
        ctx.sigma_memory(PNO, BF16)
    ctx.build_sapno(2, 1e-5)
    per_p, _, chunk_p = ctx.sigma_memory(PNO, BF16)
    assert per_p > 0 and chunk_p >= 1
