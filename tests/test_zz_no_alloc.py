"""The allocation-free ladder entry point (pnoeom_ladder_apply_noalloc) against
pnoeom_ladder_apply, through the C ABI.

Both run the same packing and MFMA kernels; the allocation-free one never splits K,
so FP64 and FP32 agree to the summation-order bounds of the ladder tests (FP64
1e-12 of max|Y|; FP32 twice the FP32 bound (naux + v+ + 6) 2^-24 L elementwise)
and BF16 bit for bit (at these sizes, under 160 rows, both take the 128 x 128 bfloat16
kernel, which never splits K).  Each precision makes two calls in a row,
the second with fewer matrices, after calls of another precision have left other
data in the shared scratch array.
"""
import numpy as np
import pytest

from synthgen import make_system, random_blocks
from oracle.ladder import ladder_apply, dressed_virtual_factors, ladder_from_factors

pytestmark = pytest.mark.gpu

U32 = 2.0 ** -24


def _torch():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return torch


def _fp32_bound(s, X, naux, v):
    F = np.abs(dressed_virtual_factors(s.B, s.o, s.t1))
    Z = np.abs(X) + np.abs(X).transpose(0, 2, 1)
    return (naux + v * (v + 1) // 2 + 6) * U32 * ladder_from_factors(F, Z)


def test_ladder_noalloc_matches_ladder_apply():
    torch = _torch()
    from paper_1802_06738_amd import PnoEom, LADDER_CACHED
    o, v, naux = 4, 37, 53
    s = make_system(o, v, naux, 91, t1_sigma=1e-2)
    B, eps, t1 = (torch.from_numpy(x).cuda() for x in (s.B, s.eps, s.t1))
    for prec in (0, 1, 2):
        ctx = PnoEom(o, v, naux)
        ctx.set_ladder_mode(LADDER_CACHED)
        ctx.build_df(B, eps, t1, precision=prec)
        for call, nmat in enumerate((23, 7)):
            print(f"[ladder noalloc] precision {prec} call {call} nmat={nmat} v={v}", flush=True)
            X = random_blocks(v, nmat, 92 + 10 * prec + call)
            Xd = torch.from_numpy(X).cuda()
            ref = ctx.ladder_apply(Xd, precision=prec).cpu().numpy()
            out = torch.full_like(Xd, float("nan"))
            got = ctx.ladder_apply_noalloc(Xd, out, precision=prec).cpu().numpy()
            assert got.shape == (nmat, v, v)
            if prec == 0:
                exact = ladder_apply(s.B, o, s.t1, X)
                assert np.max(np.abs(got - ref)) <= 1e-12 * np.max(np.abs(ref))
                assert np.max(np.abs(got - exact)) <= 1e-12 * np.max(np.abs(exact))
            elif prec == 1:
                assert np.all(np.abs(got - ref) <= 2.0 * _fp32_bound(s, X, naux, v))
            else:
                assert np.array_equal(got, ref)
        ctx.close()


def test_ladder_noalloc_limits_and_errors():
    torch = _torch()
    from paper_1802_06738_amd import PnoEom, PnoEomError, LADDER_CACHED, LADDER_STREAMED
    o, v, naux = 2, 60, 30
    s = make_system(o, v, naux, 93, t1_sigma=1e-2)
    B, eps, t1 = (torch.from_numpy(x).cuda() for x in (s.B, s.eps, s.t1))
    ctx = PnoEom(o, v, naux)
    X = torch.from_numpy(random_blocks(v, 3, 94)).cuda()
    out = torch.empty_like(X)
    print("[ladder noalloc] before build", flush=True)
    with pytest.raises(PnoEomError) as e:
        ctx.ladder_apply_noalloc(X, out)
    assert e.value.code == -5
    ctx.set_ladder_mode(LADDER_CACHED)
    ctx.build_df(B, eps, t1)
    lim = ctx.ladder_noalloc_limit(0)
    vp, vm = v * (v + 1) // 2, v * (v - 1) // 2
    assert 0 < lim and lim * 16 * (vp + vm) <= 128 << 20 < (lim + 1) * 16 * (vp + vm) + 4 * 256
    print(f"[ladder noalloc] limit {lim}: nmat = limit + 1 refused on the host", flush=True)
    big = torch.zeros((lim + 1, v, v), dtype=torch.float64, device="cuda")
    with pytest.raises(PnoEomError) as e:
        ctx.ladder_apply_noalloc(big, torch.empty_like(big))
    assert e.value.code == -1
    del big
    print("[ladder noalloc] empty batch, precision not built", flush=True)
    assert ctx.ladder_apply_noalloc(X[:0], out[:0]).shape == (0, v, v)
    with pytest.raises(PnoEomError) as e:
        ctx.ladder_apply_noalloc(X, out, precision=2)
    assert e.value.code == -1
    print("[ladder noalloc] largest accepted batch", flush=True)
    Xl = torch.from_numpy(random_blocks(v, lim, 95)).cuda()
    got = ctx.ladder_apply_noalloc(Xl, torch.empty_like(Xl)).cpu().numpy()
    ref = ctx.ladder_apply(Xl).cpu().numpy()
    assert np.max(np.abs(got - ref)) <= 1e-12 * np.max(np.abs(ref))
    del Xl
    print("[ladder noalloc] streamed ladder refused", flush=True)
    ctx2 = PnoEom(o, v, naux)
    ctx2.set_ladder_mode(LADDER_STREAMED, 4)
    ctx2.build_ladder(B, t1)
    with pytest.raises(PnoEomError) as e:
        ctx2.ladder_apply_noalloc(X, out)
    assert e.value.code == -1
