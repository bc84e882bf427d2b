"""The bfloat16 MFMA GEMM kernels (128 x 128 and 256 x 256 tiles) through the C ABI.

Reference: the same bfloat16 operands multiplied in FP64 on the host (bfloat16 values
are exact in FP64, so the reference is the exact product).  The kernels form each
product exactly and accumulate in FP32, so |C - ref| <= (K + 10) 2^-24 sum_k |a_k| |b_k|
elementwise (K additions of unit round-off, up to 7 more where K is split and the partials
are summed, plus the alpha / beta step).
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

SHAPES = [(256, 256, 64), (300, 520, 192), (513, 777, 320), (1030, 260, 640), (40, 700, 128),
          (1300, 3400, 64),    # 6 x 14 tiles of 256: XCD chunks and a ragged last tile-column group
          (300, 520, 4096),    # 6 tiles of 256 and a long K: split K (4 partials) in variants 0 and 3
          (182, 2900, 3200)]   # fewer rows than a 256 tile: clamped rows, split K


def _torch():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return torch


@pytest.mark.parametrize("M,N,K", SHAPES)
@pytest.mark.parametrize("variant", [0, 1, 2, 3, 4, 5])
def test_gemm_bf16_matches_exact_product(M, N, K, variant):
    print(f"[gemm bf16] variant {variant} M={M} N={N} K={K}", flush=True)
    torch = _torch()
    from paper_1802_06738_amd import gemm_bf16, PnoEomError
    g = torch.Generator().manual_seed(M * 7 + N * 3 + K)
    A = torch.randn((M, K), generator=g).to(torch.bfloat16)
    B = torch.randn((N, K), generator=g).to(torch.bfloat16)
    C0 = torch.randn((M, N), generator=g, dtype=torch.float32)
    Ad, Bd = A.cuda(), B.cuda()
    if variant >= 2 and (M < 160 or N < 160):
        with pytest.raises(PnoEomError):
            gemm_bf16(Ad, Bd, torch.zeros((M, N), dtype=torch.float32, device="cuda"), variant=variant)
        return
    a = A.double().numpy()
    b = B.double().numpy()
    ref = a @ b.T
    bound = (K + 10) * 2.0 ** -24 * (np.abs(a) @ np.abs(b).T)
    C = gemm_bf16(Ad, Bd, torch.full((M, N), float("nan"), dtype=torch.float32, device="cuda"),
                  variant=variant).cpu().double().numpy()
    assert np.all(np.abs(C - ref) <= bound), float(np.max(np.abs(C - ref) / bound))
    # alpha and beta
    Cb = gemm_bf16(Ad, Bd, C0.cuda(), alpha=-0.5, beta=2.0, variant=variant).cpu().double().numpy()
    ref2 = -0.5 * ref + 2.0 * C0.double().numpy()
    bound2 = 0.5 * bound + 2.0 ** -23 * (np.abs(ref2) + 1.0)
    assert np.all(np.abs(Cb - ref2) <= bound2), float(np.max(np.abs(Cb - ref2) / bound2))
