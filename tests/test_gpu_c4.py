"""Full-size sigma parity at the o=40, v=400, naux=1200 workload (config 4), through the C ABI,
against the sampled-output oracle's values stored in tests/golden/c4_sigma.json (600 seeded
entries of the sigma2 blocks of pairs (0,1), (5,5), (17,39), (39,39) and sigma1 at three
virtual orbitals, for one seeded trial vector).

FP64: |gpu - oracle| <= 1e-11 max|block| (summation order only; contraction lengths up to
~1e6).  BF16 contractions, scope 0 (ladder and one-pass ring on bfloat16 MFMA, FP32
accumulation): each sigma2 entry within the ladder's rounding bound (2.01 u + K 2^-24) L,
u = 2^-8, K = v(v+1)/2, L = sum_Q sum_cd |B~_ac| (|R_cd| + |R_dc|) |B~_bd| (stored with the
golden), plus 1e-3 (bfloat16 ring; measured 5e-5) + 2e-5 (FP32) of max|block|; sigma1 within
2e-5.  Scope 1 (the default: the hole ladder, X_klij, M1, the DF and R1 ring terms on bfloat16
too): the same plus 2^-8 of max|block| (each product term of two bfloat16-rounded operands
carries at most 2^-8 relative error), sigma1 within 2^-8 of its max.
"""
import json
import os

import numpy as np
import pytest

from synthgen import config_system, random_r

pytestmark = pytest.mark.gpu
GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "c4_sigma.json")


def test_sigma_config4_fp64_and_bf16_on_oracle_samples():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_1802_06738_amd import PnoEom
    g = json.load(open(GOLD))
    print("[sigma c4] o=40 v=400 naux=1200: generating", flush=True)
    s = config_system(4)
    o, v, naux = s.o, s.v, s.naux
    r1, r2 = random_r(o, v, g["seed_r"], nvec=1)
    ctx = PnoEom(o, v, naux)
    ctx.set_bf16_scope(0)
    print("[sigma c4] build_df (FP64 and bfloat16 intermediates, scope 0)", flush=True)
    B, eps, t1 = (torch.from_numpy(x).cuda() for x in (s.B, s.eps, s.t1))
    ctx.build_df(B, eps, t1, precision=2)
    R1, R2 = torch.from_numpy(r1).cuda(), torch.from_numpy(r2).cuda()
    ent = np.array(g["entries2"])
    idx = ent[:, :4].astype(np.int64)
    ref2 = ent[:, 4]
    pairs = [tuple(p) for p in g["pairs"]]
    bmax = {p: m for p, m in zip(pairs, g["block_max"])}
    scale2 = np.array([bmax[(int(i), int(j))] for i, j in idx[:, :2]])
    cols = g["cols"]
    ref1 = np.array(g["sigma1_cols"])
    K = v * (v + 1) // 2
    lad = (2.01 * 2.0 ** -8 + K * 2.0 ** -24) * np.array(g["ladder_abs"])
    for prec in (0, 2, 3):   # 3: BF16 scope 1
        if prec == 3:
            print("[sigma c4] build_df (bfloat16 intermediates, scope 1)", flush=True)
            ctx.set_bf16_scope(1)
            ctx.build_df(B, eps, t1, precision=2)
        print(f"[sigma c4] precision {prec}", flush=True)
        g1, g2 = ctx.sigma(R1, R2, precision=min(prec, 2))
        got2 = g2[0][idx[:, 0], idx[:, 1], idx[:, 2], idx[:, 3]].cpu().numpy()
        got1 = g1[0][:, cols].cpu().numpy()
        del g1, g2
        err2 = np.abs(got2 - ref2)
        err1 = np.abs(got1 - ref1)
        print(f"[sigma c4] precision {prec}: max sigma2 error / block max {np.max(err2 / scale2):.2e}, "
              f"sigma1 {np.max(err1) / np.max(np.abs(ref1)):.2e}", flush=True)
        if prec == 0:
            assert np.all(err2 <= 1e-11 * scale2)
            assert np.max(err1) <= 1e-11 * np.max(np.abs(ref1))
        elif prec == 2:
            assert np.all(err2 <= lad + (1e-3 + 2e-5) * scale2)
            assert np.max(err1) <= 2e-5 * np.max(np.abs(ref1))
            assert np.max(err2 / scale2) > 1e-9   # the bfloat16 path was taken
        else:
            assert np.all(err2 <= lad + (1e-3 + 2e-5 + 2.0 ** -8) * scale2)
            assert np.max(err1) <= 2.0 ** -8 * np.max(np.abs(ref1))
            # scope 1 took its own path: sigma differs from the scope-0 build
            assert np.max(np.abs(got1 - prev[0])) + np.max(np.abs(got2 - prev[1])) > 0.0
        prev = (got1, got2)
    ctx.close()
