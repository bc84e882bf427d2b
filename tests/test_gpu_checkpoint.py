"""Checkpoint, abort and resume of the Davidson (through the C ABI).

A run stopped by abort_after_iter returns EABORTED after writing the Ritz vectors of
that iteration; resuming from them reaches the roots of an uninterrupted run to 1e-10 Eh
(FP64; both converged with tol_e = 1e-11, tol_r = 1e-8).  A checkpoint of the FP64
refinement of a mixed run resumes in the refinement.  Mismatched or unreadable files are
refused with EINVAL.  The failure is forced from the host; every kernel exits normally.
"""
import os

import numpy as np
import pytest

from synthgen import config_system, make_system

pytestmark = pytest.mark.gpu
TOL = dict(tol_e=1e-11, tol_r=1e-8)


def _ctx(s, precision=0):
    import torch
    from paper_1802_06738_amd import PnoEom
    assert torch.cuda.is_available()
    ctx = PnoEom(s.o, s.v, s.naux)
    ctx.build_df(torch.from_numpy(s.B).cuda(), torch.from_numpy(s.eps).cuda(), torch.from_numpy(s.t1).cuda(),
                 precision=precision)
    return ctx


def test_abort_and_resume_fp64(tmp_path):
    print("[ckpt fp64]", flush=True)
    from paper_1802_06738_amd import PnoEomError
    s = config_system(1)
    ctx = _ctx(s)
    full = ctx.davidson(3, **TOL)
    path = str(tmp_path / "c1.ckpt")
    with pytest.raises(PnoEomError) as e:
        ctx.davidson(3, abort_after_iter=5, ckpt_path=path, **TOL)
    assert e.value.code == -7 and os.path.exists(path)
    res = ctx.davidson(3, resume_path=path, **TOL)
    assert np.max(np.abs(res["omega"] - full["omega"])) <= 1e-10
    assert res["iters"] < full["iters"]
    # periodic checkpoints do not change the result
    per = ctx.davidson(3, ckpt_every=2, ckpt_path=str(tmp_path / "p.ckpt"), **TOL)
    assert np.array_equal(per["omega"], full["omega"])


def test_resume_mixed_in_both_phases(tmp_path):
    print("[ckpt mixed]", flush=True)
    from paper_1802_06738_amd import PnoEomError
    s = make_system(4, 20, 60, 41, t1_sigma=1e-3)
    ctx = _ctx(s, precision=1)
    ref = ctx.davidson(3, **TOL)
    p0 = str(tmp_path / "m0.ckpt")
    with pytest.raises(PnoEomError) as e:
        ctx.davidson(3, precision=1, refine_fp64=True, abort_after_iter=3, ckpt_path=p0, **TOL)
    assert e.value.code == -7
    r0 = ctx.davidson(3, precision=1, refine_fp64=True, resume_path=p0, **TOL)
    assert np.max(np.abs(r0["omega"] - ref["omega"])) <= 1e-10
    # the last periodic checkpoint of a full mixed run is one of its FP64 refinement
    p1 = str(tmp_path / "m1.ckpt")
    ctx.davidson(3, precision=1, refine_fp64=True, ckpt_every=1, ckpt_path=p1, **TOL)
    r1 = ctx.davidson(3, precision=1, refine_fp64=True, resume_path=p1, **TOL)
    assert np.max(np.abs(r1["omega"] - ref["omega"])) <= 1e-10


def test_resume_refuses_mismatched_or_broken_files(tmp_path):
    print("[ckpt refuse]", flush=True)
    from paper_1802_06738_amd import PnoEomError
    s = config_system(1)
    ctx = _ctx(s)
    path = str(tmp_path / "a.ckpt")
    with pytest.raises(PnoEomError):
        ctx.davidson(3, abort_after_iter=2, ckpt_path=path, **TOL)
    other = make_system(4, 21, 60, 5)
    ctx2 = _ctx(other)
    with pytest.raises(PnoEomError) as e:
        ctx2.davidson(3, resume_path=path, **TOL)
    assert e.value.code == -1
    bad = tmp_path / "bad.ckpt"
    bad.write_bytes(b"not a checkpoint")
    with pytest.raises(PnoEomError) as e:
        ctx.davidson(3, resume_path=str(bad), **TOL)
    assert e.value.code == -1
    with pytest.raises(PnoEomError) as e:
        ctx.davidson(3, resume_path=str(tmp_path / "missing.ckpt"), **TOL)
    assert e.value.code == -1


def test_iteration_log(tmp_path):
    print("[davidson log]", flush=True)
    import json
    s = config_system(1)
    ctx = _ctx(s)
    log = tmp_path / "it.jsonl"
    r = ctx.davidson(3, log_path=str(log), **TOL)
    lines = [json.loads(x) for x in log.read_text().splitlines()]
    assert len(lines) == r["iters"]
    assert [x["it"] for x in lines] == list(range(1, r["iters"] + 1))
    assert np.allclose(lines[-1]["omega"], r["omega"], atol=0, rtol=0)
    assert all(len(x["resnorm"]) == 3 and x["m"] >= 3 for x in lines)
    assert lines[-1]["resnorm"][0] <= 1e-8 and lines[-1]["nsigma"] == r["nsigma"]
    # cumulative sigma time: positive, non-decreasing, below the elapsed time
    sig = [x["sigma_seconds"] for x in lines]
    assert sig[0] > 0 and all(b >= a for a, b in zip(sig, sig[1:]))
    assert all(x["sigma_seconds"] <= x["seconds"] + 1e-6 for x in lines)
