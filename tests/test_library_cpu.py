"""CPU checks of the C-ABI library: it loads, exports every declared symbol, and its
host-side eigensolver agrees with LAPACK (no GPU calls)."""
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _lib():
    from paper_1802_06738_amd import pnoeom
    if not os.path.exists(pnoeom.library_path()):
        from paper_1802_06738_amd import build_lib
        build_lib.build()
    return pnoeom.load_library()


def test_header_symbols_exported():
    lib = _lib()
    hdr = open(os.path.join(ROOT, "include", "pnoeom.h")).read()
    declared = set(re.findall(r"\b(pnoeom_[a-z_0-9]+)\s*\(", hdr))
    from paper_1802_06738_amd.pnoeom import EXPORTED_SYMBOLS
    assert declared == set(EXPORTED_SYMBOLS)
    for name in declared:
        assert getattr(lib, name) is not None


@pytest.mark.parametrize("n,seed", [(1, 0), (2, 1), (7, 2), (25, 3), (60, 4)])
def test_host_eig_matches_lapack(n, seed):
    _lib()
    from paper_1802_06738_amd import host_eig
    rng = np.random.default_rng(seed)
    a = rng.standard_normal((n, n)) + np.diag(np.linspace(0, 3, n))
    w, vr = host_eig(a)
    ref = np.linalg.eigvals(a)
    ref = ref[np.lexsort((-ref.imag, ref.real))]
    assert np.max(np.abs(w - ref)) < 1e-11 * max(1.0, np.abs(ref).max())
    for k in range(n):
        if abs(w[k].imag) == 0.0:
            assert np.linalg.norm(a @ vr[:, k] - w[k].real * vr[:, k]) < 1e-10


def test_host_eig_nearly_symmetric_degenerate():
    _lib()
    from paper_1802_06738_amd import host_eig
    rng = np.random.default_rng(7)
    q, _ = np.linalg.qr(rng.standard_normal((12, 12)))
    d = np.array([1.0, 1.0, 2.0, 3.0, 3.0, 3.0, 4, 5, 6, 7, 8, 9])
    a = q @ np.diag(d) @ q.T
    w, vr = host_eig(a)
    assert np.allclose(w.real, np.sort(d), atol=1e-12)
    # vectors of the degenerate eigenvalues are independent
    assert np.linalg.matrix_rank(vr[:, :2], tol=1e-6) == 2
    assert np.linalg.matrix_rank(vr[:, 3:6], tol=1e-6) == 3


def test_host_eig_rejects_bad_input():
    lib = _lib()
    assert lib.pnoeom_host_eig(0, None, None, None, None) == -1


@pytest.mark.parametrize("n,seed,kind", [(1, 0, "rand"), (2, 1, "rand"), (3, 2, "rand"), (40, 3, "rand"),
                                         (161, 4, "rand"), (130, 5, "decay"), (50, 6, "degenerate"),
                                         (30, 7, "zero"), (60, 8, "diag")])
def test_host_syev_matches_lapack(n, seed, kind):
    """The host symmetric eigensolver of the PNO build: eigenvalues against LAPACK,
    residual and orthonormality of the vectors, on random, fast-decaying (pair-density
    like), degenerate, zero and diagonal matrices."""
    _lib()
    from paper_1802_06738_amd import host_syev
    rng = np.random.default_rng(seed)
    if kind == "rand":
        x = rng.standard_normal((n, n))
        a = x + x.T
    elif kind == "decay":
        q, _ = np.linalg.qr(rng.standard_normal((n, n)))
        d = np.sign(rng.standard_normal(n)) * 10.0 ** rng.uniform(-14, -1, n)
        a = (q * d) @ q.T
    elif kind == "degenerate":
        q, _ = np.linalg.qr(rng.standard_normal((n, n)))
        d = np.repeat(np.arange(n // 5), 5).astype(float)
        a = (q * d) @ q.T
    elif kind == "zero":
        a = np.zeros((n, n))
    else:
        a = np.diag(rng.standard_normal(n))
    a = 0.5 * (a + a.T)
    w, v = host_syev(a)
    ref = np.linalg.eigvalsh(a)
    scale = max(1.0, np.abs(ref).max())
    assert np.max(np.abs(np.sort(w) - ref)) <= 1e-12 * scale
    assert np.max(np.abs(a @ v - v * w)) <= 1e-12 * scale
    assert np.max(np.abs(v.T @ v - np.eye(n))) <= 1e-12


def test_gemm_tuning_table_validation():
    """The tuning entry points validate their input without touching the GPU."""
    import ctypes as C
    lib = _lib()
    keys = (C.c_longlong * 8)(8, 0, 0, 0, 64, 64, 64, 1)
    bad = (C.c_int * 1)(12)
    assert lib.pnoeom_gemm_set_table(1, keys, bad) != 0
    assert lib.pnoeom_gemm_set_table(-1, keys, bad) != 0
    ok = (C.c_int * 1)(4)
    assert lib.pnoeom_gemm_set_table(1, keys, ok) == 0
    assert lib.pnoeom_gemm_record(1) == 0
    assert lib.pnoeom_gemm_recorded(None, 0) == 0
    assert lib.pnoeom_gemm_record(0) == 0
    from paper_1802_06738_amd.autotune import DEFAULT_TABLE, load_table, clear_table, default_variant
    clear_table(lib)
    if os.path.exists(DEFAULT_TABLE):
        assert load_table(DEFAULT_TABLE, lib) >= 0
    assert default_variant((8, 0, 0, 0, 3000, 3000, 3000, 1)) == 0
    assert default_variant((8, 0, 1, 0, 6, 9000000, 40, 1)) == 6
    assert default_variant((8, 0, 0, 0, 40, 40, 9000000, 1)) == 3


def test_library_emits_roctx_ranges():
    """The library links the roctx marker library and opens named ranges (entry points,
    sigma blocks, Davidson iterations, CCSD steps) that rocprofv3 --marker-trace records."""
    import shutil
    import subprocess
    from paper_1802_06738_amd.pnoeom import library_path
    nm = shutil.which("nm")
    if nm is None:
        pytest.skip("nm not available")
    out = subprocess.run([nm, "-D", "--undefined-only", library_path()], capture_output=True, text=True).stdout
    assert "roctxRangePushA" in out and "roctxRangePop" in out
