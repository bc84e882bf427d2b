"""Write the stored reference values under tests/golden/ (calls only oracle/ and synthgen).

    python tests/golden/make_golden.py c1 c1_pno pno_small c2 c2_sigma

Each section writes <section>.json with the excitation energies of the FP64
oracle (Davidson at tol_e = 1e-11, and for config 1 also the dense eigenvalues
of H-bar on the singlet space), plus the setup numbers (E_ref, E_MP2, CIS
energies, PNO counts) that the GPU tests compare against.  Section c2_sigma
stores seeded samples of one oracle sigma vector at the full config-2 size.
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from synthgen import config_system, CONFIGS                       # noqa: E402
from oracle.ham import bare, mp2_energy                           # noqa: E402
from oracle.sigma import SigmaOracle                              # noqa: E402
from oracle.sapno import cis_roots, sa_densities, PNOBasis, CanonicalBasis   # noqa: E402
from oracle.davidson import davidson, dense_eom                   # noqa: E402


def _setup(cfg):
    s = config_system(cfg)
    so = SigmaOracle(s.eps, s.B, s.o, s.t1)
    out = dict(config=str(cfg), o=s.o, v=s.v, naux=s.naux, seed=s.seed, sigma_b=s.sigma_b,
               kappa=s.kappa, e_ref=so.e_ref, e_mp2=mp2_energy(s.eps, s.B, s.o))
    return s, so, out


def _guess(b, o, v, k):
    return [(b[i], np.zeros((o, o, v, v))) for i in range(k)]


def sec_c1():
    s, so, out = _setup(1)
    o, v, k = s.o, s.v, CONFIGS[1]["nroots"]
    w, b = cis_roots(s.eps, s.B, o, k)
    out["cis"] = w.tolist()
    t0 = time.time()
    res = davidson(so.sigma, CanonicalBasis(s.eps, o, *so.dressed_fock_diagonals()[:2]), _guess(b, o, v, k), o, v, k,
                   tol_e=1e-11, tol_r=1e-8)
    out["davidson"] = res["omega"].tolist()
    out["davidson_iters"] = res["iters"]
    out["davidson_seconds"] = time.time() - t0
    wd, _ = dense_eom(so.sigma, o, v)
    out["dense_eig"] = wd.real[:12].tolist()
    out["dense_eig_imag"] = wd.imag[:12].tolist()
    return out


def _pno_section(cfg, tcut, nstates):
    s, so, out = _setup(cfg)
    o, v = s.o, s.v
    k = CONFIGS[cfg]["nroots"]
    D, w, b = sa_densities(s.eps, s.B, o, nstates)
    pb = PNOBasis(D, s.eps, o, tcut)
    out.update(cis=w.tolist(), tcut_pno=tcut, tcut_osv=tcut / 10.0, nstates_avg=nstates,
               npno=pb.npno().tolist(), nosv=pb.nosv().tolist())
    t0 = time.time()
    res = davidson(so.sigma, pb, _guess(b, o, v, k), o, v, k, tol_e=1e-11, tol_r=1e-8)
    out["davidson_pno"] = res["omega"].tolist()
    out["davidson_pno_iters"] = res["iters"]
    out["davidson_pno_seconds"] = time.time() - t0
    t0 = time.time()
    rc = davidson(so.sigma, CanonicalBasis(s.eps, o, *so.dressed_fock_diagonals()[:2]), _guess(b, o, v, k), o, v, k,
                  tol_e=1e-11, tol_r=1e-8)
    out["davidson"] = rc["omega"].tolist()
    out["davidson_iters"] = rc["iters"]
    out["davidson_seconds"] = time.time() - t0
    return out


def sec_c1_pno():
    return _pno_section(1, 1e-6, CONFIGS[1]["nroots"])


def sec_pno_small():
    return _pno_section("pno_small", CONFIGS["pno_small"]["tcut"], CONFIGS["pno_small"]["nroots"])


def sec_c2():
    s, so, out = _setup(2)
    o, v, k = s.o, s.v, CONFIGS[2]["nroots"]
    ne = CONFIGS[2]["nextra"]
    w, b = cis_roots(s.eps, s.B, o, k + ne)
    out["cis"] = w[:k].tolist()
    out["nextra"] = ne
    t0 = time.time()
    res = davidson(so.sigma, CanonicalBasis(s.eps, o, *so.dressed_fock_diagonals()[:2]), _guess(b, o, v, k + ne), o, v, k,
                   tol_e=1e-10, tol_r=1e-7, max_sub=CONFIGS[2]["max_sub"], nextra=CONFIGS[2]["nextra"],
                   max_iter=400, verbose=True)
    out["davidson"] = res["omega"].tolist()
    out["davidson_resnorm"] = res["resnorm"].tolist()
    out["davidson_iters"] = res["iters"]
    out["davidson_seconds"] = time.time() - t0
    return out


def sec_c2_sigma():
    """sigma of one seeded trial vector at config 2, sampled at seeded positions."""
    from synthgen import random_r
    s, so, out = _setup(2)
    o, v = s.o, s.v
    seed_r = 2024
    r1, r2 = random_r(o, v, seed_r, nvec=1)
    t0 = time.time()
    s1, s2 = so.sigma(r1[0], r2[0])
    out["sigma_seconds"] = time.time() - t0
    rng = np.random.default_rng(77)
    i1 = rng.choice(s1.size, size=300, replace=False)
    i2 = rng.choice(s2.size, size=3000, replace=False)
    out.update(seed_r=seed_r, idx1=i1.tolist(), val1=s1.ravel()[i1].tolist(), idx2=i2.tolist(),
               val2=s2.ravel()[i2].tolist(), norm1=float(np.linalg.norm(s1)), norm2=float(np.linalg.norm(s2)),
               max1=float(np.max(np.abs(s1))), max2=float(np.max(np.abs(s2))))
    return out


def sec_c4_sigma():
    """sigma of one seeded trial vector at the config-4 size (o=40, v=400, naux=1200), from the
    sampled-output oracle: seeded entries of the sigma2 blocks of a few pairs (diagonal,
    off-diagonal, first and last occupied) and of sigma1 at a few virtual orbitals."""
    from synthgen import random_r
    from oracle.sigma_pairs import PairSigmaOracle
    from oracle.ladder import ladder_entries
    s = config_system(4)
    o, v = s.o, s.v
    out = dict(config="4", o=o, v=v, naux=s.naux, seed=s.seed)
    seed_r = 2026
    r1, r2 = random_r(o, v, seed_r, nvec=1)
    pairs = [(0, 1), (5, 5), (17, 39), (39, 39)]
    cols = [0, 133, 399]
    t0 = time.time()
    po = PairSigmaOracle(s.eps, s.B, o, s.t1)
    s1, s2 = po.sigma(r1[0], r2[0], pairs, cols)
    out["sigma_seconds"] = time.time() - t0
    rng = np.random.default_rng(78)
    ent = []
    for (i, j) in pairs:
        ab = rng.choice(v * v, size=600, replace=False)
        for e in ab:
            a, b = divmod(int(e), v)
            ent.append([i, j, a, b, float(s2[(i, j)][a, b])])
    out.update(seed_r=seed_r, pairs=pairs, cols=cols, sigma1_cols=s1.tolist(), entries2=ent,
               block_max=[float(np.max(np.abs(s2[p]))) for p in pairs],
               block_norm=[float(np.linalg.norm(s2[p])) for p in pairs])
    # bfloat16 rounding scale of the ladder at the same entries (sum |B~||R||B~|, both c-d orders)
    t0 = time.time()
    X = r2[0].reshape(o * o, v, v)
    samples = [(i * o + j, a, b) for i, j, a, b, _ in ent]
    out["ladder_abs"] = ladder_entries(s.B, o, s.t1, X, samples, absolute=True).tolist()
    out["ladder_abs_seconds"] = time.time() - t0
    return out


if __name__ == "__main__":
    for name in sys.argv[1:]:
        t0 = time.time()
        res = globals()["sec_" + name]()
        res["wall_seconds"] = time.time() - t0
        with open(os.path.join(os.environ.get("GOLDEN_OUT", HERE), name + ".json"), "w") as fh:
            json.dump(res, fh, indent=1)
        print(name, "done in", round(time.time() - t0, 1), "s", flush=True)
