"""Seeded synthetic inputs for the closed-shell EOM-CCSD sigma / Davidson path.

This module only draws random numbers and lays them out; it holds none of the
method's arithmetic (no integrals, no amplitudes, no Fock builds).  Both the
FP64 oracle (tests) and the HIP path (bench, GPU tests) take their inputs from
here, so the two sides see bit-identical data.

Recipe (one seeded PCG64 stream, fixed draw order):
  1. occupied orbital energies  eps_occ ~ U[-1.5, -0.3] Eh, sorted ascending
  2. virtual orbital energies   eps_vir ~ U[ 0.1,  3.0] Eh, sorted ascending
  3. density-fitting factors    B^Q_pq for p <= q ~ N(0, sigma_B^2), Q-major,
                                each Q row in row-major upper-triangle order,
                                then mirrored so B^Q_pq = B^Q_qp
  4. optional T1 amplitudes     t_i^a ~ N(0, sigma_t1^2)
The Fock matrix is diag(eps) by construction, so Brillouin's condition f_ia = 0
holds exactly.  sigma_B defaults to 0.05 * (4*20^2*60 / (o*v^2*naux))^(1/4): the
literal 0.05 at o=4, v=20, naux=60, scaled so that the second-order correlation
energy per occupied orbital (proportional to o v^2 naux sigma_B^4) stays at that
workload's level as o, v and naux grow.  Independent Gaussian factors couple every
pair equally, so without this scaling the correlation grows like o^2 v^2 and the
doubles dominate H-bar (second-order energy -207 Eh at o=20, v=150, naux=450,
excitation energies near 10.7 Eh).  An optional virtual
envelope multiplies B^Q_pq by g_p g_q with g_i = 1 and
g_a = exp(-kappa (eps_a - eps_LUMO)); it gives the per-pair densities the
eigenvalue decay that real molecules show.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

__all__ = ["System", "make_system", "default_sigma_b", "CONFIGS", "config_system", "random_r", "random_blocks"]


@dataclasses.dataclass
class System:
    o: int
    v: int
    naux: int
    eps: np.ndarray          # (o+v,)  occupied first, each block ascending
    B: np.ndarray            # (naux, o+v, o+v) float64, symmetric in p,q
    t1: np.ndarray           # (o, v) float64 (zeros when not drawn)
    seed: int
    sigma_b: float
    kappa: float

    @property
    def nmo(self) -> int:
        return self.o + self.v


def default_sigma_b(o: int, v: int, naux: int) -> float:
    return 0.05 * (4.0 * 20.0 ** 2 * 60.0 / (o * v * v * naux)) ** 0.25


def make_system(o: int, v: int, naux: int, seed: int, *, sigma_b: float | None = None,
                kappa: float = 0.0, t1_sigma: float = 0.0, chunk: int = 64) -> System:
    if o < 1 or v < 1 or naux < 1:
        raise ValueError("o, v and naux must be positive")
    if sigma_b is None:
        sigma_b = default_sigma_b(o, v, naux)
    rng = np.random.Generator(np.random.PCG64(seed))
    eps_o = np.sort(rng.uniform(-1.5, -0.3, o))
    eps_v = np.sort(rng.uniform(0.1, 3.0, v))
    eps = np.concatenate([eps_o, eps_v])
    nmo = o + v
    upper = np.triu(np.ones((nmo, nmo), dtype=bool))   # boolean order = row-major upper triangle
    ntri = nmo * (nmo + 1) // 2
    B = np.zeros((naux, nmo, nmo), dtype=np.float64)
    for q0 in range(0, naux, chunk):
        q1 = min(naux, q0 + chunk)
        vals = rng.standard_normal((q1 - q0, ntri)) * sigma_b
        for k in range(q1 - q0):
            m = B[q0 + k]
            m[upper] = vals[k]
            m += np.triu(m, 1).T      # mirror: the lower triangle still holds zeros
    if kappa != 0.0:
        g = np.ones(nmo)
        g[o:] = np.exp(-kappa * (eps_v - eps_v[0]))
        B *= g[None, :, None]
        B *= g[None, None, :]
    if t1_sigma > 0.0:
        t1 = rng.standard_normal((o, v)) * t1_sigma
    else:
        t1 = np.zeros((o, v))
    return System(o=o, v=v, naux=naux, eps=eps, B=B, t1=t1, seed=seed,
                  sigma_b=sigma_b, kappa=kappa)


# The five workloads.  "kappa" is the virtual-envelope decay of the pair densities.
# At o=40, v=400 the lowest CIS roots are single excitations out of the top few
# occupied orbitals (the couplings are ~1e-2 Eh against a 1.2 Eh spread of the
# occupied energies), so the state-averaged densities of pairs not touching those
# orbitals have rank ~8 whatever kappa is; the mean count at T_cut = 1e-7 is largest
# without an envelope (kappa = 0: 46 PNOs/pair, 8-9 for most pairs, up to v for the
# pairs of the excited orbitals; kappa = 0.5 / 1 / 2: 41 / 27 / 17).  The reduced PNO
# workload (o=10, v=100, kappa = 1) is small enough for the oracle to converge.


def _load_configs():
    """The workloads, one JSON file each under configs/: system sizes and generator knobs,
    the seed, the number of roots and space, the Davidson options (named as the fields of
    pnoeom_davidson_opts) and the PNO cut.  Returned flattened, keyed 1..5 and "pno_small"."""
    import json
    import os
    here = os.path.join(os.path.dirname(os.path.abspath(__file__)), "configs")
    out = {}
    for fn in sorted(os.listdir(here)):
        if not fn.endswith(".json"):
            continue
        with open(os.path.join(here, fn)) as fh:
            d = json.load(fh)
        key = int(d["name"]) if d["name"].isdigit() else d["name"]
        flat = dict(d["system"])
        flat.update(nroots=d["nroots"], space=d["space"], seed=d["seed"])
        flat.update(d.get("davidson", {}))
        if "pno" in d:
            flat["tcut"] = d["pno"]["tcut_pno"]
        out[key] = flat
    return out


CONFIGS = _load_configs()


def config_system(cfg, seed: int | None = None) -> System:
    c = CONFIGS[cfg]
    if seed is None:
        seed = c["seed"]
    return make_system(c["o"], c["v"], c["naux"], seed, kappa=c["kappa"],
                       t1_sigma=c["t1_sigma"])


def random_r(o: int, v: int, seed: int, nvec: int = 1):
    """Random trial amplitudes (R1, R2) with R2[i,j,a,b] = R2[j,i,b,a].

    Returns arrays of shape (nvec, o, v) and (nvec, o, o, v, v), float64.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    r1 = rng.standard_normal((nvec, o, v))
    x = rng.standard_normal((nvec, o, o, v, v))
    r2 = 0.5 * (x + x.transpose(0, 2, 1, 4, 3))
    return r1, r2


def random_blocks(v: int, nmat: int, seed: int):
    """nmat random v x v doubles blocks (one pair of one trial vector each), N(0, 1)
    entries with no symmetry imposed.  Returns an array of shape (nmat, v, v), float64."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.standard_normal((nmat, v, v))
