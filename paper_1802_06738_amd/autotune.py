"""Tile autotuner for the library's MFMA GEMM.

Every contraction of the sigma path, the PNO transforms and the Davidson goes through
one GEMM whose tile (128x128, 64x64, 32x128, 128x32) and K-split (automatic, none,
wider) are chosen per shape.  This tuner

  1. runs the workload (build_df + Davidson, canonical and SA-PNO, FP64 and FP32)
     with shape recording on, collecting every GEMM shape key the library launches;
  2. times each of the 12 variants on scratch operands of each recorded shape;
  3. writes the variants that beat the built-in rule by more than `margin` to a JSON
     table, which `load_table` installs (the binding loads the default table, if
     present, when the library is loaded).

Run on the GPU:
    python -m paper_1802_06738_amd.autotune --config 2 --out /tmp/gemm_gfx950.json

For a workload too large to solve while recording (config 4), `--sigma-blocks` records the
shapes of a few SA-PNO sigma blocks (BF16 and FP64) instead, times only the shapes below
`--max-flops`, and adds the entries to those of the table given by `--merge`.
"""
from __future__ import annotations

import argparse
import ctypes as C
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_TABLE = os.path.join(HERE, "tuning", "gemm_gfx950.json")
NVARIANT = 12
KINDS = ("128x128", "64x64", "32x128", "128x32")
SPLITS = ("auto", "none", "wide")


def default_variant(key):
    """The built-in rule of the library for a shape key."""
    m, n = key[4], key[5]
    if m >= 128 and n >= 128:
        kind = 0
    elif m <= 32 and n >= 128:
        kind = 2
    elif n <= 32 and m >= 128:
        kind = 3
    else:
        kind = 1
    return 3 * kind


def load_table(path=DEFAULT_TABLE, lib=None):
    """Install a tuning table; returns the number of entries."""
    from .pnoeom import load_library
    lib = lib or load_library()
    with open(path) as fh:
        tab = json.load(fh)
    ent = tab["entries"]
    keys = (C.c_longlong * (8 * max(len(ent), 1)))()
    var = (C.c_int * max(len(ent), 1))()
    for i, e in enumerate(ent):
        for j in range(8):
            keys[8 * i + j] = int(e["key"][j])
        var[i] = int(e["variant"])
    st = lib.pnoeom_gemm_set_table(len(ent), keys, var)
    if st != 0:
        raise RuntimeError(f"pnoeom_gemm_set_table failed ({st})")
    return len(ent)


def clear_table(lib=None):
    from .pnoeom import load_library
    lib = lib or load_library()
    lib.pnoeom_gemm_set_table(0, None, None)


def record_shapes(config, log=print):
    """Run the workload of a config with recording on; returns the recorded keys."""
    import torch
    sys.path.insert(0, os.path.dirname(HERE))
    from synthgen import config_system, CONFIGS
    from .pnoeom import load_library, PnoEom, FP64, FP32, CANONICAL, PNO
    lib = load_library()
    cfg = CONFIGS[config]
    s = config_system(config)
    dev = torch.device("cuda:0")
    B = torch.from_numpy(s.B).to(dev)
    eps = torch.from_numpy(s.eps).to(dev)
    t1 = torch.from_numpy(s.t1).to(dev)
    ctx = PnoEom(s.o, s.v, s.naux)
    lib.pnoeom_gemm_record(1)
    runs = [(FP64, CANONICAL), (FP32, CANONICAL), (FP64, PNO)]
    if cfg.get("space") == "pno":
        runs = [(FP64, PNO), (FP32, PNO)]
    free, total = torch.cuda.mem_get_info()
    log(f"[autotune] device memory free {free / 2**30:.1f} of {total / 2**30:.1f} GiB")
    for prec, space in runs:
        t0 = time.time()
        ctx.build_df(B, eps, t1, None, precision=prec)
        if space == PNO:
            ctx.build_sapno(cfg["nroots"], cfg.get("tcut", 1e-7))
        ctx.davidson(cfg["nroots"], space=space, precision=prec, tol_e=cfg["tol_e"], tol_r=cfg.get("tol_r", 1e-5),
                     max_sub=cfg.get("max_sub", 60), nextra=cfg.get("nextra", 0), refine_fp64=(prec != FP64))
        log(f"[autotune] recorded precision {prec} space {space} in {time.time() - t0:.1f} s")
    lib.pnoeom_gemm_record(0)
    n = lib.pnoeom_gemm_recorded(None, 0)
    buf = (C.c_longlong * (8 * max(n, 1)))()
    lib.pnoeom_gemm_recorded(buf, n)
    return [tuple(buf[8 * i + j] for j in range(8)) for i in range(n)]


def record_sigma_blocks(config, log=print):
    """Shapes of the SA-PNO sigma blocks of a config (one block per precision, BF16 and FP64)."""
    import torch
    sys.path.insert(0, os.path.dirname(HERE))
    from synthgen import config_system, CONFIGS
    from .pnoeom import load_library, PnoEom, FP64, BF16
    lib = load_library()
    cfg = CONFIGS[config]
    s = config_system(config)
    dev = torch.device("cuda:0")
    B = torch.from_numpy(s.B).to(dev)
    eps = torch.from_numpy(s.eps).to(dev)
    t1 = torch.from_numpy(s.t1).to(dev)
    ctx = PnoEom(s.o, s.v, s.naux)
    ctx.build_df(B, eps, t1, precision=BF16)
    ctx.build_sapno(cfg["nroots"], cfg.get("tcut_pno", cfg.get("tcut", 1e-7)))
    _, plen = ctx.pno_layout()
    gen = torch.Generator(device=dev)
    gen.manual_seed(1808)
    X = torch.randn((cfg["nroots"], plen), generator=gen, dtype=torch.float64, device=dev)
    lib.pnoeom_gemm_record(1)
    for prec in (BF16, FP64):
        t0 = time.time()
        ctx.sigma_pno(X, precision=prec)
        torch.cuda.synchronize()
        log(f"[autotune] recorded a sigma block in precision {prec} ({time.time() - t0:.1f} s)")
    lib.pnoeom_gemm_record(0)
    ctx.close()  # (the timing allocates its own operands)
    del X, B, eps, t1
    torch.cuda.empty_cache()
    n = lib.pnoeom_gemm_recorded(None, 0)
    buf = (C.c_longlong * (8 * max(n, 1)))()
    lib.pnoeom_gemm_recorded(buf, n)
    return [tuple(buf[8 * i + j] for j in range(8)) for i in range(n)]


def time_key(lib, key, variant, reps):
    k = (C.c_longlong * 8)(*key)
    ms = C.c_double()
    st = lib.pnoeom_gemm_time(None, k, variant, reps, C.byref(ms))
    if st != 0:
        raise RuntimeError(f"pnoeom_gemm_time failed ({st}) for {key} variant {variant}")
    return ms.value


def tune(config=2, margin=0.03, log=print, sigma_blocks=False, max_flops=None):
    from .pnoeom import load_library
    lib = load_library()
    clear_table(lib)
    keys = record_sigma_blocks(config, log) if sigma_blocks else record_shapes(config, log)
    log(f"[autotune] {len(keys)} GEMM shapes")
    entries = []
    t0 = time.time()
    for i, key in enumerate(keys):
        flops = 2.0 * key[4] * key[5] * key[6] * key[7]
        if max_flops is not None and flops > max_flops:
            continue
        reps = 2 if flops > 5e11 else 5
        dv = default_variant(key)
        t_def = time_key(lib, key, dv, reps)
        if t_def < 0:
            continue
        best, t_best = dv, t_def
        times = {}
        for v in range(NVARIANT):
            t = t_def if v == dv else time_key(lib, key, v, reps)
            times[v] = t
            if 0 <= t < t_best:
                best, t_best = v, t
        if best != dv and t_best < (1.0 - margin) * t_def:
            entries.append(dict(key=list(key), variant=best,
                                variant_name=f"{KINDS[best // 3]}/{SPLITS[best % 3]}",
                                default_ms=t_def, best_ms=t_best))
        if (i + 1) % 20 == 0:
            log(f"[autotune] {i + 1}/{len(keys)} shapes timed ({time.time() - t0:.0f} s), "
                f"{len(entries)} improved")
    work = f"config {config}" + (" sigma blocks" if sigma_blocks else "")
    return dict(device="gfx950", workload=work, margin=margin, shapes=len(keys), entries=entries)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--config", type=int, default=2)
    ap.add_argument("--margin", type=float, default=0.03)
    ap.add_argument("--out", default=DEFAULT_TABLE)
    ap.add_argument("--sigma-blocks", action="store_true")
    ap.add_argument("--max-flops", type=float, default=None)
    ap.add_argument("--merge", default=None, help="table whose entries (other shapes) are kept")
    args = ap.parse_args()
    tab = tune(args.config, args.margin, log=lambda m: print(m, file=sys.stderr, flush=True),
               sigma_blocks=args.sigma_blocks, max_flops=args.max_flops)
    if args.merge:
        with open(args.merge) as fh:
            old = json.load(fh)
        mine = {tuple(e["key"]) for e in tab["entries"]}
        tab["entries"] = [e for e in old["entries"] if tuple(e["key"]) not in mine] + tab["entries"]
        tab["workload"] = old["workload"] + ", " + tab["workload"]
        tab["shapes"] = old["shapes"] + tab["shapes"]
    os.makedirs(os.path.dirname(os.path.abspath(args.out)), exist_ok=True)
    with open(args.out, "w") as fh:
        json.dump(tab, fh, indent=1)
    gain = sum(e["default_ms"] - e["best_ms"] for e in tab["entries"])
    print(json.dumps(dict(shapes=tab["shapes"], improved=len(tab["entries"]), ms_saved_per_call_sum=gain)))


if __name__ == "__main__":
    main()
