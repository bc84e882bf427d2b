"""Host-side logic of bench.py (CPU only): the one-GPU refusal and the rules that decide
when counter-measured HBM traffic may be reported."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in msg["error"]


def test_traffic_reported_only_for_the_measured_kernel_and_workload():
    import bench
    assert bench.kernel_traffic("ring", 2, False) is None or bench.kernel_traffic("ring", 2, False) > 1e9
    assert bench.kernel_traffic("ring", 3, False) is None        # other workload
    assert bench.kernel_traffic("ring", 2, True) is None         # PNO space
    assert bench.kernel_traffic("nonexistent", 2, False) is None
    saved = dict(bench.KERNEL_TRAFFIC["ring"])
    try:
        bench.KERNEL_TRAFFIC["ring"]["gemm_sha256"] = "0" * 64     # kernel changed since the counters
        assert bench.kernel_traffic("ring", 2, False) is None
    finally:
        bench.KERNEL_TRAFFIC["ring"] = saved
    # the hashed region exists and is the dense GEMM kernel with its launch
    assert len(bench.gemm_kernel_sha()) == 64


def test_metric_name():
    import bench
    assert bench.METRIC.startswith("σ evals/s & Davidson time")


def test_workload_json_mirrors_the_options_struct():
    """Each workload file names its Davidson options as the fields of pnoeom_davidson_opts
    (mirrored by the binding's ctypes structure) and gives the generator's knobs."""
    import json
    import os
    from paper_1802_06738_amd.pnoeom import DavidsonOpts
    from synthgen import CONFIGS
    fields = {f[0] for f in DavidsonOpts._fields_}
    here = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "synthgen", "configs")
    names = sorted(f for f in os.listdir(here) if f.endswith(".json"))
    assert len(names) == len(CONFIGS) == 6
    for fn in names:
        with open(os.path.join(here, fn)) as fh:
            d = json.load(fh)
        assert set(d["davidson"]) <= fields, (fn, set(d["davidson"]) - fields)
        assert set(d["system"]) == {"o", "v", "naux", "t1_sigma", "kappa"}
        assert d["space"] in ("canonical", "pno") and d["nroots"] >= 1 and isinstance(d["seed"], int)
        assert ("pno" in d) == (d["space"] == "pno" or fn == "pno_small.json")
