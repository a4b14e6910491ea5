"""bench.py without a GPU: the multi-GPU request is refused with a message
before any device use, and the host oracle baseline worker of the chain
batch prints one JSON rate (it never touches the GPU)."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
BENCH = os.path.join(ROOT, "bench.py")


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, BENCH, "--gpus", "2"], capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_cpu_baseline_worker_prints_a_rate():
    spec = dict(replica=0, n_cells=0, trials=2, site_trials=0, ion_trials=1, seconds=0.5, pairing=True)
    from workloads import cells_per_dim, config3
    c = config3()[0]
    spec["n_cells"] = cells_per_dim(c["L"], c["rc"])
    r = subprocess.run([sys.executable, BENCH, "--cpu-worker", json.dumps(spec)], capture_output=True, text=True,
                       timeout=300, cwd=ROOT)
    assert r.returncode == 0, r.stderr
    out = json.loads(r.stdout.strip().splitlines()[-1])
    assert out["unit"] == "trial moves/s" and out["value"] > 0 and out["cores"] == 1
    assert out["replica"] == 0 and out["sites"] == len(c["kind"])
