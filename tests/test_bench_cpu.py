"""Host-side checks of the benchmark driver: the one-GPU contract and the
freshness of the recorded rocprofv3 counters (no GPU needed)."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    line = json.loads(r.stdout.strip().splitlines()[-1])
    assert line["n_gpus"] == 2 and "one GPU" in line["error"]


def test_profiles_were_taken_on_the_current_step_kernel():
    """bench.py reports HBM traffic only from counters taken on the current
    kernel source; the committed profiles must match it."""
    sys.path.insert(0, ROOT)
    import bench

    with open(os.path.join(ROOT, "profiles", "traffic.json")) as fh:
        data = json.load(fh)
    assert "film3_2d_1024:f32" in data
    for key, ent in data.items():
        assert ent["kernel_digest"] == bench.kernel_digest(), key
        assert 1.0 <= ent["hbm_bytes_per_launch"] / ent["algorithmic_bytes_per_launch"] < 2.0, key
    assert bench.profiled_launch("film3_2d_1024", "f32") is not None
    md = open(os.path.join(ROOT, "profiles", "step_kernel_film3_2d_1024_f32.md")).read()
    assert bench.kernel_digest() in md
