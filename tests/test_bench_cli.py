"""bench.py on the CPU: the one-GPU contract (more GPUs are refused with a message, before
anything touches a device) and the committed headline counters matching the kernel source."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr
    assert r.stdout == ""


def test_headline_counter_profile_matches_kernel_source():
    """The bench line's `traffic` comes from the committed counter summary of the headline
    kernel only while that summary was taken on the current kernel source; a kernel change
    without new counters turns it into null. This keeps the two in step."""
    sys.path.insert(0, ROOT)
    import bench
    kv = {}
    for line in open(bench.PROFILE_COUNTERS):
        if "=" in line and not line.startswith("#"):
            k, v = line.split("=", 1)
            kv[k.strip()] = v.strip()
    assert kv["kernel_source_sha256_16"] == bench.source_digest(bench.KERNEL_SOURCES)
    assert int(kv["nodes"]) == 2048 * 2048
    assert bench.counter_traffic(2048 * 2048) == float(kv["hbm_bytes_per_launch"])
