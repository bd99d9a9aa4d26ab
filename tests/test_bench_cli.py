"""bench.py's command line without a GPU: more than one GPU is refused with a
message before anything touches a device, and the kernel-source digest that
ties the committed byte-counter summary to the sources is stable."""

import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300, cwd=ROOT)
    assert r.returncode != 0
    assert "exactly one GPU" in (r.stdout + r.stderr)


def test_kernel_source_digest_is_stable():
    sys.path.insert(0, ROOT)
    import bench
    d1, d2 = bench.kernel_source_digest(), bench.kernel_source_digest()
    assert d1 == d2 and len(d1) == 16
    # a summary taken on other sources is not used
    assert bench.read_traffic("0" * 16) is None
