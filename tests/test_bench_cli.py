"""Command-line contract of bench.py checked on the host: more than one GPU
is refused with a message and exit status 2 before any device work."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU only" in (r.stdout + r.stderr)
    assert r.stdout.strip() == "" or not r.stdout.strip().startswith("{")


def test_kernel_hash_covers_the_step_kernel_sources():
    sys.path.insert(0, ROOT)
    import bench
    names = [os.path.basename(p) for p in bench.KERNEL_SRCS]
    assert names == ["kinetic.hip", "bgk_internal.h"]
    assert len(bench.kernel_hash()) == 16
