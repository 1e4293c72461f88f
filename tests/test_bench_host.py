"""bench.py's command-line contract on the host (no GPU work): more than one
GPU is refused with a message before anything touches a device."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2",
                        "--steps", "1", "--warmup", "0"], capture_output=True, text=True,
                       timeout=300, cwd=ROOT)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr)
    assert '"metric"' not in r.stdout


def test_unknown_variant_is_refused():
    """--only names variants; an unknown name stops the bench before any
    device work."""
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--only", "mixed,bogus"],
                       capture_output=True, text=True, timeout=300, cwd=ROOT)
    assert r.returncode != 0
    assert "unknown variants: ['bogus']" in r.stderr
    assert '"metric"' not in r.stdout
