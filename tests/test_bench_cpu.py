"""Host-side behaviour of bench.py (no GPU): more than one GPU is refused with a message before anything
touches a device, and a leg's private arrays stay out of the printed record."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr and r.stdout == ""


def test_private_arrays_are_dropped():
    sys.path.insert(0, ROOT)
    import bench
    rec = bench._public({"samples_per_s": 1.0, "_x": [1, 2, 3], "m_used": 4})
    assert rec == {"samples_per_s": 1.0, "m_used": 4}
