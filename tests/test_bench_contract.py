"""CPU checks of bench.py's contract that need no GPU: more than one GPU is refused with a
message, and the committed HBM counter summary parses into a traffic figure together with the
flag that says whether it belongs to the kernel source in the tree."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""


def test_counter_summary_parses():
    sys.path.insert(0, ROOT)
    import bench
    tbytes, valid = bench.counter_traffic()
    assert tbytes is not None and tbytes > 0
    assert isinstance(valid, bool)  # bench.py reports traffic only when this is True
