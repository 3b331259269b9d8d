"""bench.py's command line on the CPU: more than one GPU is refused with a message before any
device work, and the defaults are the launch configuration of the measured runs."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2", "--no-cpu"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_defaults_are_the_measured_launch_configuration():
    from paper_2503_10263_amd import workloads as W
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--help"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 0
    assert W.FULL_STEP_PRIMARIES == 131072 and W.FULL_SLICE_STEPS == 1 << 15
    assert W.BATCHED_QUEUE == 1 << 28
    assert (W.FULL_SLICE_STEPS & (W.FULL_SLICE_STEPS - 1)) == 0   # slices are a power of two
