"""Measurement programs, built on demand (never by the package build): the achievable peaks
of the device (peaks.hip: HBM copy/triad, atomics into tally-shaped arrays, FP64 FMA and
Philox+log rates) and a copy of known size that calibrates the HBM traffic counters
(copy_calibration.hip).  `python -m paper_2503_10263_amd.measure [peaks|copy BYTES]` builds into
a temporary directory and runs the program."""
import os
import shutil
import subprocess
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
FLAGS = ["--offload-arch=gfx950", "-O3", "-munsafe-fp-atomics",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def build(name: str, out_dir: str = "") -> str:
    """Compile measure/<name>.hip into out_dir (default: a new temporary directory)."""
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    out_dir = out_dir or tempfile.mkdtemp(prefix="karl_measure_")
    out = os.path.join(out_dir, name)
    subprocess.run([hipcc, *FLAGS, "-o", out, os.path.join(HERE, name + ".hip")], check=True,
                   capture_output=True)
    return out
