"""Build libkarl.so in-tree for gfx950 with hipcc."""
import os
import shutil
import subprocess

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
LIB = os.path.join(PKG, "libkarl.so")
SOURCES = [os.path.join(PKG, "csrc", f) for f in ("karl_kernels.hip", "karl_api.hip", "karl_server.hip")]

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    # every operation rounded once, as in the reference evaluation of the method
    "-ffp-contract=off",
    # hardware FP64 atomics for the density tallies
    "-munsafe-fp-atomics",
    # no packed FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def hipcc() -> str:
    return shutil.which("hipcc") or "/opt/rocm/bin/hipcc"


def build(verbose: bool = False, out: str = LIB, extra=()) -> str:
    tmp = out + ".tmp"
    cmd = [hipcc()] + HIPCC_FLAGS + list(extra) + ["-I", os.path.join(ROOT, "include"),
                                                   "-I", os.path.join(PKG, "csrc"), "-o", tmp] + SOURCES
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + res.stdout + res.stderr)
    if verbose:
        print(res.stderr)
    os.replace(tmp, out)
    return out


def build_calibration() -> str:
    """Copy kernel of known traffic used to scale the HBM counters (FETCH_SIZE, WRITE_SIZE)."""
    out = os.path.join(PKG, "copy_calibration")
    cmd = [hipcc(), "--offload-arch=gfx950", "-O3", "-Xclang", "-target-feature", "-Xclang",
           "-packed-fp32-ops", "-o", out, os.path.join(PKG, "csrc", "copy_calibration.hip")]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + res.stdout + res.stderr)
    return out


if __name__ == "__main__":
    print(build(verbose=True))
