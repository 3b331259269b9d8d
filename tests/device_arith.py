"""Test support: builds and loads libkarl_device_arith.so, the kernels' elementary device
arithmetic applied element-wise to host arrays (device_arith.hip), once per kernel unit.

build() is called by __graft_entry__.build() beside the library and the oracle, so that the GPU
tests find it built; load() fails loudly if it is missing."""
import ctypes as C
import os
import subprocess
import sys
import tempfile
from concurrent.futures import ThreadPoolExecutor

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRC = os.path.join(HERE, "device_arith.hip")
LIB_PATH = os.path.join(HERE, "libkarl_device_arith.so")
# kernel unit -> (entry point, defines); the flags of each unit as the library builds it
UNITS = {
    "single": ("karl_test_arith_single", []),
    "drain": ("karl_test_arith_drain", ["-DKARL_DRAIN_UNIT=1"]),
    "batched": ("karl_test_arith_batched", ["-DKARL_BATCHED_UNIT=1"]),
}
UNIT_SOURCE = {"single": "karl_kernels.hip", "drain": "karl_kernels_drain.hip",
               "batched": "karl_kernels_batched.hip"}

DIV64, SQRT64, LOG64, SINCOS64, LOG32, SINCOS32, PHILOX, U53, MIX64 = range(9)
# bytes per element of (a, b, out0, out1), as device_arith.hip copies them
SIZES = {DIV64: (8, 8, 8, 8), SQRT64: (8, 0, 8, 8), LOG64: (8, 0, 8, 0), SINCOS64: (8, 0, 8, 8),
         LOG32: (4, 0, 4, 0), SINCOS32: (4, 0, 4, 4), PHILOX: (24, 0, 16, 0), U53: (8, 0, 8, 0),
         MIX64: (8, 0, 8, 0)}


def build() -> str:
    if ROOT not in sys.path:
        sys.path.insert(0, ROOT)
    from paper_2503_10263_amd import build as B
    own = dict(B.UNITS)
    inc = ["-I", os.path.join(ROOT, "include"), "-I", os.path.join(ROOT, "paper_2503_10263_amd", "csrc")]
    with tempfile.TemporaryDirectory(prefix="karl_arith_") as tmp:
        cmds = []
        for unit, (name, defs) in UNITS.items():
            obj = os.path.join(tmp, unit + ".o")
            cmds.append((obj, [B.hipcc()] + B.HIPCC_FLAGS + own[UNIT_SOURCE[unit]] + defs +
                         [f"-DKARL_TEST_NAME={name}"] + inc + ["-c", "-o", obj, SRC]))
        with ThreadPoolExecutor(max_workers=len(cmds)) as ex:
            list(ex.map(B._run, [c for _, c in cmds]))
        tmp_lib = LIB_PATH + ".tmp"
        B._run([B.hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp_lib] +
               [o for o, _ in cmds])
    os.replace(tmp_lib, LIB_PATH)
    return LIB_PATH


_lib = None


def load() -> C.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built: run python -c \"import __graft_entry__ as g; g.build()\"")
        L = C.CDLL(LIB_PATH)
        for name, _ in UNITS.values():
            f = getattr(L, name)
            f.argtypes = [C.c_int, C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]
            f.restype = C.c_int
        _lib = L
    return _lib


def apply(unit: str, op: int, a: np.ndarray, b: np.ndarray = None, out0_dtype=np.float64,
          out0_width: int = 1, out1: bool = False):
    """Runs `op` of `unit` over the elements of `a` (and `b`); returns out0 (and out1)."""
    f = getattr(load(), UNITS[unit][0])
    a = np.ascontiguousarray(a)
    n = a.shape[0]
    o0 = np.zeros((n, out0_width) if out0_width > 1 else n, dtype=out0_dtype)
    o1 = np.zeros(n, dtype=out0_dtype) if out1 else None
    bp = None
    if b is not None:
        b = np.ascontiguousarray(b)
        assert b.shape[0] == n
        bp = b.ctypes.data
    want = SIZES[op]
    got = (a.nbytes, b.nbytes if b is not None else 0, o0.nbytes, o1.nbytes if out1 else 0)
    assert got == tuple(w * n for w in want), f"op {op}: buffers of {got} bytes, need {want} per element"
    rc = f(op, n, a.ctypes.data, bp, o0.ctypes.data, o1.ctypes.data if out1 else None)
    if rc != 0:
        raise RuntimeError(f"{UNITS[unit][0]}(op {op}, n {n}) returned {rc}")
    return (o0, o1) if out1 else o0
