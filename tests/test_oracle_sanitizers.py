"""The oracle under AddressSanitizer and UndefinedBehaviorSanitizer (with leak checking): its C
source and a small runner (oracle_sanitize_runner.c) built as one sanitized program, run on the
workloads of every feature -- straight lines and guiding centres, the full case with tracked
ions and energy-resolved densities, angle tables, density fields, ion chemistry, the Boris
mover -- with any report failing the run; and its tallies equal to the parity build's, bit for
bit (same source, every operation rounded once)."""
import ctypes as C
import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle
from paper_2503_10263_amd import workloads as W

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
RUNNER_SRC = os.path.join(HERE, "oracle_sanitize_runner.c")


@pytest.fixture(scope="module")
def runner(tmp_path_factory):
    if shutil.which("gcc") is None:
        pytest.skip("no gcc")
    out = str(tmp_path_factory.mktemp("oracle_san") / "oracle_san")
    cmd = ["gcc", "-std=c99", "-O1", "-g", "-fno-omit-frame-pointer", "-ffp-contract=off",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           "-I", os.path.join(ROOT, "oracle"), "-o", out, RUNNER_SRC,
           os.path.join(ROOT, "oracle", "karl_oracle.c"), "-lm"]
    subprocess.run(cmd, check=True)
    return out


def _arr(ptr, n, dtype=np.float64):
    if not ptr or n == 0:
        return np.zeros(0, dtype)
    return np.ctypeslib.as_array(ptr, shape=(n,)).astype(dtype, copy=True)


def write_descriptor(path, w, lo, hi, digests=True, hist=True):
    """The descriptor file that oracle_sanitize_runner.c reads (see its header)."""
    D = oracle.Desc(w)
    d = D.d
    ns = d.n_species or 2
    parts = [np.int64(C.sizeof(d)).tobytes(), C.string_at(C.addressof(d), C.sizeof(d))]

    def put(a, dtype=np.float64):
        a = np.ascontiguousarray(a, dtype=dtype)
        parts.append(np.int64(a.size).tobytes())
        parts.append(a.tobytes())

    put(_arr(d.n_gas, d.n_z))
    for s in range(4):
        put(_arr(d.n_field[s], d.n_r * d.n_z))
    for s in range(4):
        put(_arr(d.sp[s].edges, d.n_bins + 1 if s < ns else 0))
        put(_arr(d.sp[s].dens_edges, d.n_dens_bins + 1 if s < ns else 0))
    for i in range(16):
        p = d.proc[i]
        put(_arr(p.xs, d.n_e if i < d.n_proc else 0))
        put(_arr(p.ang_edges, p.ang_bins + 1 if p.ang_bins > 0 else 0))
        put(_arr(p.ang_theta, p.ang_nodes if p.ang_bins > 0 else 0))
        put(_arr(p.ang_pdf, p.ang_bins * p.ang_nodes))
    put(_arr(d.planes, d.n_planes, np.int32), np.int32)
    put(_arr(d.e_field, d.field_nr * d.field_nz * 3))
    put(_arr(d.b_field, d.field_nr * d.field_nz * 3))
    parts.append(np.array([lo, hi, int(digests), int(hist)], np.int64).tobytes())
    with open(path, "wb") as f:
        f.write(b"".join(parts))


def read_result(path, ref):
    """The runner's tallies, in the layout of the parity build's (ref)."""
    raw = open(path, "rb").read()
    out, off = {}, 0
    for k in ("counters", "ledger", "density_time", "recomb", "jz", "jr", "spectra", "digests",
              "hist", "density_time_e"):
        if k not in ref:
            continue
        n = ref[k].nbytes
        out[k] = np.frombuffer(raw[off:off + n], dtype=ref[k].dtype).reshape(ref[k].shape)
        off += n
    assert off == len(raw), (off, len(raw))
    return out


def _full_dense():
    w = W.cfg_full(n_primaries=12)
    w.species[W.ION].cap = 300
    w.dens_edges = (np.geomspace(1.0, 2.0e4, 17), np.geomspace(1e-4, 1e2, 17))
    return w


def _tiny_angles():
    w = W.cfg_tiny(n_primaries=600, column_cm2=1.0e17, bz=2.5, n_r=8, n_z=16)
    w.planes = [0, 8, 16]
    w.processes[0].angular = W.screened_table(e_iso=50.0)
    return w


CASES = {
    "tiny straight line": lambda: W.cfg_tiny(n_primaries=1500, column_cm2=1.0e17),
    "guiding centre with an angle table": _tiny_angles,
    "full case, ions, energy-resolved density": _full_dense,
    "paired beam on density fields": lambda: W.recombination_pair(3e-19, 1e-19, n_primaries=600),
    "hydrogen chemistry": lambda: W.hydrogen_chemistry(n_primaries=200),
    "charge exchange box": lambda: W.charge_exchange_box(n_primaries=300),
    "Boris mover": lambda: W.boris_column(n_primaries=60),
}


@pytest.mark.parametrize("name", list(CASES))
def test_oracle_clean_under_sanitizers(runner, tmp_path, name):
    w = CASES[name]()
    lo, hi = 0, w.n_primaries
    desc, res = str(tmp_path / "desc.bin"), str(tmp_path / "res.bin")
    write_descriptor(desc, w, lo, hi)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:halt_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    p = subprocess.run([runner, desc, res], env=env, capture_output=True, text=True, timeout=600)
    assert p.returncode == 0, f"{name}: exit {p.returncode}\n{p.stderr[-4000:]}"
    assert "runtime error" not in p.stderr and "Sanitizer" not in p.stderr, p.stderr[-4000:]
    ref = oracle.run(w, lo, hi, digests=True, hist=True)
    got = read_result(res, ref)
    for k, v in ref.items():
        np.testing.assert_array_equal(got[k].view(np.uint8), np.ascontiguousarray(v).view(np.uint8),
                                      err_msg=f"{name}: {k}")
    assert ref["counters"][oracle.C_BIRTH:oracle.C_BIRTH + 4].sum() > 0
