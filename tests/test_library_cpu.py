"""CPU checks of the C-ABI library: it loads, exports every entry point that include/karl.h
declares, sizes workspaces and rejects invalid descriptors before touching a device."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_2503_10263_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def karl():
    from paper_2503_10263_amd import karl as K
    if not os.path.exists(K.LIB_PATH):
        from paper_2503_10263_amd import build
        build.build()
    return K


def declared_entry_points():
    text = open(os.path.join(ROOT, "include", "karl.h")).read()
    return sorted(set(re.findall(r"^\s*(?:karl_status|const char\*)\s+(karl_\w+)\s*\(", text, re.M)))


def test_library_exports_every_declared_symbol(karl):
    names = declared_entry_points()
    assert len(names) >= 8
    lib = karl.lib()
    for n in names:
        assert hasattr(lib, n), n
    assert sorted(karl.ENTRY_POINTS) == names


def test_workspace_bytes(karl):
    w = W.cfg_full(n_primaries=1000)
    d = karl.Descriptor(w, queue_capacity=1 << 20)
    n = d.workspace_bytes()
    # four queues of 76-byte entries (two generation buffers, two deferred buffers) dominate
    assert 4 * (1 << 20) * 72 < n < 4 * (1 << 20) * 72 + 32 * 2**20
    d32 = karl.Descriptor(w, precision=karl.FP32, queue_capacity=1 << 20)
    assert d32.workspace_bytes() < n
    dd = karl.Descriptor(w, flags=karl.FLAG_DIGESTS | karl.FLAG_HISTORY, queue_capacity=1 << 20)
    # tallies and their snapshot, each region aligned to 256 bytes
    assert dd.workspace_bytes() >= n + 2 * 1000 * (8 + 32) - 2 * 256


def test_slice_ring_in_the_workspace(karl):
    """Slices of the deferred launch add a ring of 160-byte particle states and an 8-byte flag
    per entry -- by default queue_capacity + 2^20 entries -- and nothing without slices."""
    w = W.cfg_full(n_primaries=1000)
    n = karl.Descriptor(w, queue_capacity=1 << 20).workspace_bytes()
    ring = (1 << 20) + (1 << 20)
    assert karl.Descriptor(w, queue_capacity=1 << 20, slice_ring=999).workspace_bytes() == n
    ns = karl.Descriptor(w, queue_capacity=1 << 20, slice_steps=1 << 15).workspace_bytes()
    assert n + ring * 168 <= ns <= n + ring * 168 + 2 * 256
    nr = karl.Descriptor(w, queue_capacity=1 << 20, slice_steps=64, slice_ring=1000).workspace_bytes()
    assert n + 1000 * 168 <= nr <= n + 1000 * 168 + 2 * 256


@pytest.mark.parametrize("steps,ring", [(3, 0), (-64, 0), (1 << 31, 0), (96, 0), (64, -1)])
def test_bad_slices_are_rejected(karl, steps, ring):
    w = W.cfg_tiny(n_primaries=10)
    d = karl.Descriptor(w, queue_capacity=1024, slice_steps=steps, slice_ring=ring)
    n = C.c_uint64()
    assert karl.lib().karl_workspace_bytes(C.byref(d.d), C.byref(n)) == karl.EINVAL
    assert "slice" in karl.lib().karl_last_error().decode()


def _create(karl, desc):
    h = C.c_void_p()
    return karl.lib().karl_create_job(C.byref(desc.d), C.byref(h))


@pytest.mark.parametrize("mutate,code", [
    (lambda d: setattr(d.d, "n_r", 0), -1),
    (lambda d: setattr(d.d, "radius", -1.0), -1),
    (lambda d: setattr(d.d, "n_e", 1), -1),
    (lambda d: setattr(d.d, "n_e", 1025), -1),
    (lambda d: setattr(d.d.proc[0], "kind", 9), -1),
    (lambda d: setattr(d.d, "precision", 7), -1),
    (lambda d: setattr(d.d, "n_primaries", -5), -1),
    (lambda d: setattr(d.d, "workspace", None), -1),
])
def test_create_rejects_invalid(karl, mutate, code):
    w = W.cfg_tiny(n_primaries=10)
    d = karl.Descriptor(w, queue_capacity=1024)
    d.d.workspace = 1 << 40
    d.d.workspace_bytes = d.workspace_bytes()
    mutate(d)
    assert _create(karl, d) == code
    assert len(karl.lib().karl_last_error()) > 0


def test_create_rejects_small_workspace(karl):
    w = W.cfg_tiny(n_primaries=10)
    d = karl.Descriptor(w, queue_capacity=1024)
    d.d.workspace = 1 << 40
    d.d.workspace_bytes = d.workspace_bytes() - 1
    assert _create(karl, d) == karl.ENOMEM


def test_bad_plane_and_nonfinite_density(karl):
    w = W.cfg_tiny(n_primaries=10)
    w.planes = [0, 5]
    d = karl.Descriptor(w, queue_capacity=1024)
    n = C.c_uint64()
    assert karl.lib().karl_workspace_bytes(C.byref(d.d), C.byref(n)) == karl.EINVAL
    w = W.cfg_tiny(n_primaries=10)
    w.n_gas = np.array([np.nan])
    d = karl.Descriptor(w, queue_capacity=1024)
    assert karl.lib().karl_workspace_bytes(C.byref(d.d), C.byref(n)) == karl.EINVAL


def test_null_job_is_an_error_not_a_crash(karl):
    lib = karl.lib()
    assert lib.karl_transport(None, 0, 1, None) == karl.ESTATE
    assert lib.karl_transport_noalloc(None, 0, 1, None) == karl.ESTATE
    assert lib.karl_destroy_job(None) == karl.EINVAL
    n = C.c_int64(-1)
    assert lib.karl_job_slices(None, C.byref(n)) == karl.EINVAL and n.value == -1
    assert lib.karl_batch_wave_segments(None, C.byref(n)) == karl.EINVAL and n.value == -1


def test_invalid_angle_tables_are_rejected(karl):
    w = W.cfg_tiny(n_primaries=10)
    w.processes[0].angular = W.screened_table()
    w.processes[0].angular.pdf[2][:] = 0.0                # a bin without area
    with pytest.raises(karl.KarlError) as ei:
        karl.Descriptor(w, queue_capacity=1024).workspace_bytes()
    assert ei.value.code == karl.EINVAL
    w = W.cfg_tiny(n_primaries=10)
    w.processes[2].angular = W.screened_table()           # the excitation process
    with pytest.raises(karl.KarlError) as ei:
        karl.Descriptor(w, queue_capacity=1024).workspace_bytes()
    assert ei.value.code == karl.EINVAL


def test_chemistry_descriptor_rules():
    """Invalid chemistry descriptors are rejected before any device work."""
    from paper_2503_10263_amd import karl
    import copy

    def rejected(w):
        with pytest.raises(karl.KarlError) as ei:
            karl.Descriptor(w, queue_capacity=1024).workspace_bytes()
        return ei.value.code == karl.EINVAL

    base = W.hydrogen_chemistry(n_primaries=10)
    assert karl.Descriptor(base, queue_capacity=1024).workspace_bytes() > 0
    w = copy.deepcopy(base)
    w.processes[1].product = 0                      # ionization making an electron slot
    assert rejected(w)
    w = copy.deepcopy(base)
    w.processes[7].product = 1                      # clustering into its own species
    assert rejected(w)
    w = copy.deepcopy(base)
    w.processes[4].partner = 4                      # no species slot 4
    assert rejected(w)
    w = copy.deepcopy(base)
    w.processes.append(W.Process(W.RECOMBINATION, W.ELECTRON, W.TARGET_FIELD, 0.0,
                                 np.full(w.n_e, 1e-20), "second partner", partner=1))
    assert rejected(w)                              # electron field processes must share a partner
    w = copy.deepcopy(base)
    w.processes[4].density_power = 2                # three-body rate on a field target
    assert rejected(w)
    w = copy.deepcopy(base)
    w.beam_species = 4
    w.source = W.SOURCE_BEAM
    assert rejected(w)


def test_boris_descriptor_rules():
    """Invalid mover descriptors are rejected before any device work."""
    from paper_2503_10263_amd import karl
    import math as _m

    def rejected(w):
        with pytest.raises(karl.KarlError) as ei:
            karl.Descriptor(w, queue_capacity=1024).workspace_bytes()
        return ei.value.code == karl.EINVAL

    assert karl.Descriptor(W.boris_column(n_primaries=10), queue_capacity=1024).workspace_bytes() > 0
    w = W.boris_column(n_primaries=10)
    w.mover = W.MOVER_DRIFT                          # field arrays with the drift mover
    assert rejected(w)
    w = W.boris_column(n_primaries=10)
    w.species[0].lifetime = _m.inf                  # a Boris particle must end
    assert rejected(w)
    w = W.boris_column(n_primaries=10)
    w.boris_dt = [1e-16, 1e-7]                      # 2e10 pushes per lifetime
    assert rejected(w)
    w = W.boris_column(n_primaries=10)
    w.boris_dt = [2e-11, 0.0]
    assert rejected(w)
    w = W.boris_column(n_primaries=10)
    w.e_field = np.full_like(w.e_field, np.nan)
    assert rejected(w)


def test_device_arith_helper_loads_and_rejects_bad_calls():
    """The GPU tests' helper of the kernels' elementary arithmetic is built beside the library,
    exports one entry point per kernel unit, and rejects an unknown operation or a negative
    count (and does nothing for none) before any device work."""
    import device_arith as D
    if not os.path.exists(D.LIB_PATH):
        D.build()
    L = D.load()
    for unit, (name, _) in D.UNITS.items():
        f = getattr(L, name)
        assert f(99, 1, None, None, None, None) == -1, unit
        assert f(D.DIV64, -1, None, None, None, None) == -1, unit
        assert f(D.DIV64, 0, None, None, None, None) == 0, unit
    with pytest.raises(AssertionError):
        D.apply("drain", D.LOG64, np.zeros(4, np.float32))     # FP32 buffer for an FP64 operation


def test_tables_beyond_lds_and_fp32_range_are_rejected_before_device_work(karl):
    """Sizing already rejects a job whose tables and grid faces overflow the 64 KiB of LDS a
    workgroup stages them in, and an FP32 job whose tables or geometry leave the FP32 range (its
    kernels would read infinities); the same values in FP64 are accepted."""
    import re as _re

    def code_and_message(w, precision):
        try:
            prec = {"fp64": karl.FP64, "fp32": karl.FP32}[precision]
            karl.Descriptor(w, precision=prec, queue_capacity=1024).workspace_bytes()
        except karl.KarlError as e:
            return e.code, str(e)
        return karl.OK, ""

    code, msg = code_and_message(W.cfg_full(n_primaries=10, n_e=1024), "fp64")
    assert code == karl.EINVAL and _re.search(r"tables need \d+ bytes of LDS", msg), msg
    assert code_and_message(W.cfg_full(n_primaries=10, n_e=1024), "fp32")[0] == karl.OK   # half the bytes
    assert code_and_message(W.cfg_full(n_primaries=10, n_e=512), "fp64")[0] == karl.OK
    dense = W.cfg_tiny(n_primaries=10, n_z=4)
    dense.n_gas = np.full(4, 1e38)                   # the birth CDF sums to 4e38
    assert code_and_message(dense, "fp32")[0] == karl.EINVAL
    assert code_and_message(dense, "fp64")[0] == karl.OK
    big = W.cfg_tiny(n_primaries=10)
    big.processes[0].xs = big.processes[0].xs * 1e60
    assert code_and_message(big, "fp32")[0] == karl.EINVAL
    assert code_and_message(big, "fp64")[0] == karl.OK
