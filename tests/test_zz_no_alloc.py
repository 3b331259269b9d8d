"""karl_transport_noalloc (queues in the library's static device array, no allocation during
the call) against karl_transport on the same jobs: identical digests, integer tallies
bit-exact, FP64 tallies within 1e-12 relative.  Two calls in a row share the array, the second
with a smaller input; a dense column overflows the array's queues and exercises the undo of a
chunk."""
import numpy as np
import pytest

from paper_2503_10263_amd import karl
from paper_2503_10263_amd import workloads as W

pytestmark = pytest.mark.gpu

INT_KEYS = ["counters", "recomb", "jz", "jr", "spectra", "digests"]


def _same(a, b):
    for k in INT_KEYS:
        assert np.array_equal(a[k], b[k]), k
    for k in ["density_time", "ledger"]:
        d = np.abs(a[k] - b[k])
        assert np.all(d <= 1e-12 * np.maximum(np.abs(b[k]), 1e-300)), (k, float(d.max()))


def _pair(w, begin, end, **kw):
    ref = karl.Job(w, digests=True, device="cuda:0", **kw)
    ref.transport(begin, end)
    r = ref.read_tallies()
    ref.close()
    job = karl.Job(w, digests=True, device="cuda:0", **kw)
    job.transport_noalloc(begin, end)
    g = job.read_tallies()
    job.close()
    return g, r


def test_noalloc_equals_transport_two_calls_second_smaller():
    # guiding-centre grid, then a smaller straight-line job: the second call finds the first
    # call's queues and control words in the array
    w1 = W.cfg_tiny(n_primaries=30000, bz=2.5, column_cm2=3.0e17, n_r=8, n_z=16, seed=3)
    print("noalloc: call 1, tiny case in 2.5 T, 8x16 grid, column 3e17, 30000 primaries", flush=True)
    g, r = _pair(w1, 0, 30000)
    _same(g, r)
    assert int(g["counters"][karl.C_COLL]) > 0
    w2 = W.cfg_tiny(n_primaries=4000, seed=4, column_cm2=1.0e17)
    print("noalloc: call 2, tiny case straight lines, 4000 primaries", flush=True)
    g, r = _pair(w2, 0, 4000)
    _same(g, r)


def test_noalloc_full_case_ions():
    # the full case with tracked ions: the deferred launch runs whole histories from the
    # array's queues (the job's slices are not used)
    w = W.cfg_full(n_primaries=1000)
    w.species[W.ION].cap = 2000
    print("noalloc: full case, 400 primaries, ion cap 2000, slices of 2^10 steps in the reference", flush=True)
    g, r = _pair(w, 0, 400, slice_steps=1 << 10)
    _same(g, r)
    assert int(g["counters"][karl.C_COLL + 1]) > 0      # ion collisions ran


def test_noalloc_queue_overflow():
    # a dense column in a 2.5 T field (the electrons stay in the gas until they have lost
    # their energy) whose generations overflow the array's queues (about 2.2e5 entries) at the
    # first chunk: the chunk is undone and halved
    w = W.cfg_tiny(n_primaries=100000, column_cm2=1.0e18, bz=2.5, seed=5)
    print("noalloc: tiny case in 2.5 T, column 1e18, 100000 primaries", flush=True)
    ref = karl.Job(w, digests=True, device="cuda:0")
    ref.transport(0, 100000)
    r = ref.read_tallies()
    st = ref.stats()
    ref.close()
    print(f"noalloc: reference largest generation {st['max_queue']}", flush=True)
    job = karl.Job(w, digests=True, device="cuda:0")
    job.transport_noalloc(0, 100000)
    g = job.read_tallies()
    job.close()
    _same(g, r)
    # the reference's first chunk (65536 primaries) made a generation larger than the array's
    # queues hold, so the transport without allocation had to undo and halve its chunks
    assert st["max_queue"] > (64 << 20) // (4 * 76), st


def test_noalloc_rejects_tallies_beyond_the_array():
    # per-primary digests of 1e7 primaries (80 MB) do not fit in the 64 MiB array
    w = W.cfg_tiny(n_primaries=10_000_000)
    job = karl.Job(w, digests=True, queue_capacity=1024, device="cuda:0")
    with pytest.raises(karl.KarlError) as e:
        job.transport_noalloc(0, 10)
    assert e.value.code == karl.EINVAL
    job.close()
