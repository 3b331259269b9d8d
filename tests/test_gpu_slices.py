"""The deferred launch in slices (karl_job_desc.slice_steps): particles of the species that make
no products go round through a ring of whole particle states, so that a history may run on
several lanes one slice after another.  That changes which lane runs which part of a history
and nothing else.  Through the C ABI: FP64 parity with the oracle with slices on (digests,
integer tallies bit-exact, FP64 tallies to 1e-12), a ring so small that it wraps many times and
finds its slots still in use, and FP32 with and without slices (same digests and integer
tallies)."""
import numpy as np
import pytest

import oracle
from paper_2503_10263_amd import workloads as W
from parity_util import parity

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    import oracle
    oracle.build(force=False)


def _full(n=60, cap=3000):
    """Full-case geometry and physics with tracked H2+ (the deferred species), ion cap lowered
    so that the oracle finishes in seconds."""
    w = W.cfg_full(n_primaries=n)
    w.species[W.ION].cap = cap
    return w


def _run(w, **kw):
    from paper_2503_10263_amd import karl
    job = karl.Job(w, **kw)
    try:
        job.transport(0, w.n_primaries)
        return job.read_tallies(), job.slices()
    finally:
        job.close()


def test_full_case_in_slices_matches_oracle():
    w = _full()
    g, o, frac = parity(w, slice_steps=64)
    assert frac == 1.0
    assert o["counters"][oracle.C_BIRTH + 1] > 100        # ions born and tracked
    _, n = _run(w, slice_steps=64)
    assert n > 0, "no particle went round the ring"


def test_ring_smaller_than_the_launch_wraps():
    """A 16-entry ring for hundreds of ions in slices of 32 steps: it wraps many times, and
    particles whose slot still holds an unread entry stay on their lanes."""
    w = _full()
    g, o, frac = parity(w, slice_steps=32, slice_ring=16)
    assert frac == 1.0
    _, n = _run(w, slice_steps=32, slice_ring=16)
    assert n > 16 * 4, f"the ring took {n} entries, expected it to wrap"


def test_fp32_slices_change_nothing():
    w = _full(n=200, cap=5000)
    a, n0 = _run(w, precision="fp32", digests=True)
    b, n = _run(w, precision="fp32", digests=True, slice_steps=128)
    assert n0 == 0 and n > 0
    np.testing.assert_array_equal(a["digests"], b["digests"])
    for k in ("counters", "recomb", "jz", "jr", "spectra"):
        np.testing.assert_array_equal(a[k], b[k], err_msg=k)
    # the same FP32 contributions summed in FP64 in another order
    np.testing.assert_allclose(b["density_time"], a["density_time"], rtol=1e-9, atol=0.0)
    np.testing.assert_allclose(b["ledger"], a["ledger"], rtol=1e-9, atol=1e-9 * abs(a["ledger"][0]))
