"""Flight mappings of karl_transport: one particle per lane (lane mapping) or flights advanced
by the whole wave (wave mapping, guiding-centre mode), and the tuning that picks one.

The wave mapping gives segment k of a flight to lane k with its own draw (step ordinal s+k) and
accumulates time and path in step order, so it must reproduce the segment-by-segment event
sequence exactly: identical per-history digests and tallies to the oracle's bar."""
import numpy as np
import pytest

from paper_2503_10263_amd import workloads as W
from parity_util import compare_tallies, run_oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    import oracle
    oracle.build(force=False)


def _run(w, **kw):
    from paper_2503_10263_amd import karl
    job = karl.Job(w, **kw)
    try:
        job.transport(0, w.n_primaries)
        return job.read_tallies(), job.mapping()
    finally:
        job.close()


def _long_flights(n):
    """Low column on a fine grid: keV electrons cross hundreds of faces between interactions."""
    w = W.cfg_tiny(n_primaries=n, column_cm2=1.0e16, bz=2.5, n_r=4, n_z=256)
    w.planes = [0, 100, 256]
    return w


@pytest.mark.parametrize("case", ["long_flights", "full_capped"])
def test_wave_mapping_equals_oracle(case):
    if case == "long_flights":
        w = _long_flights(600)
    else:
        w = W.cfg_full(n_primaries=40)
        w.species[W.ION].cap = 2000
    g, m = _run(w, digests=True, history=True, mapping="wave")
    assert m["mapping"] == "wave" and m["wave_segments"] > 0
    o = run_oracle(w, [(0, w.n_primaries)], digests=True, hist=True)
    np.testing.assert_array_equal(g["digests"], o["digests"])
    compare_tallies(g, o, max(abs(o["ledger"][0]), 1.0))
    np.testing.assert_array_equal(g["hist"][:, 2:], o["hist"][:, 2:])


def test_wave_mapping_fp32_equals_lane_fp32():
    w = _long_flights(2000)
    gw, mw = _run(w, precision="fp32", digests=True, mapping="wave")
    gl, ml = _run(w, precision="fp32", digests=True, mapping="lane")
    assert mw["wave_segments"] > 0 and ml["wave_segments"] == 0
    np.testing.assert_array_equal(gw["digests"], gl["digests"])
    for k in ["counters", "recomb", "jz", "jr", "spectra"]:
        np.testing.assert_array_equal(gw[k], gl[k], err_msg=k)


@pytest.mark.parametrize("column,n_z,expect", [(1.0e16, 512, "wave"), (1.0e17, 64, "lane")])
def test_auto_mapping_is_tuned_and_result_independent(column, n_z, expect):
    """The first chunk (2000 primaries) runs lane-mapped; its segments per interaction pick the
    mapping of the rest (the wave mapping from 32 on).  The result equals a lane-mapped run."""
    w = W.cfg_tiny(n_primaries=8000, column_cm2=column, bz=2.5, n_r=4, n_z=n_z)
    ga, ma = _run(w, digests=True, mapping="auto", chunk=2000)
    gl, _ = _run(w, digests=True, mapping="lane")
    assert ma["mapping"] == expect
    assert (ma["segments_per_interaction"] >= 32.0) == (expect == "wave")
    assert ma["ms_per_segment_lane"] > 0
    assert (ma["wave_segments"] > 0) == (expect == "wave")
    np.testing.assert_array_equal(ga["digests"], gl["digests"])
    for k in ["counters", "recomb", "jz", "jr", "spectra"]:
        np.testing.assert_array_equal(ga[k], gl[k], err_msg=k)


def test_straight_line_jobs_use_the_lane_mapping():
    from paper_2503_10263_amd import karl
    w = W.cfg_tiny(n_primaries=100)
    job = karl.Job(w, mapping="wave")
    try:
        assert job.mapping()["mapping"] == "lane"
    finally:
        job.close()
