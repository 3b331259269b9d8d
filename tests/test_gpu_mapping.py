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


def _mixed_batch(n_long=1200):
    """Jobs of one batch: long flights (low column on fine grids: the wave mapping), short
    flights, a job without a field (always lane-mapped)."""
    ws = [W.cfg_tiny(n_primaries=n_long, column_cm2=1.0e16, bz=2.5, n_r=4, n_z=512, seed=2),
          W.cfg_tiny(n_primaries=900, column_cm2=1.0e17, bz=2.5, n_r=4, n_z=64, seed=3),
          W.cfg_tiny(n_primaries=700, column_cm2=1.0e16, bz=1.5, n_r=8, n_z=512, seed=4),
          W.cfg_tiny(n_primaries=500, seed=5)]
    ws[0].planes, ws[1].planes, ws[2].planes = [0, 100, 512], [0, 32, 64], [0, 256, 512]
    return ws


@pytest.mark.parametrize("mode", ["forced", "tuned"])
def test_batched_wave_flights_equal_oracle(mode):
    """Batched FP64 launches with wave-cooperative flights for the jobs on the wave mapping
    (forced at creation, or tuned from KARL_MAP_AUTO by the first of two transport calls):
    every job's digests and tallies equal the oracle's."""
    from paper_2503_10263_amd import karl
    ws = _mixed_batch()
    maps = ["wave", "lane", "wave", "lane"] if mode == "forced" else ["auto"] * 4
    jobs = [karl.Job(w, digests=True, queue_capacity=1 << 12, mapping=m) for w, m in zip(ws, maps)]
    batch = karl.Batch(max_jobs=8, queue_capacity=1 << 20)
    try:
        if mode == "forced":
            batch.transport(jobs, [(0, w.n_primaries) for w in ws])
        else:
            # the first call tunes each job's mapping, the second uses it
            batch.transport(jobs, [(0, w.n_primaries // 2) for w in ws])
            assert batch.wave_segments() == 0
            batch.transport(jobs, [(w.n_primaries // 2, w.n_primaries) for w in ws])
        chosen = [j.mapping()["mapping"] for j in jobs]
        got = [j.read_tallies() for j in jobs]
        wave_segs = batch.wave_segments()
    finally:
        for j in jobs:
            j.close()
        batch.close()
    assert chosen[0] == "wave" and chosen[2] == "wave" and chosen[3] == "lane", chosen
    assert wave_segs > 0
    for w, g in zip(ws, got):
        o = run_oracle(w, [(0, w.n_primaries)], digests=True)
        np.testing.assert_array_equal(g["digests"], o["digests"])
        compare_tallies(g, o, max(abs(o["ledger"][0]), 1.0))


def test_batched_wave_flights_fp32_equal_lane():
    from paper_2503_10263_amd import karl
    ws = _mixed_batch(3000)
    res = {}
    for m in ("wave", "lane"):
        jobs = [karl.Job(w, precision="fp32", digests=True, queue_capacity=1 << 12, mapping=m) for w in ws]
        batch = karl.Batch(max_jobs=8, queue_capacity=1 << 20)
        try:
            batch.transport(jobs, [(0, w.n_primaries) for w in ws])
            res[m] = ([j.read_tallies() for j in jobs], batch.wave_segments())
        finally:
            for j in jobs:
                j.close()
            batch.close()
    assert res["wave"][1] > 0 and res["lane"][1] == 0
    for gw, gl in zip(res["wave"][0], res["lane"][0]):
        np.testing.assert_array_equal(gw["digests"], gl["digests"])
        for k in ["counters", "recomb", "jz", "jr", "spectra"]:
            np.testing.assert_array_equal(gw[k], gl[k], err_msg=k)
