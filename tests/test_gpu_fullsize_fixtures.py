"""Parity at the full sizes against stored oracle results (tests/golden/make_fullsize_fixtures.py
writes them on the CPU; only the oracle produced them).

Full case, primaries 0..999 at the real interaction cap of 1e6 (each ion history up to 1e6
collisions), transported in the launch configuration bench.py times: one karl_transport call
of the bench's step batch as one chunk, the deferred launch in slices of 2^15 steps.  Every
history's event digest, every integer tally bit-exact, FP64 tallies and per-history ledgers
within 1e-12 relative.

Batched case, the first 1000 primaries of each of its 256 jobs in FP64 through one batched
launch sequence (karl_transport_batch), and each job's share again with its own plain
launches: digests, counters and integer tallies (by SHA-256) exact per job, FP64 tallies and
ledgers within 1e-12 relative."""
import hashlib
import os

import numpy as np
import pytest

from paper_2503_10263_amd import workloads as W

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
FULL = os.path.join(HERE, "golden", "full_case_pids_0_1000.npz")
BATCHED = os.path.join(HERE, "golden", "batched_case_first_1000.npz")
INT_KEYS = ("recomb", "jz", "jr", "spectra")
RTOL = 1e-12


def _close(name, got, ref, scale=0.0):
    got, ref = np.asarray(got, np.float64), np.asarray(ref, np.float64)
    tol = np.maximum(RTOL * np.abs(ref), RTOL * scale)
    bad = np.abs(got - ref) > tol
    assert not bad.any(), f"{name}: {int(bad.sum())} elements beyond {RTOL:g} relative"


def _int_sha(t) -> str:
    h = hashlib.sha256()
    for k in INT_KEYS:
        h.update(np.ascontiguousarray(t[k], dtype=np.int64).tobytes())
    return h.hexdigest()


@pytest.mark.timeout(300)
def test_full_case_first_1000_primaries_at_the_real_cap():
    from paper_2503_10263_amd import karl
    import bench
    ref = np.load(FULL)
    n = int(ref["pid_end"])
    w = W.cfg_full(n_primaries=1_000_000)
    assert w.species[W.ION].cap == 1_000_000
    batch = bench.plan(bench.parse(["--gpus", "1", "--steps", "20", "--warmup", "5"]))["batch"]
    print(f"full case: primaries 0..{n - 1}, chunk {batch}, slices of {W.FULL_SLICE_STEPS} steps", flush=True)
    job = karl.Job(w, precision="fp64", digests=True, history=True, chunk=batch,
                   slice_steps=W.FULL_SLICE_STEPS)
    try:
        job.transport(0, n)
        g = job.read_tallies()
    finally:
        job.close()
    match = g["digests"][:n] == ref["digests"]
    assert match.all(), f"{int((~match).sum())} of {n} histories differ, first {np.nonzero(~match)[0][:5]}"
    np.testing.assert_array_equal(g["counters"], ref["counters"])
    assert int(g["counters"][karl.C_DEATH + karl.NREASON + W.REASONS.index("cap")]) > 0   # capped ions
    for k in INT_KEYS:
        np.testing.assert_array_equal(g[k], ref[k], err_msg=k)
    _close("density_time", g["density_time"], ref["density_time"])
    _close("ledger", g["ledger"], ref["ledger"], scale=abs(float(ref["ledger"][0])))
    np.testing.assert_array_equal(g["hist"][:n, 2:], ref["hist"][:, 2:])
    _close("hist", g["hist"][:n, :2], ref["hist"][:, :2], scale=1e-3)


def _check_job(j, t, ref):
    n = int(ref["pid_end"][j])
    match = t["digests"][:n] == ref["digests"][j, :n]
    assert match.all(), f"job {j}: {int((~match).sum())} of {n} histories differ"
    np.testing.assert_array_equal(t["counters"], ref["counters"][j], err_msg=f"job {j}")
    assert _int_sha(t) == str(ref["int_sha"][j]), f"job {j}: integer tallies differ"
    _close(f"job {j} density_time", t["density_time"], ref["density_time"][j])
    _close(f"job {j} ledger", t["ledger"], ref["ledger"][j], scale=abs(float(ref["ledger"][j][0])))


@pytest.mark.timeout(300)
def test_batched_case_first_1000_primaries_of_every_job_fp64():
    from paper_2503_10263_amd import karl
    ref = np.load(BATCHED)
    ws = W.cfg_batched(n_jobs=256)
    ends = [int(e) for e in ref["pid_end"]]
    print("batched case: 256 jobs, first 1000 primaries each, FP64 batched launches", flush=True)
    jobs = [karl.Job(w, precision="fp64", digests=True, queue_capacity=1024) for w in ws]
    batch = karl.Batch(max_jobs=len(ws), queue_capacity=1 << 24)
    try:
        batch.transport(jobs, [(0, e) for e in ends])
        got = [j.read_tallies() for j in jobs]
    finally:
        for j in jobs:
            j.close()
        batch.close()
    for j, t in enumerate(got):
        _check_job(j, t, ref)
    print("batched case: every job again with its own plain launches", flush=True)
    for j, w in enumerate(ws):
        job = karl.Job(w, precision="fp64", digests=True, queue_capacity=1 << 20)
        try:
            job.transport(0, ends[j])
            _check_job(j, job.read_tallies(), ref)
        finally:
            job.close()
