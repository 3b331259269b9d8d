"""Parity at the full sizes, in the launch configuration that bench.py times.

Full case (1e6-primary job, 64x512 grid, tracked H2+ capped at 1e6 interactions): the
benchmark's step of 131072 primary ids in one karl_transport call, as one chunk, its deferred
launch in slices of 2^15 steps.  The oracle computes
sampled histories one by one: their event digests and per-history energy ledgers must be
identical.  Over the whole batch, properties that hold at any size: every particle deleted
exactly once, one electron and one ion per ionization, the energy budget.  Again for the
bench's last timed step at --steps 20 --warmup 5 (primary ids 960000..999999).

Batched case (256 jobs, FP32) at full size in one karl_transport_batch: the same integer
identities per job, the energy budget per job within the FP32 bound, and sampled jobs equal
to themselves transported alone."""
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

from paper_2503_10263_amd import workloads as W
from parity_util import assert_identities as _identities

pytestmark = pytest.mark.gpu

BENCH_BATCH = W.FULL_STEP_PRIMARIES
SAMPLED = [0, 7919, 31337, 104729, BENCH_BATCH - 1]


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    import oracle
    oracle.build(force=False)


@pytest.mark.timeout(600)
def test_full_case_bench_batch_sampled_histories():
    import oracle
    from paper_2503_10263_amd import karl
    w = W.cfg_full(n_primaries=1_000_000)
    job = karl.Job(w, precision="fp64", digests=True, history=True, chunk=BENCH_BATCH,
                   slice_steps=W.FULL_SLICE_STEPS)
    try:
        job.transport(0, BENCH_BATCH)
        g = job.read_tallies()
        assert job.slices() > 0          # the deferred launch ran in slices
    finally:
        job.close()
    _identities(g["counters"], g["ledger"], BENCH_BATCH, w.processes, 1e-10)
    assert g["counters"][karl.C_DEATH + karl.NREASON + W.REASONS.index("cap")] > 0   # cap-bound ions
    assert np.all(g["digests"][BENCH_BATCH:] == 0)

    def one(pid):
        return oracle.run(w, pid, pid + 1, digests=True, hist=True)

    with ThreadPoolExecutor(max_workers=len(SAMPLED)) as ex:
        refs = list(ex.map(one, SAMPLED))
    for pid, o in zip(SAMPLED, refs):
        assert g["digests"][pid] == o["digests"][pid], f"primary {pid}: event sequence differs"
        h_g, h_o = g["hist"][pid], o["hist"][pid]
        np.testing.assert_array_equal(h_g[2:], h_o[2:])               # particles born / deleted
        assert np.all(np.abs(h_g[:2] - h_o[:2]) <= 1e-12 * abs(h_o[0])), f"primary {pid}: ledger"


@pytest.mark.timeout(600)
def test_full_case_last_bench_step_sampled_histories():
    """The last timed step of bench.py --steps 20 --warmup 5 (primary ids up to 999999, the
    keys' high bits), one karl_transport call as the bench makes it: sampled histories equal to
    the oracle's, and the identities over the step."""
    import bench
    import oracle
    from paper_2503_10263_amd import karl
    pl = bench.plan(bench.parse(["--gpus", "1", "--steps", "20", "--warmup", "5"]))
    batch = pl["batch"]
    lo = (pl["warmup"] + pl["steps"] - 1) * batch
    hi = lo + batch
    assert hi <= 1_000_000
    w = W.cfg_full(n_primaries=1_000_000)
    print(f"full case: primaries {lo}..{hi - 1} in one call, slices of {pl['slice_steps']} steps", flush=True)
    job = karl.Job(w, precision="fp64", digests=True, history=True, chunk=batch,
                   slice_steps=pl["slice_steps"])
    try:
        job.transport(lo, hi)
        g = job.read_tallies()
    finally:
        job.close()
    _identities(g["counters"], g["ledger"], batch, w.processes, 1e-10)
    assert np.all(g["digests"][:lo] == 0)
    sampled = [lo, lo + 1, lo + 12345, 999983, hi - 1]

    def one(pid):
        return oracle.run(w, pid, pid + 1, digests=True, hist=True)

    with ThreadPoolExecutor(max_workers=len(sampled)) as ex:
        refs = list(ex.map(one, sampled))
    for pid, o in zip(sampled, refs):
        assert g["digests"][pid] == o["digests"][pid], f"primary {pid}: event sequence differs"
        np.testing.assert_array_equal(g["hist"][pid][2:], o["hist"][pid][2:])
        assert np.all(np.abs(g["hist"][pid][:2] - o["hist"][pid][:2]) <= 1e-12 * abs(o["hist"][pid][0])), \
            f"primary {pid}: ledger"


def test_batched_case_full_size_fp32():
    from paper_2503_10263_amd import karl
    ws = W.cfg_batched(n_jobs=256)
    jobs = [karl.Job(w, precision="fp32", queue_capacity=1024) for w in ws]
    batch = karl.Batch(max_jobs=256, queue_capacity=W.BATCHED_QUEUE)
    try:
        batch.transport(jobs, [(0, w.n_primaries) for w in ws])
        tallies = [j.read_tallies() for j in jobs]
    finally:
        for j in jobs:
            j.close()
        batch.close()
    for w, t in zip(ws, tallies):
        # per-history energies are FP32; each of up to ~1e5 interactions rounds at 2^-24
        _identities(t["counters"], t["ledger"], w.n_primaries, w.processes, 1e-3)
    # the two smallest jobs and one of median size, each transported alone
    order = np.argsort([w.n_primaries for w in ws])
    for k in [order[0], order[1], order[len(order) // 2]]:
        w = ws[k]
        alone = karl.Job(w, precision="fp32", queue_capacity=1 << 16)
        try:
            alone.transport(0, w.n_primaries)
            a = alone.read_tallies()
        finally:
            alone.close()
        for key in ["counters", "recomb", "jz", "jr", "spectra"]:
            np.testing.assert_array_equal(tallies[k][key], a[key], err_msg=f"job {k}: {key}")
