"""Serving: continuous batching of transport requests with admission by device memory.

Each served job must give the same result as the same job transported alone: integer tallies
exactly; the FP64 sums (cell times, energy ledger) up to the order of their additions, which
the atomics leave free.  Their addends are the same per-history values, so two orders differ by
at most n_add * 2^-53 of the sum of magnitudes; 1e-9 of the job's primary energy (ledger) or of
each cell's value (times) covers n_add up to 1e7."""
import numpy as np
import pytest

from paper_2503_10263_amd import workloads as W
from parity_util import compare_tallies, run_oracle

pytestmark = pytest.mark.gpu

INT_KEYS = ["counters", "recomb", "jz", "jr", "spectra"]
ORDER_RTOL = 1e-9


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    import oracle
    oracle.build(force=False)


def _requests(n, scale, rate=20.0, cap=None):
    reqs = W.serving_requests(n=n, rate=rate, scale=scale)
    if cap is not None:
        for _, w in reqs:
            w.n_primaries = min(w.n_primaries, cap)
    return reqs


def _alone(w, precision):
    from paper_2503_10263_amd import karl
    job = karl.Job(w, precision=precision, queue_capacity=1 << 16)
    try:
        job.transport(0, w.n_primaries)
        return job.read_tallies()
    finally:
        job.close()


def _same_up_to_order(got, ref):
    for k in INT_KEYS:
        np.testing.assert_array_equal(got[k], ref[k], err_msg=k)
    d_g, d_r = got["density_time"], ref["density_time"]
    assert np.all(np.abs(d_g - d_r) <= ORDER_RTOL * np.abs(d_r)), "density_time"
    scale = max(abs(ref["ledger"][0]), 1.0)
    assert np.all(np.abs(got["ledger"] - ref["ledger"]) <= ORDER_RTOL * scale), "ledger"


def _descriptor_bytes(w, precision):
    from paper_2503_10263_amd import karl
    p = karl.FP32 if precision == "fp32" else karl.FP64
    return karl.Descriptor(w, p, 0, 256, 0).workspace_bytes()


@pytest.mark.parametrize("threaded", [False, True])
def test_served_mix_equals_alone_fp32(threaded):
    """Eight jobs of the serving mix (grids 32x256 .. 64x512, columns 1e16-1e18, B 1-3.6 T)
    through a server whose arena holds only a few of them at a time, in short rounds (by the
    calling thread, or by two worker threads whose rounds run concurrently): each job's
    tallies equal its tallies transported alone."""
    from paper_2503_10263_amd import karl, serve
    reqs = _requests(8, scale=3e-4)
    sizes = sorted(_descriptor_bytes(w, "fp32") for _, w in reqs)
    arena = sizes[-1] + sizes[-2] + 4096
    srv = karl.Server(max_jobs=4, arena_bytes=arena, precision="fp32", queue_capacity=1 << 16,
                      round_ms=2.0, min_quantum=8, max_quantum=256)
    res = serve.replay(srv, reqs, realtime=False, keep_tallies=True, threaded=threaded)
    st = srv.stats()
    assert st["completed"] == 8 and st["released"] == 8
    assert st["arena_used"] == 0 and 0 < st["arena_peak"] <= arena
    assert st["rounds"] > 4
    assert st["primaries"] == sum(w.n_primaries for _, w in reqs)
    for (_, w), got in zip(reqs, res["tallies"]):
        _same_up_to_order(got, _alone(w, "fp32"))
    srv.close()


def test_served_fp64_matches_oracle():
    """FP64 server: per-history event digests and tallies of served jobs match the oracle."""
    from paper_2503_10263_amd import karl
    reqs = _requests(3, scale=1e-4, cap=120)
    srv = karl.Server(max_jobs=2, arena_bytes=1 << 30, precision="fp64", queue_capacity=1 << 16,
                      round_ms=1.0, min_quantum=16, max_quantum=64)
    tickets = [srv.submit(w, digests=True) for _, w in reqs]
    got = {}
    while len(got) < len(tickets):
        srv.step()
        for t in srv.poll():
            got[t] = srv.read_tallies(t, digests=True)
            srv.release(t)
    for t, (_, w) in zip(tickets, reqs):
        o = run_oracle(w, [(0, w.n_primaries)], digests=True)
        np.testing.assert_array_equal(got[t]["digests"], o["digests"])
        compare_tallies(got[t], o, max(abs(o["ledger"][0]), 1.0))
    srv.close()


def test_server_admission_rules():
    from paper_2503_10263_amd import karl
    reqs = _requests(3, scale=1e-4, cap=50)
    w0 = reqs[0][1]
    need = _descriptor_bytes(w0, "fp32")
    srv = karl.Server(max_jobs=2, arena_bytes=need, precision="fp32", queue_capacity=1 << 14,
                      round_ms=1.0, min_quantum=8, max_quantum=16)
    # a job larger than the whole arena can never run
    big = W.cfg_tiny(n_primaries=10, n_r=256, n_z=4096)
    with pytest.raises(karl.KarlError) as ei:
        srv.submit(big)
    assert ei.value.code == karl.EINVAL
    # another precision is refused
    s64 = karl.Descriptor(w0, karl.FP64, 0, 256, 0)
    import ctypes as C
    t = C.c_int64()
    assert karl.lib().karl_server_submit(srv.h, C.byref(s64.d), C.byref(t)) == karl.EINVAL
    # one job fits at a time: the second waits until the first is released
    ws = [W.with_primaries(w0, 40), W.with_primaries(w0, 40)]
    a, b = srv.submit(ws[0]), srv.submit(ws[1])
    with pytest.raises(karl.KarlError) as ei:
        srv.release(a)
    assert ei.value.code == karl.ESTATE
    n_act, n_pend = srv.step()
    assert n_pend == 1
    with pytest.raises(karl.KarlError) as ei:
        srv.read_tallies(b, only=("counters",))
    assert ei.value.code == karl.ESTATE
    while True:
        done = srv.poll()
        if done:
            break
        srv.step()
    assert done == [a]
    srv.release(a)
    while not srv.poll():
        srv.step()
    st = srv.stats()
    assert st["admitted"] == 2 and st["completed"] == 2
    srv.release(b)
    assert srv.stats()["arena_used"] == 0
    srv.close()


def test_realtime_replay_reports_latency():
    from paper_2503_10263_amd import karl, serve
    reqs = _requests(16, scale=2e-5, rate=80.0)
    srv = karl.Server(max_jobs=16, arena_bytes=2 << 30, precision="fp32", queue_capacity=1 << 18,
                      round_ms=5.0)
    res = serve.replay(srv, reqs, realtime=True)
    assert np.all(res["latency_s"] > 0)
    assert res["p99_s"] >= res["p50_s"] > 0
    assert res["collisions"].sum() > 0
    assert srv.stats()["completed"] == 16
    srv.close()


@pytest.mark.timeout(400)
def test_served_fp64_requests_at_their_drawn_sizes():
    """Five requests of the serving case at the sizes it draws (1.2e4-6.9e4 primaries, grids
    32x256-64x512, columns 1e16-4e17 cm^-2, B 1.1-2.9 T) through an FP64 server with the
    bench's round length: every history's event digest equal to the oracle's on sampled primary
    ids, and each job's identities (one electron per primary and per ionization, one ion per
    ionization, each particle deleted once, the energy budget)."""
    from concurrent.futures import ThreadPoolExecutor
    import oracle
    from paper_2503_10263_amd import karl
    from parity_util import assert_identities
    reqs = W.serving_requests(n=13)
    pick = [1, 2, 6, 9, 12]
    ws = [reqs[k][1] for k in pick]
    print("serving requests", pick, [w.n_primaries for w in ws], flush=True)
    srv = karl.Server(max_jobs=8, arena_bytes=4 << 30, precision="fp64", queue_capacity=1 << 22,
                      round_ms=200.0)
    tickets = [srv.submit(w, digests=True) for w in ws]
    got = {}
    while len(got) < len(tickets):
        srv.step()
        for t in srv.poll():
            got[t] = srv.read_tallies(t, digests=True)
            srv.release(t)
    srv.close()
    rng = np.random.default_rng(5)
    tasks = []
    for t, w in zip(tickets, ws):
        assert_identities(got[t]["counters"], got[t]["ledger"], w.n_primaries, w.processes, 1e-10)
        for pid in [0, w.n_primaries - 1] + [int(p) for p in rng.integers(1, w.n_primaries - 1, 4)]:
            tasks.append((t, w, pid))
    with ThreadPoolExecutor(max_workers=8) as ex:
        refs = list(ex.map(lambda a: oracle.run(a[1], a[2], a[2] + 1, digests=True)["digests"][a[2]], tasks))
    for (t, w, pid), d in zip(tasks, refs):
        assert got[t]["digests"][pid] == d, f"{w.name} primary {pid}: event sequence differs"


@pytest.mark.timeout(400)
def test_served_fp32_requests_at_their_drawn_sizes_equal_alone():
    """The same five serving-case requests at their drawn sizes in FP32 through the server
    configured as the bench runs it (four worker threads, 200 ms rounds): each job's integer
    tallies equal to its tallies transported alone, its FP64 sums up to their order."""
    from paper_2503_10263_amd import karl, serve
    reqs = W.serving_requests(n=13)
    sel = [reqs[k] for k in [1, 2, 6, 9, 12]]
    srv = karl.Server(max_jobs=8, arena_bytes=4 << 30, precision="fp32", queue_capacity=1 << 22,
                      round_ms=200.0, n_workers=4)
    res = serve.replay(srv, sel, realtime=False, keep_tallies=True, threaded=True)
    assert srv.stats()["completed"] == len(sel)
    srv.close()
    for (_, w), got in zip(sel, res["tallies"]):
        _same_up_to_order(got, _alone(w, "fp32"))
