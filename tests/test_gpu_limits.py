"""Table sizes at the limits a job accepts.  A job's cross-section tables, gas densities and
face positions are staged in LDS, at most 64 KiB per workgroup (the library's limit; the
device allows more), and a table has at most 1024 nodes.

* FP64 full case (nine processes, 64x512 grid, tracked H2+ in the deferred launch, whose kernel
  adds its own LDS copy of the series constants) with tables at the largest node count that
  fits the LDS limit: parity with the oracle.  One node more is rejected with KARL_EINVAL, the
  message naming the bytes it needs, before any device work; the jobs made after it run.
* FP32 full case at the node limit of 1024 (its tables take half the bytes): the identities of
  a transport."""
import re

import pytest

import oracle
from paper_2503_10263_amd import workloads as W
from parity_util import assert_identities, parity

pytestmark = pytest.mark.gpu

LDS_LIMIT = 65536


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    oracle.build(force=False)


def _full(n_e, n_primaries=40):
    w = W.cfg_full(n_primaries=n_primaries, n_e=n_e)
    w.species[W.ION].cap = 3000          # the oracle finishes in seconds
    return w


def _lds_need(w, precision):
    """The LDS bytes the library names when it rejects w's tables; None if it accepts them."""
    from paper_2503_10263_amd import karl
    try:
        job = karl.Job(w, precision=precision, queue_capacity=1 << 12)
    except karl.KarlError as e:
        assert e.code == karl.EINVAL, str(e)
        m = re.search(r"tables need (\d+) bytes of LDS", str(e))
        assert m, str(e)
        return int(m.group(1))
    job.close()
    return None


def test_fp64_tables_at_the_lds_limit_equal_oracle():
    per_node = len(_full(2).processes) * 8
    big = _lds_need(_full(1024), "fp64")
    assert big is not None and big > LDS_LIMIT
    # the need is the tables' bytes rounded up to 16, and grows by per_node a node: the
    # largest node count that fits is est or est - 1
    est = 1024 - (big - 15 - LDS_LIMIT + per_node - 1) // per_node
    n = next((k for k in (est, est - 1) if _lds_need(_full(k), "fp64") is None), None)
    assert n is not None, f"neither {est} nor {est - 1} nodes fit"
    over = _lds_need(_full(n + 1), "fp64")
    assert over is not None and LDS_LIMIT < over <= LDS_LIMIT + per_node + 15
    print(f"FP64 full case: {n} nodes fit ({over} bytes for {n + 1})", flush=True)
    g, o, frac = parity(_full(n))
    assert frac == 1.0
    assert o["counters"][oracle.C_BIRTH + 1] > 0                 # ions, in the deferred launch
    assert o["counters"][oracle.C_DEATH + oracle.NREASON + W.REASONS.index("cap")] > 0


def test_fp32_tables_at_the_node_limit():
    from paper_2503_10263_amd import karl
    w = _full(1024, n_primaries=200)
    job = karl.Job(w, precision="fp32", queue_capacity=1 << 16)
    try:
        job.transport(0, w.n_primaries)
        t = job.read_tallies()
    finally:
        job.close()
    assert_identities(t["counters"], t["ledger"], w.n_primaries, w.processes, 1e-3)
    assert t["counters"][karl.C_BIRTH + 1] > 0
