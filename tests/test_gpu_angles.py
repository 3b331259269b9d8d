"""Tabulated and composite elastic angle distributions (Sec. 3.3 "Elastic scattering") on the
GPU against the oracle: identical event digests and tallies to the parity bar, plain and in a
batch, straight-line and guiding-centre transport."""
import numpy as np
import pytest

import oracle
from paper_2503_10263_amd import workloads as W
from parity_util import compare_tallies, parity, run_oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    import oracle
    oracle.build(force=False)


def _with_table(w, e_iso=100.0):
    w.processes[0].angular = W.screened_table(e_iso=e_iso)
    return w


def test_composite_table_straight_line():
    w = _with_table(W.cfg_tiny(n_primaries=3000, column_cm2=1.0e17))
    g, o, frac = parity(w)
    assert o["counters"][oracle.C_PROC] > 1000        # elastic collisions happened


def test_table_guiding_centre_grid():
    w = _with_table(W.cfg_tiny(n_primaries=1200, column_cm2=1.0e17, bz=2.5, n_r=8, n_z=16), 0.0)
    w.planes = [0, 8, 16]
    parity(w)


def test_table_in_a_batch_equals_oracle():
    from paper_2503_10263_amd import karl
    ws = [_with_table(W.cfg_tiny(n_primaries=300, column_cm2=c, bz=b, seed=s), e)
          for c, b, s, e in [(1e17, 2.0, 3, 100.0), (3e17, 0.0, 4, 0.0), (1e16, 3.0, 5, 500.0)]]
    ws.append(W.cfg_tiny(n_primaries=300, column_cm2=1e17, bz=2.0, seed=6))   # isotropic
    jobs = [karl.Job(w, digests=True, queue_capacity=1 << 14) for w in ws]
    batch = karl.Batch(max_jobs=4, queue_capacity=1 << 16)
    batch.transport(jobs, [(0, w.n_primaries) for w in ws])
    for w, job in zip(ws, jobs):
        g = job.read_tallies()
        o = run_oracle(w, [(0, w.n_primaries)], digests=True)
        np.testing.assert_array_equal(g["digests"], o["digests"])
        compare_tallies(g, o, abs(o["ledger"][0]))
        job.close()
    batch.close()
