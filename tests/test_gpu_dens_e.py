"""Energy-resolved density field (Sec. 3.4) on the GPU against the oracle.

Each flight segment adds its time to the bin of the particle's energy; the GPU sums these in
another order than the oracle (FP64 atomics), with up to ~1e6 addends per bin at these sizes,
so bins are compared to n_add * 2^-53 ~ 1e-10 of the bin (1e-9 used), and every other tally to
the usual bar.  Lane and wave mappings, FP64."""
import numpy as np
import pytest

from paper_2503_10263_amd import workloads as W
from parity_util import compare_tallies, run_gpu, run_oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    import oracle
    oracle.build(force=False)


@pytest.mark.parametrize("mapping", ["lane", "wave"])
def test_energy_resolved_density_matches_oracle(mapping):
    w = W.cfg_tiny(n_primaries=1500, column_cm2=3.0e16, bz=2.5, n_r=4, n_z=64)
    w.planes = [0, 32, 64]
    w.dens_edges = (np.geomspace(1.0, 2.0e4, 41), np.geomspace(1e-3, 1e2, 41))
    g, _ = run_gpu(w, [(0, w.n_primaries)], digests=True, mapping=mapping)
    o = run_oracle(w, [(0, w.n_primaries)], digests=True)
    np.testing.assert_array_equal(g["digests"], o["digests"])
    compare_tallies(g, o, max(abs(o["ledger"][0]), 1.0))
    ge, oe = g["density_time_e"], o["density_time_e"]
    assert np.all(np.abs(ge - oe) <= 1e-9 * np.abs(oe)), np.max(np.abs(ge - oe) / np.maximum(np.abs(oe), 1e-300))
    np.testing.assert_allclose(ge.sum(axis=3), g["density_time"], rtol=1e-9)


def test_full_case_with_energy_resolved_ions():
    w = W.cfg_full(n_primaries=30)
    w.species[W.ION].cap = 2000
    w.dens_edges = (np.geomspace(1.0, 2.0e4, 17), np.geomspace(1e-4, 1e2, 17))
    g, _ = run_gpu(w, [(0, w.n_primaries)], digests=True)
    o = run_oracle(w, [(0, w.n_primaries)], digests=True)
    np.testing.assert_array_equal(g["digests"], o["digests"])
    ge, oe = g["density_time_e"], o["density_time_e"]
    assert np.all(np.abs(ge - oe) <= 1e-9 * np.abs(oe))
    assert ge[1].sum() > 0                     # the tracked ions fill their own bins
