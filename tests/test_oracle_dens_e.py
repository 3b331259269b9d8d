"""Pins of the oracle's energy-resolved density field (Sec. 3.4: times per segment with an
energy axis, the fastest-varying one).

* Summed over the energy bins it equals the plain density field.
* An excitation-only beam (constant cross section, no deflection) occupies energy levels
  E0 - j E_x; the time spent at level j in a z-segment follows the Poisson law of the number
  of excitations along the path: N/(v_j mu) [P(j+1, mu z_b) - P(j+1, mu z_a)] with P the
  regularized lower incomplete gamma function."""
import math

import numpy as np
import pytest
from scipy import special

from paper_2503_10263_amd import workloads as W


@pytest.fixture(scope="module")
def oracle_lib():
    import oracle
    oracle.build(force=False)
    return oracle


def test_energy_bins_sum_to_the_density_field(oracle_lib):
    w = W.cfg_tiny(n_primaries=1500, column_cm2=1.0e17, bz=2.5, n_r=4, n_z=8)
    w.dens_edges = (np.geomspace(1.0, 2.0e4, 33), np.geomspace(1e-3, 1e2, 33))
    t = oracle_lib.run(w)
    de = t["density_time_e"]
    assert de.shape == (2, 4, 8, 34)
    np.testing.assert_allclose(de.sum(axis=3), t["density_time"], rtol=1e-12, atol=0.0)
    assert de[0, :, :, 1:-1].sum() > 0.99 * de[0].sum()     # almost all within the edges


def test_excitation_levels_follow_poisson(oracle_lib):
    e0, ex, sig, n, L, n_z, N = 100.0, 10.0, 2.0e-20, 1.0e20, 1.0, 10, 20000
    proc = [W.Process(W.EXCITATION, W.ELECTRON, W.TARGET_GAS, ex, np.full(256, sig), "exc")]
    w = W.beam_problem(e0, proc, np.full(n_z, n), L, n_primaries=N)
    levels = 6
    edges = e0 - ex * (np.arange(levels - 1, -2, -1) + 0.5)    # one bin per level, increasing
    w.dens_edges = (edges, np.linspace(0.0, 1.0, levels + 1))
    t = oracle_lib.run(w)
    de = t["density_time_e"][0, 0]                                # [z][bin]
    mu = n * sig
    zf = np.linspace(0.0, L, n_z + 1)
    for j in range(levels):
        b = levels - j                                            # bin of level j (bin 0: below)
        v = math.sqrt(2.0 * (e0 - j * ex) * W.QE / W.M_E)
        for iz in range(n_z):
            expect = N / (v * mu) * (special.gammainc(j + 1, mu * zf[iz + 1]) -
                                     special.gammainc(j + 1, mu * zf[iz]))
            frac = expect * v / (N * (zf[iz + 1] - zf[iz]))       # mean share of the beam there
            tol = 5.0 / math.sqrt(max(N * frac, 1.0))
            assert abs(de[iz, b] / expect - 1.0) < tol, (j, iz, de[iz, b], expect)
