"""Pins of the oracle's density-field coupling (Sec. 2.2 "Density fields", Sec. 3.3
"Recombination", Sec. 3.6 cycles, Sec. 4 "Recombination"):

* a paired beam injects electrons on even and ions on odd primary ids;
* an ion beam recombining on a fixed electron field decays as exp(-n sigma z) and its
  recombinations are logged in the electron field, cell by cell;
* electrons and ions recombining on each other's field, with the fields updated from the
  tallies after every cycle of primaries, settle where n_e = (sigma_e / sigma_i) n_i + c (the
  relation the paper derives from the coupled advection equations with a sink)."""
import math

import numpy as np
import pytest
from scipy import stats

from paper_2503_10263_amd import workloads as W

P_MIN = 1e-4


@pytest.fixture(scope="module")
def oracle_lib():
    import oracle
    oracle.build(force=False)
    return oracle


def test_pair_source_species_by_parity(oracle_lib):
    w = W.recombination_pair(1e-20, 1e-20, n_primaries=10)
    for pid in range(6):
        t = oracle_lib.run(w, pid, pid + 1)
        c = t["counters"]
        sp = pid & 1
        assert c[oracle_lib.C_BIRTH + sp] == 1 and c[oracle_lib.C_BIRTH + 1 - sp] == 0
        # with empty fields both exit at the far end with their injection energy
        assert c[oracle_lib.C_DEATH + sp * oracle_lib.NREASON + W.REASONS.index("exit_high")] == 1
        e_exit = t["ledger"][oracle_lib.L_E_DEATH + sp * oracle_lib.NREASON + W.REASONS.index("exit_high")]
        assert e_exit == (w.beam_energy_1 if sp else w.beam_energy)


def test_ion_recombination_on_fixed_electron_field(oracle_lib):
    n_e, sig, n_z, L = 1.0e18, 2.0e-18, 40, 1.0
    w = W.recombination_pair(1e-30, sig, n_primaries=40000, n_z=n_z, length=L,
                             n_elec=np.full(n_z, n_e), n_ion=np.zeros(n_z))
    t = oracle_lib.run(w)
    N = w.n_primaries // 2                       # odd ids are ions
    mu = n_e * sig
    trans = t["counters"][oracle_lib.C_DEATH + oracle_lib.NREASON + W.REASONS.index("exit_high")]
    p = math.exp(-mu * L)
    assert abs(trans - N * p) < 4.0 * math.sqrt(N * p * (1 - p))
    counts = t["recomb"][0, 0]                    # ion recombinations, logged in the electron field
    assert t["recomb"][1].sum() == 0              # electrons see an empty ion field
    zf = np.linspace(0.0, L, n_z + 1)
    exp_counts = N * (np.exp(-mu * zf[:-1]) - np.exp(-mu * zf[1:]))
    chi2 = np.sum((counts - exp_counts) ** 2 / exp_counts)
    assert stats.chi2.sf(chi2, n_z - 1) > P_MIN
    assert counts.sum() + trans == N


def run_cycles(oracle_lib, w, activity, cycle, n_cycles):
    """The cycle scheme: transport `cycle` primaries, set both target fields to the densities
    of everything transported so far, repeat."""
    t = oracle_lib.empty_tallies(w, False, False)
    dens = None
    for k in range(n_cycles):
        oracle_lib.run(w, k * cycle, (k + 1) * cycle, tallies=t)
        dens = oracle_lib.fields(w, t, (k + 1) * cycle, activity)["density"]
        w.n_elec = np.clip(dens[0].reshape(-1), 0.0, None)
        w.n_ion = np.clip(dens[1].reshape(-1), 0.0, None)
    return t, dens


def test_coupled_recombination_slope(oracle_lib):
    sig_e, sig_i = 2.0e-17, 1.6e-17
    n_z, L, R, n0 = 40, 1.0, 0.05, 2.0e16
    w = W.recombination_pair(sig_e, sig_i, n_primaries=200000, n_z=n_z, length=L, radius=R)
    v = math.sqrt(2.0 * w.beam_energy * W.QE / W.M_E)
    activity = 2.0 * n0 * v * math.pi * R * R      # each species alone would have density n0
    t, dens = run_cycles(oracle_lib, w, activity, 4000, 12)
    ne, ni = dens[0, 0], dens[1, 0]
    assert abs(ne[0] / n0 - 1.0) < 0.02 and abs(ni[0] / n0 - 1.0) < 0.02
    assert ne[-1] < 0.8 * n0 and ni[-1] < 0.85 * n0        # both decay along the tube
    slope = np.polyfit(ni, ne, 1)[0]
    assert abs(slope / (sig_e / sig_i) - 1.0) < 0.05
    # every recombination of one species is a deletion logged in the other's field
    c = t["counters"]
    assert c[oracle_lib.C_DEATH + W.REASONS.index("recombined")] == t["recomb"][1].sum()
    assert c[oracle_lib.C_DEATH + oracle_lib.NREASON + W.REASONS.index("recombined")] == t["recomb"][0].sum()
