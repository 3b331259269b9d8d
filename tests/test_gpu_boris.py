"""The Boris mover on the GPU against the oracle (Sec. 3.1 "Boris mover"; vector fields from
arrays, Sec. 3.8).

Beta electrons and tracked H2+ pushed through a binned magnetic bottle with a radial electric
field, with gas interactions and secondaries: event digests and tallies to the parity bar,
the field work in the ledger included.  An accelerated beam with energy-resolved density
fields (movements also stop at energy-bin changes), an absorbing field (the interaction at the
end of a movement), Boris jobs inside a batch next to a drift job, and the FP32 state against
the closed-form transmission."""
import math

import numpy as np
import pytest

import oracle
from paper_2503_10263_amd import workloads as W
from parity_util import assert_float_close, parity, run_gpu, run_oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    oracle.build(force=False)


def test_boris_column_parity():
    w = W.boris_column(n_primaries=600)
    g, o, frac = parity(w)
    assert o["counters"][oracle.C_COLL] > 500 and o["counters"][oracle.C_BIRTH + 1] > 50
    # trapped electrons end by lifetime; the field worked on the particles
    assert o["counters"][oracle.C_DEATH + W.REASONS.index("lifetime")] > 20
    assert o["ledger"][oracle.L_E_FIELD] != 0.0


def _accelerated_beam(n_primaries, n_z=12, L=0.6, e_z=-40.0):
    w = W.beam_problem(2.0, [], np.zeros(n_z), L, radius=0.05, n_primaries=n_primaries)
    w = W.with_boris(w, dt=[2.0e-11, 1e-9], lifetime=[1e-5, 1.0],
                     e_field=W.uniform_vector_field(2, 3, (5.0, 0.0, e_z)))
    w.dens_edges = (np.linspace(0.0, 30.0, 16), np.linspace(0.0, 1.0, 16))
    return w


def test_accelerated_beam_energy_bins():
    w = _accelerated_beam(40)
    g, o, frac = parity(w)
    assert_float_close("density_time_e", g["density_time_e"], o["density_time_e"])
    assert np.count_nonzero(o["density_time_e"][0].sum(axis=(0, 1))) > 5


def test_absorbing_field_interactions():
    n_z, L, N, sig, n3 = 20, 1.0, 4000, 1.0e-18, 8.0e17
    E = 5.0
    v = math.sqrt(2.0 * E * W.QE / W.M_E)
    dt = L / (v * 300.45)
    species = [W.electron(e_cut=0.0, edges=np.linspace(0, 10, 11)), W.ion_species("H2+", W.M_H2P, n_bins=10)]
    species[1].edges = np.linspace(0, 10, 11)
    procs = [W.Process(W.RECOMBINATION, W.ELECTRON, W.TARGET_FIELD, 0.0, np.full(256, sig), "rec", partner=1)]
    w = W.beam_problem(E, procs, np.zeros(n_z), L, radius=0.05, n_primaries=N, species=species,
                       n_ion=np.full(n_z, n3))
    w = W.with_boris(w, dt=[dt, 1e-9], lifetime=[1e-5, 1.0],
                     b_field=W.uniform_vector_field(1, 1, (0.0, 0.0, 0.2)))
    g, o, frac = parity(w)
    assert o["recomb"][1].sum() > 500


def test_boris_jobs_in_a_batch():
    from paper_2503_10263_amd import karl
    ws = [W.boris_column(n_primaries=150, seed=61), W.cfg_tiny(n_primaries=500, bz=2.0, column_cm2=3e17),
          _accelerated_beam(20)]
    jobs = [karl.Job(w, digests=True, queue_capacity=4096) for w in ws]
    batch = karl.Batch(max_jobs=len(ws), queue_capacity=1 << 18)
    try:
        batch.transport(jobs, [(0, w.n_primaries) for w in ws])
        for k, (w, job) in enumerate(zip(ws, jobs)):
            g = job.read_tallies()
            o = run_oracle(w, [(0, w.n_primaries)], digests=True)
            match = float(np.mean(g["digests"] == o["digests"]))
            assert match >= 0.999, (k, match)
            if match == 1.0:
                for key in ["counters", "recomb", "jz", "jr", "spectra"]:
                    np.testing.assert_array_equal(g[key], o[key], err_msg=f"job {k}: {key}")
                assert_float_close("density_time", g["density_time"], o["density_time"])
    finally:
        for j in jobs:
            j.close()
        batch.close()


def test_fp32_boris_transmission():
    """FP32 state: the transmission through an absorbing field follows the discrete closed form
    exp(-mu v dt (K - n_z)) of the Boris movement."""
    n_z, L, N, sig, n3 = 40, 1.0, 20000, 1.0e-18, 8.0e17
    E = 5.0
    v = math.sqrt(2.0 * E * W.QE / W.M_E)
    dt = L / (v * 300.45)
    species = [W.electron(e_cut=0.0, edges=np.linspace(0, 10, 11)), W.ion_species("H2+", W.M_H2P, n_bins=10)]
    species[1].edges = np.linspace(0, 10, 11)
    procs = [W.Process(W.RECOMBINATION, W.ELECTRON, W.TARGET_FIELD, 0.0, np.full(256, sig), "rec", partner=1)]
    w = W.beam_problem(E, procs, np.zeros(n_z), L, radius=0.05, n_primaries=N, species=species,
                       n_ion=np.full(n_z, n3))
    w = W.with_boris(w, dt=[dt, 1e-9], lifetime=[1e-5, 1.0])
    g, _ = run_gpu(w, [(0, N)], precision="fp32")
    K = math.ceil(L / (v * dt))
    p = math.exp(-n3 * sig * v * dt * (K - n_z))
    trans = g["counters"][oracle.C_DEATH + W.REASONS.index("exit_high")]
    assert abs(trans - N * p) < 4.5 * math.sqrt(N * p * (1 - p)), (trans, N * p)
