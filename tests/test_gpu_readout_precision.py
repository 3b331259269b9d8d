"""GPU tests of the normalised readout and of the FP32 transport mode."""
import math

import numpy as np
import pytest
from scipy import stats

from paper_2503_10263_amd import karl as K
from paper_2503_10263_amd import workloads as W
from parity_util import run_oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    import oracle
    oracle.build(force=False)


def test_fields_match_oracle():
    """Densities and currents (eq. 3-5) computed on the device from the device tallies agree
    with the oracle's plain evaluation on the oracle's tallies."""
    import oracle
    from paper_2503_10263_amd import karl
    w = W.cfg_full(n_primaries=40)
    w.species[W.ION].cap = 2000
    act = 1.0e11
    job = karl.Job(w, queue_capacity=1 << 18)
    job.transport(0, 40)
    g = job.read_fields(act)
    job.close()
    o = oracle.fields(w, run_oracle(w, [(0, 40)]), 40, act)
    for k in ("density", "jz", "jr"):
        ref = o[k]
        tol = 1e-12 * np.maximum(np.abs(ref), np.abs(ref).max() * 1e-300)
        assert np.all(np.abs(g[k] - ref) <= tol + 1e-12 * np.abs(ref).max()), k
    assert np.abs(o["density"]).max() > 0


def test_fields_require_transported_primaries():
    from paper_2503_10263_amd import karl
    w = W.cfg_tiny(n_primaries=10)
    job = karl.Job(w, queue_capacity=1024)
    with pytest.raises(karl.KarlError) as ei:
        job.read_fields(1.0)
    assert ei.value.code == karl.ESTATE
    job.close()


def _merged_chi2(a, b, min_count=20):
    """Two-sample chi-square on histograms a, b with equal totals, bins merged to >= min_count."""
    ga, gb, ca, cb = [], [], 0, 0
    for x, y in zip(a, b):
        ca += x
        cb += y
        if ca + cb >= 2 * min_count:
            ga.append(ca)
            gb.append(cb)
            ca = cb = 0
    if ga:
        ga[-1] += ca
        gb[-1] += cb
    ga, gb = np.array(ga, float), np.array(gb, float)
    na, nb = ga.sum(), gb.sum()
    chi2 = np.sum((ga * math.sqrt(nb / na) - gb * math.sqrt(na / nb)) ** 2 / (ga + gb))
    return chi2, len(ga) - 1


@pytest.mark.parametrize("bz,column", [(0.0, 1e18), (2.5, 1e17)])
def test_fp32_statistics_against_fp64_oracle(bz, column):
    """FP32 transport state (FP64 tallies and ledgers) against the FP64 oracle: per-bin
    two-sample chi-square of the exit spectra (p > 0.01) and the mean energy deposited in the
    gas per primary within 0.1 %."""
    from paper_2503_10263_amd import karl
    N = 4000
    w = W.cfg_tiny(n_primaries=N, column_cm2=column, bz=bz)
    job = karl.Job(w, precision="fp32", queue_capacity=1 << 20)
    job.transport(0, N)
    g = job.read_tallies()
    job.close()
    o = run_oracle(w, [(0, N)])
    for end in range(2):
        a = g["spectra"][0, end].sum(axis=0)
        b = o["spectra"][0, end].sum(axis=0)
        chi2, dof = _merged_chi2(a, b)
        if dof > 0:
            assert stats.chi2.sf(chi2, dof) > 0.01, (end, chi2, dof)
    def deposited(t):
        L = t["ledger"]
        nr = K.NREASON
        escaped = L[K.L_E_DEATH:K.L_E_DEATH + 2 * nr].reshape(2, nr)[:, :3].sum()   # ends and wall
        return (L[K.L_E_PRIMARY] - escaped) / N
    dg, do = deposited(g), deposited(o)
    assert abs(dg / do - 1.0) < 1e-3, (dg, do)
    # particle bookkeeping is exact in any precision
    c = g["counters"]
    nr = K.NREASON
    assert c[K.C_DEATH:K.C_DEATH + nr].sum() == c[K.C_BIRTH]
    assert c[K.C_DEATH + nr:K.C_DEATH + 2 * nr].sum() == c[K.C_BIRTH + 1]
