"""The mixed-precision case at its real size (the tiny case at 1e8 primaries, FP32 particle state
and arithmetic, FP64/int64 tallies and ledgers) against FP64 on identical random streams, and
the FP64 path against the oracle on a prefix of the same primaries.

Bar for FP32 (the reading of Sec. 2.1's estimator: the same process, rounded more coarsely):
mean energy deposited per primary within 0.1 % of FP64, and the exit spectra equal by a
two-sample chi-square over bins merged to >= 20 counts at p > 0.01.  The runs share their
streams, so the batch-paired statistics (the same primaries in each batch) are reported too."""
import pytest

from paper_2503_10263_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.mark.timeout(300)
def test_fp64_equals_oracle_on_a_prefix_of_the_mixed_case():
    import parity_util as P
    w = W.cfg_mixed(n_primaries=100_000_000)
    print("mixed case FP64: primaries 0..99999 against the oracle", flush=True)
    _, _, frac = P.parity(w, 0, 100_000, queue_capacity=1 << 20)
    assert frac == 1.0


@pytest.mark.timeout(300)
def test_fp32_against_fp64_at_1e8_primaries():
    import bench
    print("mixed case: 1e8 primaries in FP64 and FP32, 50 paired batches", flush=True)
    r = bench.mixed_precision(100_000_000, 50)
    print({k: v for k, v in r.items() if not isinstance(v, str)}, flush=True)
    assert abs(r["mean_loss_rel_err"]) < 1e-3, r
    assert r["spectrum_p"] > 0.01, r
    assert r["spectrum_bins"] > 1000
