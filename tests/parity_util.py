"""Helpers shared by the GPU parity tests: run the HIP path and the oracle on the same
workload and pid set, and compare them to the stated bar.

Bar (FP64 path): identical per-primary event digests for at least 99.9 % of the
histories; over the histories that match, every integer tally bit-exact; FP64 weighted
tallies within 1e-12 relative (element-wise, summation order of atomics is free)."""
import numpy as np

INT_KEYS = ["counters", "recomb", "jz", "jr", "spectra"]
FLOAT_KEYS = ["density_time", "ledger"]
RTOL = 1e-12


def ranges_excluding(lo, hi, bad):
    """Contiguous pid ranges covering [lo, hi) without the pids in `bad`."""
    out, start = [], lo
    for b in sorted(int(x) for x in bad):
        if start < b:
            out.append((start, b))
        start = b + 1
    if start < hi:
        out.append((start, hi))
    return out


def run_gpu(w, ranges, **kw):
    from paper_2503_10263_amd import karl
    job = karl.Job(w, **kw)
    try:
        for a, b in ranges:
            job.transport(a, b)
        return job.read_tallies(), job.stats()
    finally:
        job.close()


def run_oracle(w, ranges, digests=False, hist=False):
    import oracle
    t = oracle.empty_tallies(w, digests, hist)
    for a, b in ranges:
        oracle.run(w, a, b, tallies=t)
    return t


def assert_float_close(name, got, ref, scale=None):
    got = np.asarray(got, np.float64)
    ref = np.asarray(ref, np.float64)
    tol = RTOL * np.abs(ref)
    if scale is not None:
        tol = np.maximum(tol, RTOL * scale)
    bad = np.abs(got - ref) > tol
    assert not bad.any(), (f"{name}: {bad.sum()} elements differ beyond {RTOL:g} relative; "
                           f"worst {np.max(np.abs(got - ref)[bad] / np.maximum(np.abs(ref[bad]), 1e-300)):.3e}")


def compare_tallies(g, o, energy_scale):
    for k in INT_KEYS:
        np.testing.assert_array_equal(g[k], o[k], err_msg=k)
    assert_float_close("density_time", g["density_time"], o["density_time"])
    assert_float_close("ledger", g["ledger"], o["ledger"], scale=energy_scale)


def parity(w, lo=0, hi=None, min_match=0.999, **gpu_kw):
    """Full parity check of pids [lo, hi); returns (gpu tallies, oracle tallies, match fraction)."""
    hi = w.n_primaries if hi is None else hi
    g, _ = run_gpu(w, [(lo, hi)], digests=True, history=True, **gpu_kw)
    o = run_oracle(w, [(lo, hi)], digests=True, hist=True)
    dg, do = g["digests"][lo:hi], o["digests"][lo:hi]
    match = dg == do
    frac = float(match.mean()) if hi > lo else 1.0
    assert frac >= min_match, f"only {frac:.5f} of histories have identical event sequences"
    e_scale = max(abs(o["ledger"][0]), 1.0)
    if frac < 1.0:
        bad = lo + np.nonzero(~match)[0]
        rng = ranges_excluding(lo, hi, bad)
        g2, _ = run_gpu(w, rng, **gpu_kw)
        o2 = run_oracle(w, rng)
        compare_tallies(g2, o2, e_scale)
    else:
        compare_tallies(g, o, e_scale)
        # per-history ledgers: entry, accounted energy, births, deletions
        hg, ho = g["hist"][lo:hi], o["hist"][lo:hi]
        np.testing.assert_array_equal(hg[:, 2:], ho[:, 2:])
        assert_float_close("hist", hg[:, :2], ho[:, :2], scale=1e-3)
    return g, o, frac


def assert_identities(c, L, n_primaries, processes, energy_rtol):
    """Identities of a transport that hold at any size: one electron per primary and per
    ionization, one ion per ionization, every particle deleted exactly once, and the energy
    budget (primary energy = energy leaving + excitation + binding + given to the gas) within
    energy_rtol."""
    from paper_2503_10263_amd import karl as K
    from paper_2503_10263_amd import workloads as W
    nr = K.NREASON
    n_ion = sum(int(c[K.C_PROC + i]) for i, p in enumerate(processes) if p.kind == W.IONIZATION)
    assert c[K.C_BIRTH] == n_primaries + n_ion    # electrons: primaries + one per ionization
    assert c[K.C_BIRTH + 1] == n_ion              # ions: one per ionization
    deaths = c[K.C_DEATH:K.C_DEATH + 2 * nr].reshape(2, nr)
    assert deaths[0].sum() == c[K.C_BIRTH] and deaths[1].sum() == c[K.C_BIRTH + 1]   # each deleted once
    out = L[K.L_E_DEATH:K.L_E_DEATH + 2 * nr].sum() + L[K.L_E_EXC] + L[K.L_E_BIND] + L[K.L_E_GAS]
    assert abs(out / L[K.L_E_PRIMARY] - 1.0) < energy_rtol
