"""Writes the oracle's results for the parity subsets of the full-size configurations (calls
only oracle/ and the seeded input generators; run on the CPU, the GPU tests read the files):

  full_case_pids_0_1000.npz       the full case (10 m, 2.5 T, 64x512 grid, 9 processes, tracked
                                  H2+ at the interaction cap of 1e6) for primaries 0..999:
                                  per-history digests and ledgers, every tally
  batched_case_first_1000.npz     each of the 256 jobs of the batched case for its primaries
                                  0..999 (or all, if it has fewer): per-history digests, counters,
                                  ledger, density times, and a SHA-256 of the integer tallies
                                  (recombinations, currents, spectra) per job

    python tests/golden/make_fullsize_fixtures.py {full|batched} [--procs N]

The main simulation cycle is the paper's Sec. 2.1; the workloads are the seeded synthetic
cases of paper_2503_10263_amd/workloads.py.  Histories are independent, so the primaries are
split over processes and the tallies summed.
"""
import argparse
import hashlib
import os
import sys
import time
from multiprocessing import Pool

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

FULL_PIDS = 1000
BATCHED_PIDS = 1000
INT_KEYS = ("recomb", "jz", "jr", "spectra")


def int_tally_sha(t) -> str:
    """SHA-256 over the integer tallies (int64, C order) in a fixed order."""
    h = hashlib.sha256()
    for k in INT_KEYS:
        h.update(np.ascontiguousarray(t[k], dtype=np.int64).tobytes())
    return h.hexdigest()


def _full_task(rng):
    import oracle
    from paper_2503_10263_amd import workloads as W
    w = W.cfg_full(n_primaries=1_000_000)
    t = oracle.run(w, rng[0], rng[1], digests=True, hist=True)
    t["digests"], t["hist"] = t["digests"][rng[0]:rng[1]], t["hist"][rng[0]:rng[1]]
    return rng, t


def _batched_task(args):
    import oracle
    from paper_2503_10263_amd import workloads as W
    j, b, e = args
    w = W.cfg_batched(n_jobs=256)[j]
    t = oracle.run(w, b, e, digests=True)
    t["digests"] = t["digests"][b:e]
    return (j, b, e), t


def make_full(procs: int):
    tasks = [(b, min(b + 10, FULL_PIDS)) for b in range(0, FULL_PIDS, 10)]
    total = None
    t0 = time.time()
    with Pool(procs) as pool:
        for n, (rng, t) in enumerate(pool.imap_unordered(_full_task, tasks)):
            if total is None:
                total = {k: np.zeros_like(v) for k, v in t.items() if k not in ("digests", "hist")}
                total["digests"] = np.zeros(FULL_PIDS, dtype=np.uint64)
                total["hist"] = np.zeros((FULL_PIDS, t["hist"].shape[1]))
            for k, v in t.items():
                if k in ("digests", "hist"):
                    total[k][rng[0]:rng[1]] = v
                else:
                    total[k] += v
            print(f"full: {n + 1}/{len(tasks)} tasks, {time.time() - t0:.0f} s", flush=True)
    out = os.path.join(HERE, f"full_case_pids_0_{FULL_PIDS}.npz")
    np.savez_compressed(out, pid_end=FULL_PIDS, digests=total["digests"][:FULL_PIDS],
                        hist=total["hist"][:FULL_PIDS], counters=total["counters"],
                        ledger=total["ledger"], density_time=total["density_time"],
                        recomb=total["recomb"], jz=total["jz"], jr=total["jr"],
                        spectra=total["spectra"])
    print("wrote", out, os.path.getsize(out), "bytes")


def make_batched(procs: int):
    from paper_2503_10263_amd import workloads as W
    ws = W.cfg_batched(n_jobs=256)
    ends = [min(BATCHED_PIDS, w.n_primaries) for w in ws]
    tasks = [(j, b, min(b + 100, ends[j])) for j in range(len(ws)) for b in range(0, ends[j], 100)]
    # the densest columns first, so that the pool ends together
    tasks.sort(key=lambda t: -ws[t[0]].n_gas[0])
    acc = [None] * len(ws)
    t0 = time.time()
    with Pool(procs) as pool:
        for n, ((j, b, e), t) in enumerate(pool.imap_unordered(_batched_task, tasks)):
            if acc[j] is None:
                acc[j] = {k: np.zeros_like(v) for k, v in t.items() if k != "digests"}
                acc[j]["digests"] = np.zeros(BATCHED_PIDS, dtype=np.uint64)
            for k, v in t.items():
                if k == "digests":
                    acc[j][k][b:e] = v
                else:
                    acc[j][k] += v
            if (n + 1) % 100 == 0 or n + 1 == len(tasks):
                print(f"batched: {n + 1}/{len(tasks)} tasks, {time.time() - t0:.0f} s", flush=True)
    digests = np.zeros((len(ws), BATCHED_PIDS), dtype=np.uint64)
    for j in range(len(ws)):
        digests[j, :ends[j]] = acc[j]["digests"][:ends[j]]
    out = os.path.join(HERE, f"batched_case_first_{BATCHED_PIDS}.npz")
    np.savez_compressed(out, pid_end=np.array(ends), digests=digests,
                        counters=np.stack([a["counters"] for a in acc]),
                        ledger=np.stack([a["ledger"] for a in acc]),
                        density_time=np.stack([a["density_time"] for a in acc]),
                        int_sha=np.array([int_tally_sha(a) for a in acc]))
    print("wrote", out, os.path.getsize(out), "bytes")


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("which", choices=["full", "batched"])
    ap.add_argument("--procs", type=int, default=max(1, (os.cpu_count() or 2) - 2))
    a = ap.parse_args()
    (make_full if a.which == "full" else make_batched)(a.procs)
