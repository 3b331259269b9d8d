"""Request loop over a libkarl server: replays a stream of transport requests (arrival time,
workload) against karl.Server in real time and reports job latency and throughput.

Admission, the arena allocator and the rounds of batched transport are native (libkarl);
this loop only submits requests when they arrive, steps the server and collects completions.
"""
import time
from typing import Dict, List, Sequence, Tuple

import numpy as np

from . import karl


def collisions_of(counters: np.ndarray) -> int:
    """Performed interactions of all species (the KARL_C_COLL entries of the counters)."""
    return int(sum(counters[karl.C_COLL + k] for k in range(karl.MAX_SPECIES)))


def replay(server: "karl.Server", requests: Sequence[Tuple[float, object]], realtime: bool = True,
           keep_tallies: bool = False, threaded: bool = True, on_complete=None,
           deadline_s: float = float("inf")) -> Dict[str, object]:
    """Submit request i at its arrival time (seconds after the start; all at once when
    `realtime` is False) until every request has completed; read each job's counters (or all
    its tallies with keep_tallies) and release it.  With `threaded` the server's worker
    threads run the rounds and this loop only submits, waits and collects; otherwise the loop
    steps the server itself.

    Latency of a job = completion time - arrival time, where completion is the end of the
    round that transported its last primary (as seen by this loop).  Returns per-job
    latency/collisions, their p50/p99, the throughput and the server's statistics.  A run
    still going `deadline_s` seconds after the start is stopped: jobs not completed by then
    count with their latency so far (a lower bound; "censored" gives their number)."""
    n = len(requests)
    order = sorted(range(n), key=lambda k: requests[k][0])
    arrival: Dict[int, float] = {}
    index_of: Dict[int, int] = {}
    latency = np.zeros(n)
    collisions = np.zeros(n, dtype=np.int64)
    tallies: List[object] = [None] * n
    backlog = []
    nxt = 0
    done = 0
    if threaded:
        server.start()
    t0 = time.perf_counter()
    try:
        while done < n:
            now = time.perf_counter() - t0
            if now > deadline_s:
                break
            while nxt < n and (not realtime or requests[order[nxt]][0] <= now):
                k = order[nxt]
                t = server.submit(requests[k][1])
                index_of[t] = k
                arrival[t] = requests[k][0] if realtime else now
                nxt += 1
            if threaded:
                until_next = requests[order[nxt]][0] - now if (realtime and nxt < n) else 0.05
                n_active, n_pending = server.wait(1e3 * min(max(until_next, 0.0), 0.05))
            else:
                n_active, n_pending = server.step()
            backlog.append((time.perf_counter() - t0, n_active + n_pending))
            for t in server.poll():
                end = time.perf_counter() - t0
                k = index_of[t]
                if keep_tallies:
                    tallies[k] = server.read_tallies(t)
                    c = tallies[k]["counters"]
                else:
                    c = server.read_tallies(t, only=("counters",))["counters"]
                latency[k] = end - arrival[t]
                collisions[k] = collisions_of(c)
                if on_complete is not None:
                    on_complete(k, t)
                server.release(t)
                done += 1
            if not threaded and n_active == 0 and n_pending == 0 and nxt < n and realtime:
                wait = requests[order[nxt]][0] - (time.perf_counter() - t0)
                if wait > 0:
                    time.sleep(wait)
    finally:
        if threaded:
            server.stop()
    wall = time.perf_counter() - t0
    censored = 0
    for t, k in index_of.items():
        if latency[k] == 0.0:
            latency[k] = wall - arrival[t]
            censored += 1
    censored += n - len(index_of)
    first = min(r[0] for r in requests) if realtime else 0.0
    st = server.stats()
    return {
        "latency_s": latency,
        "collisions": collisions,
        "tallies": tallies,
        "p50_s": float(np.percentile(latency, 50)),
        "p99_s": float(np.percentile(latency, 99)),
        "mean_s": float(latency.mean()),
        "wall_s": wall,
        "collisions_per_s": float(collisions.sum() / max(wall - first, 1e-9)),
        "busy_fraction": st["busy_ms"] / 1e3 / max(wall, 1e-9),
        "max_backlog": max(b for _, b in backlog) if backlog else 0,
        "censored": censored,
        "stats": st,
    }


def window(server: "karl.Server", requests: Sequence[Tuple[float, object]], window_s: float) -> Dict[str, object]:
    """Submit the requests arriving within `window_s` seconds at their arrival times while the
    server's worker threads run, collect what completes, and stop at the end of the window
    (the workers finish their current rounds; unfinished jobs stay in the server, which the
    caller destroys).  Returns what arrived and completed, the primaries still to transport,
    and the collisions per second the device transported over the window (completed and
    unfinished jobs alike)."""
    order = sorted(range(len(requests)), key=lambda k: requests[k][0])
    tickets = {}
    done = set()
    nxt = 0
    server.start()
    t0 = time.perf_counter()
    try:
        while True:
            now = time.perf_counter() - t0
            if now >= window_s:
                break
            while nxt < len(order) and requests[order[nxt]][0] <= now:
                k = order[nxt]
                tickets[server.submit(requests[k][1])] = k
                nxt += 1
            until_next = requests[order[nxt]][0] - now if nxt < len(order) else window_s - now
            server.wait(1e3 * min(max(until_next, 0.0), 0.05))
            for t in server.poll():
                done.add(t)
    finally:
        server.stop()
    elapsed = time.perf_counter() - t0
    for t in server.poll():
        done.add(t)
    collisions = 0
    for t in tickets:
        try:
            c = server.read_tallies(t, only=("counters",))["counters"]
        except karl.KarlError:       # never admitted: nothing transported
            continue
        collisions += collisions_of(c)
    st = server.stats()
    arrived_prims = sum(requests[k][1].n_primaries for k in tickets.values())
    return {"arrived": len(tickets), "completed": len(done), "elapsed_s": elapsed,
            "primaries": int(st["primaries"]), "primaries_backlog": int(arrived_prims - st["primaries"]),
            "collisions": int(collisions), "collisions_per_s": collisions / elapsed}
