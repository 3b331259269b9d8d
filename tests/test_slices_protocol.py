"""Model check (CPU) of the work protocol of the deferred launch in slices.

The kernel's lanes claim work from one counter over the launch's items and a ring of particle
states; a particle goes back into the ring every `slice` of its steps if the ring slot it would
take has been read; waves end when nothing is claimable and none of their lanes holds work.
This test restates that protocol at the granularity of its shared-memory operations -- every
atomic load, compare-and-swap and flag store is one step of a wave -- and runs it under seeded
random interleavings of the waves, with rings so small that they wrap and find their slots
still in use.  Checked: every particle runs exactly its number of steps, every ring index is
written once and read once, and every wave ends (no lane waits on an entry nobody writes).
It checks the protocol's design, independently of the GPU; the GPU tests check the kernel."""
import random

import pytest

TRIES = 16   # attempts per claim / put, as in the kernel


class Shared:
    def __init__(self, n_items, ring_cap):
        self.n = n_items
        self.cap = ring_cap
        self.fetch = 0
        self.tail = 0
        self.flag = [0] * ring_cap
        self.ring = [None] * ring_cap
        self.written = {}
        self.read = {}

    def cas(self, name, old, new):
        if getattr(self, name) == old:
            setattr(self, name, new)
            return True
        return False


def run_model(seed, n_waves, lanes, n_items, ring_cap, slice_steps, max_len):
    rng = random.Random(seed)
    items = [rng.randint(1, max_len) for _ in range(n_items)]
    n_static = min(n_items, n_waves * lanes)
    sh = Shared(n_items, ring_cap)
    sh.fetch = n_static
    done_steps = [0] * n_items
    gens = [wave(sh, lanes, items, slice_steps, done_steps, w) for w in range(n_waves)]
    live = list(range(n_waves))
    ticks = 0
    budget = 200 * (sum(items) + 10 * n_items + 1000)
    while live:
        ticks += 1
        assert ticks < budget, "no progress: a wave never ends"
        w = rng.choice(live)
        try:
            next(gens[w])
        except StopIteration:
            live.remove(w)
    return items, done_steps, sh


def wave(sh, lanes, items, slice_steps, done_steps, w):
    """Wave w as a generator that yields after each shared-memory operation.  Lane state: None
    (idle), ("run", pid, steps so far, steps left) or ("wait", ring index).  Its lanes start on
    the items of their thread index (the claim counter starts past them)."""
    st = [("run", u, 0, items[u]) if u < sh.n else None for u in (w * lanes + k for k in range(lanes))]
    skip = 0
    while True:
        for k in range(lanes):
            if st[k] and st[k][0] == "wait":
                i = st[k][1]
                slot = i % sh.cap
                f = sh.flag[slot]
                yield
                if f == 2 * i + 1:
                    pid, s, left = sh.ring[slot]
                    assert i not in sh.read, f"ring index {i} read twice"
                    sh.read[i] = pid
                    yield
                    sh.flag[slot] = 2 * i + 2
                    yield
                    st[k] = ("run", pid, s, left)
        need = [k for k in range(lanes) if st[k] is None]
        if need:
            busy = any(x is not None for x in st)
            if not busy or skip == 0:
                res, base, got = -1, 0, 0
                for _ in range(TRIES):
                    h = sh.fetch
                    yield
                    total = sh.n + sh.tail
                    yield
                    if h >= total:
                        res = 0
                        break
                    take = min(len(need), total - h)
                    ok = sh.cas("fetch", h, h + take)
                    yield
                    if ok:
                        base, got, res = h, take, 1
                        break
                for r, k in enumerate(need[:got]):
                    u = base + r
                    st[k] = ("run", u, 0, items[u]) if u < sh.n else ("wait", u - sh.n)
                if res == 0 and not busy:
                    return
                skip = 0 if res == 1 else (32 if res == 0 else 4)
            else:
                skip -= 1
        for k in range(lanes):
            if st[k] and st[k][0] == "run":
                _, pid, s, left = st[k]
                done_steps[pid] += 1
                st[k] = None if left == 1 else ("run", pid, s + 1, left - 1)
        yield
        want = [k for k in range(lanes)
                if st[k] and st[k][0] == "run" and st[k][2] % slice_steps == 0]
        for _ in range(TRIES):
            if not want:
                break
            keep = []
            for k in want:
                j = sh.tail
                yield
                slot = j % sh.cap
                free = 0 if j < sh.cap else 2 * (j - sh.cap) + 2
                f = sh.flag[slot]
                yield
                if f != free:
                    if sh.tail != j:
                        keep.append(k)   # the tail moved: try the next index
                    continue             # else the slot is still in use: keep the particle
                if sh.cas("tail", j, j + 1):
                    yield
                    _, pid, s, left = st[k]
                    assert j not in sh.written, f"ring index {j} written twice"
                    sh.written[j] = pid
                    sh.ring[slot] = (pid, s, left)
                    yield
                    sh.flag[slot] = 2 * j + 1
                    yield
                    st[k] = None
                else:
                    keep.append(k)
            want = keep


@pytest.mark.parametrize("seed", range(12))
@pytest.mark.parametrize("ring_cap,slice_steps", [(2, 2), (5, 3), (64, 4), (1000, 1)])
def test_every_particle_runs_its_steps_and_every_wave_ends(seed, ring_cap, slice_steps):
    items, done, sh = run_model(seed, n_waves=5, lanes=4, n_items=37, ring_cap=ring_cap,
                                slice_steps=slice_steps, max_len=40)
    assert done == items                                   # every particle ran all its steps
    assert set(sh.written) == set(sh.read)                 # every ring entry written was read
    assert sorted(sh.written) == list(range(sh.tail))      # indices 0..tail-1, once each
    assert sh.fetch == sh.n + sh.tail                      # every index claimed
    if ring_cap >= 64:
        assert sh.tail > 0                                 # particles did go round the ring


def test_more_lanes_than_items_and_empty_launch():
    items, done, sh = run_model(3, n_waves=4, lanes=8, n_items=5, ring_cap=3, slice_steps=2, max_len=30)
    assert done == items and set(sh.written) == set(sh.read)
    items, done, sh = run_model(4, n_waves=3, lanes=4, n_items=0, ring_cap=3, slice_steps=2, max_len=1)
    assert done == [] and sh.tail == 0
