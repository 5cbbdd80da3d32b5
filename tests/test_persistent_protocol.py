"""A CPU model of the persistent batched launch's cross-workgroup protocol.

The persistent kernels (batch mode 0, one- and two-step passes) give each
workgroup the items it, it + G, it + 2G, ... of every pass.  Before pass s of
an item of lattice b it waits until the per-lattice counter done[b] reaches
s * n_b (n_b: the lattice's item count); after the item it adds one to
done[b].  The wait is bounded: past a spin limit the workgroup raises an abort
flag, and a raised flag makes every waiting workgroup leave.

Here each workgroup is a generator whose every step is one atomic action of
the kernel (a poll of done[b], the work of an item, its counter increment, a
claim on a queue); a seeded adversarial scheduler interleaves them, with at
most R workgroups resident at a time (the rest start, in order, as resident
ones finish), as the hardware dispatches a grid that does not fit at once.
The model is sequentially consistent: it checks the protocol's logic
(safety, liveness, that the bound ends every wait), not the memory orders,
which the kernels take as acquire on each poll and release after each
item's stores at device scope.

The kernels open with a census: each workgroup adds one to an arrival
counter and waits (bounded) until the whole grid has arrived.  A workgroup
whose census wait runs out closes the census by a compare-and-swap that sets a
high bit on the count it last saw, which fails if anyone arrived meanwhile;
late and waiting workgroups that see the bit leave.  No item starts unless the
whole grid is resident, so a grid too large for the device fails with the
state untouched, and the host retries with the closing count.

Also modelled: a pass-major job queue (one claim counter over all
(pass, item) jobs in order), a variant that was tried on the GPU and ran past
its time limit.  In this model it is live for any residency: a claimed job
waits only for jobs claimed before it, all held by resident workgroups.
"""
import random

import pytest

SPIN = 4000          # polls before a wait gives up (the kernels' bound is far larger)


class Deadlock(Exception):
    pass


def layout(rng, nlat, max_items):
    """Random lattices with 1..max_items items each; items of a lattice contiguous."""
    items = []
    for b in range(nlat):
        items += [b] * rng.randint(1, max_items)
    return items


class Machine:
    def __init__(self, items, npass, G, R, rng):
        self.items, self.npass, self.G, self.R, self.rng = items, npass, G, R, rng
        self.nl = {}
        for b in items:
            self.nl[b] = self.nl.get(b, 0) + 1
        self.done = {b: 0 for b in self.nl}
        self.abort = False
        self.ended = set()          # (pass, item) finished
        self.started = set()
        self.claim = 0
        self.arrive = 0
        self.closed_at = None

    # -- safety: an item of lattice b starts pass s only after every item of b ended pass s-1
    def check_start(self, s, it):
        b = self.items[it]
        if s > 0:
            for j, bj in enumerate(self.items):
                if bj == b:
                    assert (s - 1, j) in self.ended, (s, it, j)
        assert (s, it) not in self.started
        self.started.add((s, it))

    def wait(self, b, need):
        """Bounded poll of done[b] >= need; returns True to leave (abort)."""
        spins = 0
        while True:
            if self.done[b] >= need:          # acquire load
                return False
            if self.abort:
                return True
            spins += 1
            if spins > SPIN:
                self.abort = True             # raise the flag
                return True
            yield

    def item(self, s, it):
        self.check_start(s, it)
        yield                                 # the item's work (its stores)
        self.ended.add((s, it))
        self.done[self.items[it]] += 1        # release fetch_add
        yield

    CLOSED = 1 << 30

    def census(self):
        """Arrive, then wait until all G arrived; True to leave (census closed)."""
        old = self.arrive                     # atomic fetch_add
        self.arrive += 1
        yield
        if old & self.CLOSED:
            return True
        spins = 0
        while True:
            v = self.arrive                   # atomic load
            if v & self.CLOSED:
                return True
            if v >= self.G:
                return False
            spins += 1
            if spins > SPIN:
                if self.arrive == v:          # compare-and-swap v -> v | CLOSED
                    self.arrive = v | self.CLOSED
                    self.closed_at = v
                    return True
                spins = 0                     # someone arrived: wait again
            yield

    def round_robin(self, w, with_census=False):
        """The kernels' protocol: pass-major, items w, w + G, ... each pass."""
        if with_census:
            left = yield from self.census()
            if left:
                return "closed"
        for s in range(self.npass):
            for it in range(w, len(self.items), self.G):
                b = self.items[it]
                if s > 0:
                    left = yield from self.wait(b, s * self.nl[b])
                    if left:
                        return "aborted"
                yield from self.item(s, it)
        return "done"

    def queue(self, w):
        """Pass-major job queue: job j = (j // nitems, j % nitems), claimed in order."""
        n = len(self.items)
        while True:
            j = self.claim                    # atomic fetch_add on the claim counter
            self.claim += 1
            yield
            if j >= self.npass * n:
                return "done"
            s, it = divmod(j, n)
            b = self.items[it]
            if s > 0:
                left = yield from self.wait(b, s * self.nl[b])
                if left:
                    return "aborted"
            yield from self.item(s, it)

    def run(self, program, max_steps=10 ** 7):
        pending = list(range(self.G))         # dispatched in order as slots free up
        resident = {}
        results = {}
        steps = 0
        while pending or resident:
            while pending and len(resident) < self.R:
                w = pending.pop(0)
                resident[w] = program(w)
            w = self.rng.choice(sorted(resident))
            try:
                next(resident[w])
            except StopIteration as e:
                results[w] = e.value
                del resident[w]
            steps += 1
            if steps > max_steps:
                raise Deadlock("no workgroup left after %d steps" % steps)
        return results


@pytest.mark.parametrize("seed", range(40))
@pytest.mark.parametrize("npass", [1, 2, 5])
def test_round_robin_safe_and_live_when_co_resident(seed, npass):
    rng = random.Random(seed)
    items = layout(rng, rng.randint(1, 6), 5)
    G = rng.randint(1, len(items))            # the launcher caps the grid at the item count
    m = Machine(items, npass, G, R=G, rng=rng)
    res = m.run(m.round_robin)
    assert set(res.values()) == {"done"} and not m.abort
    assert m.ended == {(s, it) for s in range(npass) for it in range(len(items))}
    assert all(m.done[b] == npass * m.nl[b] for b in m.nl)


def test_round_robin_needs_co_residency_and_the_bound_ends_every_wait():
    # one lattice of two items on two workgroups with one resident slot: workgroup 0
    # waits in pass 1 for the lattice's other item, whose workgroup cannot start while
    # workgroup 0 holds the slot
    items = [0, 0]
    m = Machine(items, npass=2, G=2, R=1, rng=random.Random(0))
    res = m.run(m.round_robin)
    assert m.abort
    assert set(res) == {0, 1}                 # every workgroup left (none hangs)
    assert "aborted" in res.values()


@pytest.mark.parametrize("seed", range(30))
def test_round_robin_abort_under_partial_residency_always_terminates(seed):
    rng = random.Random(seed)
    items = layout(rng, rng.randint(2, 6), 4)
    G = len(items)
    R = rng.randint(1, max(1, G - 1))
    m = Machine(items, npass=3, G=G, R=R, rng=rng)
    res = m.run(m.round_robin)
    assert set(res) == set(range(G))          # all left: finished or aborted
    if not m.abort:
        assert set(res.values()) == {"done"}


@pytest.mark.parametrize("seed", range(30))
def test_pass_major_queue_is_live_for_any_residency(seed):
    rng = random.Random(1000 + seed)
    items = layout(rng, rng.randint(1, 6), 5)
    G = rng.randint(1, 2 * len(items))
    R = rng.randint(1, G)
    m = Machine(items, npass=4, G=G, R=R, rng=rng)
    res = m.run(m.queue)
    assert set(res.values()) == {"done"} and not m.abort
    assert m.ended == {(s, it) for s in range(4) for it in range(len(items))}


def test_model_catches_a_missing_wait():
    # planted mistake: a protocol that skips the wait must trip the safety check
    items = [0, 0, 1]
    m = Machine(items, npass=2, G=3, R=3, rng=random.Random(3))

    def no_wait(w):
        for s in range(m.npass):
            for it in range(w, len(items), m.G):
                yield from m.item(s, it)
        return "done"

    with pytest.raises(AssertionError):
        for seed in range(50):
            m = Machine(items, npass=2, G=3, R=3, rng=random.Random(seed))
            m.run(no_wait)


@pytest.mark.parametrize("seed", range(60))
def test_census_admits_only_a_co_resident_grid_and_the_retry_finishes(seed):
    rng = random.Random(5000 + seed)
    items = layout(rng, rng.randint(1, 6), 6)
    R = rng.randint(1, len(items))            # workgroups the device holds at once
    G = rng.randint(1, len(items))            # grid the host tries first
    tries = 0
    while True:
        tries += 1
        m = Machine(items, npass=3, G=G, R=R, rng=rng)
        res = m.run(lambda w: m.round_robin(w, with_census=True))
        if set(res.values()) == {"closed"}:
            # closed: every workgroup left before any item started, the state is untouched
            assert G > R and not m.started and m.closed_at is not None and m.closed_at <= R
            G = m.closed_at                   # the host's retry
            continue
        assert set(res.values()) == {"done"} and not m.abort and G <= R
        assert m.ended == {(s, it) for s in range(3) for it in range(len(items))}
        break
    assert tries <= 2
