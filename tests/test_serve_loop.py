"""The serving loop's host logic on the CPU: the arena allocator against a
brute-force model, FIFO admission, the continuous-batching loop with a fake
executor and a fake clock (slots, memory, rollback, rejection, latencies)."""
import random

import pytest

from paper_2010_10039_amd import serve as S


# ---------------------------------------------------------------------------
# arena
# ---------------------------------------------------------------------------
def test_arena_matches_bitmap_model():
    rng = random.Random(3)
    cap = 256 * 400
    a = S.Arena(cap)
    used = [False] * (cap // 256)
    live = []
    for _ in range(3000):
        if live and rng.random() < 0.45:
            off, nb = live.pop(rng.randrange(len(live)))
            a.release(off, nb)
            for u in range(off // 256, (off + S.align(nb)) // 256):
                assert used[u]
                used[u] = False
        else:
            nb = rng.randint(1, 256 * 20)
            units = S.align(nb) // 256
            off = a.alloc(nb)
            # first fit: the lowest run of free units long enough
            want = None
            run = 0
            for u, b in enumerate(used):
                run = 0 if b else run + 1
                if run == units:
                    want = (u - units + 1) * 256
                    break
            assert off == want
            if off is not None:
                for u in range(off // 256, off // 256 + units):
                    used[u] = True
                live.append((off, nb))
        assert a.used == 256 * sum(used)
        # free list is sorted, disjoint and fully coalesced
        fr = a.free_ranges()
        for (o1, s1), (o2, s2) in zip(fr, fr[1:]):
            assert o1 + s1 < o2
    for off, nb in live:
        a.release(off, nb)
    assert a.free_ranges() == [(0, cap)] and a.used == 0


def test_arena_double_free_is_caught():
    a = S.Arena(4096)
    off = a.alloc(300)
    a.release(off, 300)
    with pytest.raises(AssertionError):
        a.release(off, 300)


class _R:
    def __init__(self, name, nbytes=1):
        self.name, self.nbytes = name, nbytes

    def __repr__(self):
        return self.name


def test_admit_is_fifo_without_overtaking():
    q = [_R("big"), _R("small"), _R("small2")]
    got = S.admit(q, 1, 8, lambda r: r.name != "big")
    assert got == [] and [r.name for r in q] == ["big", "small", "small2"]
    got = S.admit(q, 1, 2, lambda r: True)
    assert [r.name for r in got] == ["big", "small"] and [r.name for r in q] == ["small2"]
    assert S.admit(q, 0, 8, lambda r: True) == []


def test_admit_runs_solo_requests_alone_and_caps_batch_bytes():
    class R:
        def __init__(self, name, nbytes, solo=False):
            self.name, self.nbytes, self.is_solo = name, nbytes, solo

    q = [R("a", 10), R("b", 10), R("big", 10, True), R("c", 10)]
    solo = lambda r: r.is_solo  # noqa: E731
    got = S.admit(q, 1, 8, lambda r: True, solo)
    assert [r.name for r in got] == ["a", "b"]  # stops before the solo one
    got = S.admit(q, 1, 8, lambda r: True, solo)
    assert [r.name for r in got] == ["big"]
    q = [R("x", 60), R("y", 30), R("z", 10), R("w", 5)]
    got = S.admit(q, 1, 8, lambda r: True, solo, max_batch_bytes=100)
    assert [r.name for r in got] == ["x", "y", "z"]
    q = [R("huge", 500), R("t", 1)]
    got = S.admit(q, 1, 8, lambda r: True, solo, max_batch_bytes=100)
    assert [r.name for r in got] == ["huge"]  # the first always goes


def test_percentile_nearest_rank():
    xs = list(range(1, 101))
    assert S.percentile(xs, 50) == 50 and S.percentile(xs, 99) == 99 and S.percentile(xs, 100) == 100
    assert S.percentile([7.0], 99) == 7.0


# ---------------------------------------------------------------------------
# loop with a fake executor
# ---------------------------------------------------------------------------
class FakeClock:
    def __init__(self, step=1e-5):
        self.t, self.step = 0.0, step

    def __call__(self):
        self.t += self.step
        return self.t


class FakeExecutor:
    """A batch takes overhead + bytes / rate seconds on its slot; several
    slots run at once.  Records every launch and checks that no two live
    buffers overlap."""

    def __init__(self, clock, rate=1e9, overhead=2e-5, ws_per_req=1024):
        self.clock, self.rate, self.overhead, self.ws_per_req = clock, rate, overhead, ws_per_req
        self.launches = []
        self.max_inflight = 0
        self.inflight = set()

    def solo(self, req):
        return not req.batched

    def footprint(self, req):
        return req.nbytes // 2 + 1000

    def batch_bytes(self, reqs):
        return 256 + self.ws_per_req * sum(1 for r in reqs if r.batched)

    def launch(self, batch):
        ranges = [r.region for r in batch.requests] + [batch.ws]
        for b in self.inflight:
            ranges += [r.region for r in b.requests] + [b.ws]
        spans = sorted((o, o + S.align(n)) for o, n in ranges)
        for (a0, a1), (b0, b1) in zip(spans, spans[1:]):
            assert a1 <= b0, "overlapping live buffers"
        end = self.clock.t + self.overhead + sum(r.nbytes for r in batch.requests) / self.rate
        self.launches.append((self.clock.t, [r.rid for r in batch.requests]))
        self.inflight.add(batch)
        self.max_inflight = max(self.max_inflight, len(self.inflight))
        return (end, batch)

    def finished(self, handle):
        if self.clock.t >= handle[0]:
            self.inflight.discard(handle[1])
            return True
        return False

    def statuses(self, handle):
        return [0] * len(handle[1].requests)


def _trace(nreq, seed, qps, min_b=10_000, max_b=2_000_000, big_alphabet_every=0):
    rng = random.Random(seed)
    t, reqs = 0.0, []
    for i in range(nreq):
        t += rng.expovariate(qps)
        sb = rng.choice([1, 2])
        nbytes = int(min_b * (max_b / min_b) ** rng.random())
        A = 65536 if big_alphabet_every and i % big_alphabet_every == 0 and sb == 2 else (256 if sb == 1 else 1024)
        reqs.append(S.Request(i, nbytes // sb, sb, A, t))
    return reqs


@pytest.mark.parametrize("slots,max_batch,cap", [(1, 1, 1 << 24), (3, 16, 1 << 24), (2, 64, 3 << 20)])
def test_loop_serves_everything_in_order(slots, max_batch, cap):
    clock = FakeClock()
    ex = FakeExecutor(clock)
    loop = S.ServeLoop(ex, cap, slots, max_batch)
    reqs = _trace(200, slots * 7 + max_batch, qps=4000, big_alphabet_every=5)
    done = loop.run(reqs, clock)
    assert len(done) == 200 and not loop.rejected
    assert all(r.status == 0 and r.done >= r.admitted >= r.arrival for r in done)
    # FIFO: admission order is arrival order
    admitted = [rid for _, ids in ex.launches for rid in ids]
    assert admitted == sorted(admitted)
    assert all(len(ids) <= max_batch for _, ids in ex.launches)
    assert ex.max_inflight <= slots
    assert loop.arena.used == 0 and loop.arena.free_ranges() == [(0, loop.arena.capacity)]


def test_loop_batches_when_arrivals_overlap():
    """Arrivals faster than service: later batches hold several requests."""
    clock = FakeClock()
    ex = FakeExecutor(clock, rate=2e8)
    loop = S.ServeLoop(ex, 1 << 26, 2, 32)
    loop.run(_trace(100, 1, qps=50_000), clock)
    assert max(len(ids) for _, ids in ex.launches) > 4
    assert len(ex.launches) < 100


def test_loop_rolls_back_when_workspace_does_not_fit():
    """Own buffers fit but the batch workspace does not: the last admitted
    requests go back to the head of the queue, in order, and run later."""
    clock = FakeClock()
    ex = FakeExecutor(clock, ws_per_req=200_000)
    reqs = [S.Request(i, 400_000, 1, 256, 1e-6 * i) for i in range(6)]
    # each own region ~201 KB; capacity holds about 4 of them plus little room
    loop = S.ServeLoop(ex, 1_100_000, 1, 8)
    done = loop.run(reqs, clock)
    assert [r.rid for r in done] == list(range(6))
    sizes = [len(ids) for _, ids in ex.launches]
    assert max(sizes) < 6 and sum(sizes) == 6
    assert loop.arena.used == 0


def test_loop_rejects_a_request_that_can_never_fit():
    clock = FakeClock()
    ex = FakeExecutor(clock)
    reqs = [S.Request(0, 10_000_000, 2, 1024, 0.0), S.Request(1, 1000, 1, 256, 0.0)]
    loop = S.ServeLoop(ex, 1 << 20, 2, 8)
    done = loop.run(reqs, clock)
    assert [r.rid for r in done] == [1]
    assert [r.rid for r in loop.rejected] == [0] and loop.rejected[0].status == -1


def test_kept_results_that_fill_the_arena_raise():
    clock = FakeClock()
    ex = FakeExecutor(clock)
    reqs = [S.Request(i, 600_000, 1, 256, 0.0) for i in range(4)]
    loop = S.ServeLoop(ex, 1_000_000, 1, 1, keep_results=True)
    with pytest.raises(RuntimeError, match="kept results"):
        loop.run(reqs, clock)
    assert len(loop.finished) == 3  # three 301000-byte results fill the 1 MB arena
