"""Serving: a continuous-batching loop over the encoding path.

Requests (a symbol stream already in HBM, its alphabet, a chunk size) arrive
over time.  The loop keeps a FIFO queue; whenever one of its device streams
is idle it admits requests from the head of the queue for as long as the
HBM arena can hold each one's footprint (output bound, chunk offsets,
histogram, codebook and its share of the batch workspace) and launches them
together: requests with alphabets up to 8192 as one hf_encode_batch call,
larger alphabets as plain hf_histogram / hf_build_codebook / hf_encode calls
on the same stream.  Several batches are in flight at once on separate
streams, so requests that arrive while others run are admitted as soon as a
stream and memory free up, and their work overlaps on the device.  Results
(bitstream, offsets, codebook, histogram) stay in the arena, device
resident, until the request is released.

The queue, admission and arena logic are plain Python with no device calls
(`Arena`, `admit`, `ServeLoop`); the device work sits behind `GpuExecutor`.
"""
from __future__ import annotations

import bisect
import math
import time
from dataclasses import dataclass

ALIGN = 256
BATCH_MAX_ALPHABET = 8192
MAX_CODELEN = 64


def align(n: int) -> int:
    return (n + ALIGN - 1) // ALIGN * ALIGN


class Arena:
    """First-fit allocator of byte ranges in [0, capacity), 256-byte
    granular, with coalescing of adjacent free ranges."""

    def __init__(self, capacity: int):
        self.capacity = capacity // ALIGN * ALIGN
        self._free = [(0, self.capacity)]  # sorted (offset, size)
        self.used = 0

    def alloc(self, nbytes: int) -> int | None:
        size = align(max(1, nbytes))
        for i, (off, sz) in enumerate(self._free):
            if sz >= size:
                if sz == size:
                    del self._free[i]
                else:
                    self._free[i] = (off + size, sz - size)
                self.used += size
                return off
        return None

    def release(self, off: int, nbytes: int) -> None:
        size = align(max(1, nbytes))
        i = bisect.bisect_left(self._free, (off, 0))
        if i > 0:
            po, ps = self._free[i - 1]
            assert po + ps <= off, "double free or overlap"
        if i < len(self._free):
            assert off + size <= self._free[i][0], "double free or overlap"
        self._free.insert(i, (off, size))
        self.used -= size
        # merge with the right, then with the left neighbour
        if i + 1 < len(self._free) and off + size == self._free[i + 1][0]:
            self._free[i] = (off, size + self._free[i + 1][1])
            del self._free[i + 1]
        if i > 0 and self._free[i - 1][0] + self._free[i - 1][1] == off:
            po, ps = self._free[i - 1]
            self._free[i - 1] = (po, ps + self._free[i][1])
            del self._free[i]

    def largest_free(self) -> int:
        return max((sz for _, sz in self._free), default=0)

    def free_ranges(self):
        return list(self._free)


@dataclass(eq=False)
class Request:
    rid: int
    n: int
    sym_bytes: int
    alphabet: int
    arrival: float                # seconds from the start of the trace
    chunk: int = 4096
    r: int = 0
    sym: object = None            # device tensor (GPU executor only)
    # filled by the loop
    admitted: float | None = None
    done: float | None = None
    status: int | None = None
    region: tuple | None = None   # (offset, bytes) of the request's own buffers
    result: object = None

    @property
    def nbytes(self) -> int:
        return self.n * self.sym_bytes

    @property
    def batched(self) -> bool:
        return self.alphabet <= BATCH_MAX_ALPHABET

    @property
    def latency(self) -> float | None:
        return None if self.done is None else self.done - self.arrival


def admit(queue: list, free_slots: int, max_batch: int, reserve, solo=lambda r: False,
          max_batch_bytes: int | None = None) -> list:
    """Takes requests from the head of `queue` (FIFO, no overtaking) while
    `reserve(req)` succeeds, and only if a slot is free.  A request for
    which solo(req) holds is launched alone; otherwise consecutive
    non-solo requests are gathered, at most max_batch of them and, past the
    first, at most max_batch_bytes of input.  `reserve` returns False when
    the arena cannot hold the request now.  Returns the admitted requests
    (removed from the queue)."""
    if free_slots <= 0 or not queue:
        return []
    if solo(queue[0]):
        return [queue.pop(0)] if reserve(queue[0]) else []
    out, nbytes = [], 0
    while queue and len(out) < max_batch and not solo(queue[0]):
        r = queue[0]
        if out and max_batch_bytes is not None and nbytes + r.nbytes > max_batch_bytes:
            break
        if not reserve(r):
            break
        out.append(queue.pop(0))
        nbytes += r.nbytes
    return out


@dataclass(eq=False)
class Batch:
    requests: list
    slot: int
    ws: tuple | None              # (offset, bytes) of the batch workspace
    handle: object = None         # executor's completion handle


class ServeLoop:
    """The queue / admission / completion loop, independent of the device.

    executor.solo(req) -> True if the request is launched alone
    executor.footprint(req) -> own bytes (kept until release)
    executor.batch_bytes(reqs) -> shared workspace bytes of a batch
    executor.launch(batch) -> handle (asynchronous; batch.ws is its workspace range)
    executor.finished(handle) -> bool (non-blocking)
    executor.statuses(handle) -> list of per-request status codes
    """

    def __init__(self, executor, capacity: int, slots: int = 3, max_batch: int = 64,
                 keep_results: bool = False, max_batch_bytes: int | None = None):
        self.ex = executor
        self.max_batch_bytes = max_batch_bytes
        self.arena = Arena(capacity)
        self.slots = [None] * slots
        self.max_batch = max_batch
        self.keep_results = keep_results
        self.queue: list = []
        self.finished: list = []
        self.rejected: list = []
        self.max_busy = 0
        self.max_batch_seen = 0
        self.batches = 0

    # -- memory ------------------------------------------------------------
    def _fits_empty(self, req: Request) -> bool:
        return align(self.ex.footprint(req)) + align(self.ex.batch_bytes([req])) <= self.arena.capacity

    def _reserve(self, req: Request) -> bool:
        own = self.ex.footprint(req)
        off = self.arena.alloc(own)
        if off is None:
            return False
        req.region = (off, own)
        return True

    def release(self, req: Request) -> None:
        if req.region is not None:
            self.arena.release(*req.region)
            req.region = None
            req.result = None

    # -- loop --------------------------------------------------------------
    def submit(self, req: Request) -> None:
        if not self._fits_empty(req):
            req.status = -1  # can never fit
            self.rejected.append(req)
            return
        self.queue.append(req)

    def poll(self, now: float) -> list:
        """Collects finished batches; frees their workspaces (and the
        requests' own buffers unless results are kept)."""
        done = []
        for i, b in enumerate(self.slots):
            if b is not None and self.ex.finished(b.handle):
                for req, st in zip(b.requests, self.ex.statuses(b.handle)):
                    req.done = now
                    req.status = st
                    if not self.keep_results:
                        self.release(req)
                    done.append(req)
                self.arena.release(*b.ws)
                self.slots[i] = None
        self.finished.extend(done)
        return done

    def launch_ready(self, now: float) -> Batch | None:
        """Admits requests from the head of the queue into a free slot and
        launches them; the batch workspace is allocated after the requests'
        own buffers, and requests are handed back to the queue head, last
        first, until it fits."""
        free = [i for i, b in enumerate(self.slots) if b is None]
        if not free or not self.queue:
            return None
        reqs = admit(self.queue, len(free), self.max_batch, self._reserve, self.ex.solo, self.max_batch_bytes)
        ws = None
        while reqs:
            wsb = self.ex.batch_bytes(reqs)
            off = self.arena.alloc(wsb)
            if off is not None:
                ws = (off, wsb)
                break
            back = reqs.pop()
            self.release(back)
            self.queue.insert(0, back)
        if not reqs:
            return None
        for r in reqs:
            r.admitted = now
        b = Batch(reqs, free[0], ws)
        b.handle = self.ex.launch(b)
        self.slots[free[0]] = b
        self.max_busy = max(self.max_busy, sum(1 for x in self.slots if x is not None))
        self.max_batch_seen = max(self.max_batch_seen, len(reqs))
        self.batches += 1
        return b

    def idle(self) -> bool:
        return not self.queue and all(b is None for b in self.slots)

    def run(self, requests: list, clock, wait=None) -> list:
        """Serves `requests` (sorted by arrival) in real time on `clock`
        (seconds since the trace started).  `wait(dt)` may sleep while
        nothing can happen.  Returns the requests in completion order."""
        i = 0
        while i < len(requests) or not self.idle():
            now = clock()
            while i < len(requests) and requests[i].arrival <= now:
                self.submit(requests[i])
                i += 1
            self.poll(now)
            while self.launch_ready(now) is not None:
                pass
            if self.queue and all(b is None for b in self.slots):
                raise RuntimeError("the arena is full of kept results; release some before serving more")
            if wait is not None and i < len(requests) and self.idle():
                wait(max(0.0, requests[i].arrival - clock()))
        return self.finished


def percentile(xs, q: float) -> float:
    """q-th percentile (0..100) by the nearest-rank method."""
    if not xs:
        return float("nan")
    s = sorted(xs)
    k = max(1, math.ceil(q / 100.0 * len(s)))
    return s[k - 1]


# ---------------------------------------------------------------------------
# device executor
# ---------------------------------------------------------------------------
class _Carver:
    """Carves 256-byte aligned typed views out of the arena tensor."""

    def __init__(self, buf, off: int, nbytes: int):
        self.buf, self.pos, self.end = buf, off, off + nbytes

    def take(self, count: int, dtype):
        import torch

        size = torch.tensor([], dtype=dtype).element_size() * max(1, count)
        assert self.pos + size <= self.end, "region overflow"
        v = self.buf.narrow(0, self.pos, size).view(dtype)[:count]
        self.pos += align(size)
        return v


def own_bytes(n: int, A: int, chunk: int, batched: bool, bound_words: int, plain_ws: int,
              slab_words: int) -> int:
    """Bytes of one request's own buffers: output, offsets, histogram,
    codebook, status word (and, for the plain path, its workspace and
    per-slab counts)."""
    nch = (n + chunk - 1) // chunk
    parts = [4 * max(1, bound_words), 8 * (nch + 1), 4 * A,          # out, offsets, hist
             A, 8 * A, 8 * (MAX_CODELEN + 1), 4 * (MAX_CODELEN + 1),  # cl, cw, first, entry
             4 * A, 8 * 4, 4]                                         # rev, info, status
    if not batched:
        parts += [plain_ws, 4 * slab_words]
    return sum(align(max(1, p)) for p in parts)


@dataclass
class Result:
    out: object
    offsets: object
    hist: object
    book: object
    ws: object = None             # plain path only
    nslabs: int = 0
    slab_hist: object = None


class GpuExecutor:
    """Launches batches on `slots` HIP streams of the current device, with
    buffers carved from one preallocated arena tensor.  A batch's workspace
    region starts with one status word per request (in launch order: the
    batched requests first)."""

    def __init__(self, capacity: int, slots: int, max_batch: int, device="cuda", use_batch: bool = True,
                 solo_bytes: int = 32 << 20):
        import torch

        from . import hf

        assert max_batch * 4 <= ALIGN
        self.torch, self.hf = torch, hf
        self.use_batch = use_batch
        self.solo_bytes = solo_bytes
        self.buf = torch.empty(capacity, dtype=torch.uint8, device=device)
        self.streams = [torch.cuda.Stream(device=device) for _ in range(slots)]
        self.host_status = [torch.zeros(max_batch, dtype=torch.int32).pin_memory() for _ in range(slots)]
        self._ws_cache: dict = {}

    # sizes ---------------------------------------------------------------
    def solo(self, req: Request) -> bool:
        """Large requests (or large alphabets) fill the device by
        themselves: they run alone, with plain calls, on their own stream."""
        return not self.use_batch or not req.batched or req.nbytes >= self.solo_bytes

    def batched(self, req: Request) -> bool:
        """Whether the request goes through hf_encode_batch (else plain
        per-request calls)."""
        return not self.solo(req)

    def _single_desc_ws(self, req: Request) -> int:
        key = (req.n, req.sym_bytes, req.alphabet, req.chunk, req.r)
        v = self._ws_cache.get(key)
        if v is None:
            d = self.hf.hf_stream_desc()
            d.sym, d.n, d.sym_bytes, d.chunk_symbols, d.reduce_log2 = 0x1000, req.n, req.sym_bytes, req.chunk, req.r
            d.hist, d.out, d.out_capacity_words, d.chunk_bit_offsets = 0, 0x1000, 1, 0x1000
            b = self.hf.hf_codebook()
            b.alphabet = req.alphabet
            b.cl = b.cw = b.first = b.entry = b.rev = b.info = 0x1000
            d.book = b
            v = self.hf.hf_batch_workspace_bytes((self.hf.hf_stream_desc * 1)(d))
            assert v > 0, "invalid request for the batch path"
            self._ws_cache[key] = v
        return v

    def footprint(self, req: Request) -> int:
        hf = self.hf
        bw = hf.hf_bound_words(req.n, req.alphabet)
        b = self.batched(req)
        plain_ws = 0 if b else hf.hf_workspace_bytes(req.n, req.alphabet, req.chunk)
        slabs = 0 if b else hf.hf_slab_count(req.n, req.alphabet)
        return own_bytes(req.n, req.alphabet, req.chunk, b, bw, plain_ws, slabs * req.alphabet)

    def batch_bytes(self, reqs: list) -> int:
        return ALIGN + sum(align(self._single_desc_ws(r)) for r in reqs if self.batched(r))

    # launch --------------------------------------------------------------
    def _carve(self, req: Request) -> Result:
        torch, hf = self.torch, self.hf
        c = _Carver(self.buf, *req.region)
        A, n = req.alphabet, req.n
        out = c.take(max(1, hf.hf_bound_words(n, A)), torch.int32)
        offs = c.take((n + req.chunk - 1) // req.chunk + 1, torch.int64)
        hist = c.take(A, torch.int32)
        book = hf.Codebook(A, c.take(A, torch.uint8), c.take(A, torch.int64), c.take(MAX_CODELEN + 1, torch.int64),
                           c.take(MAX_CODELEN + 1, torch.int32), c.take(A, torch.int32), c.take(4, torch.int64))
        c.take(1, torch.int32)  # status word of the request (kept for layout stability)
        res = Result(out, offs, hist, book)
        if not self.batched(req):
            res.ws = c.take(hf.hf_workspace_bytes(n, A, req.chunk), torch.uint8)
            res.nslabs = hf.hf_slab_count(n, A)
            res.slab_hist = c.take(res.nslabs * A, torch.int32) if res.nslabs else None
        return res

    def launch(self, batch: Batch):
        torch, hf = self.torch, self.hf
        st = self.streams[batch.slot]
        hs = self.host_status[batch.slot]
        small = [r for r in batch.requests if self.batched(r)]
        large = [r for r in batch.requests if not self.batched(r)]
        order = small + large
        cws = _Carver(self.buf, *batch.ws)
        status = cws.take(len(order), torch.int32)
        with torch.cuda.stream(st):
            status.zero_()
            for r in order:
                r.result = self._carve(r)
            if small:
                descs = (hf.hf_stream_desc * len(small))()
                for k, r in enumerate(small):
                    d, res = descs[k], r.result
                    d.sym, d.n, d.sym_bytes = (hf._dptr(r.sym) if r.n else 0), r.n, r.sym_bytes
                    d.chunk_symbols, d.reduce_log2, d.reserved = r.chunk, r.r, 0
                    d.hist = hf._dptr(res.hist)
                    d.book = res.book.struct()
                    d.out, d.out_capacity_words = hf._dptr(res.out), res.out.numel()
                    d.chunk_bit_offsets = hf._dptr(res.offsets)
                ws = cws.take(batch.ws[1] - ALIGN, torch.uint8)
                hf.hf_encode_batch(descs, ws, status[:len(small)])
            for k, r in enumerate(large):
                res, stk = r.result, status[len(small) + k:len(small) + k + 1]
                hf.hf_histogram(r.sym, r.alphabet, res.hist, res.nslabs, res.slab_hist, res.ws, stk)
                hf.hf_build_codebook(res.hist, res.book, res.ws, stk)
                hf.hf_encode(r.sym, res.book, r.chunk, r.r, res.out, res.offsets, res.ws, stk,
                             res.nslabs, res.slab_hist)
            hs[:len(order)].copy_(status, non_blocking=True)
            ev = torch.cuda.Event()
            ev.record(st)
        # statuses come back in launch order; report them in batch order
        pos = {id(r): k for k, r in enumerate(order)}
        return (ev, [pos[id(r)] for r in batch.requests], hs)

    def finished(self, handle) -> bool:
        return handle[0].query()

    def statuses(self, handle) -> list:
        ev, idx, hs = handle
        vals = hs.tolist()
        return [int(vals[k]) for k in idx]


def serve(requests: list, capacity: int, slots: int = 8, max_batch: int = 32, keep_results: bool = False,
          device="cuda", use_batch: bool = True, solo_bytes: int = 32 << 20, max_batch_bytes: int = 64 << 20):
    """Serves `requests` (sorted by arrival, each with .sym on the device)
    in real time; returns the ServeLoop (finished requests with their
    latencies, results when kept).  use_batch=False, slots=1, max_batch=1
    is the one-request-at-a-time server with plain launches."""
    ex = GpuExecutor(capacity, slots, max_batch, device, use_batch, solo_bytes)
    loop = ServeLoop(ex, capacity, slots, max_batch, keep_results, max_batch_bytes)
    t0 = time.perf_counter()
    loop.run(requests, clock=lambda: time.perf_counter() - t0)
    return loop
