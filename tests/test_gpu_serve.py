"""Served encoding on the GPU: every request's result (histogram, codebook,
bitstream, offsets) is identical whether it is encoded alone or in the mix
of overlapping batches, and equal to the oracle's."""
import time

import numpy as np
import pytest

import oracle
from paper_2010_10039_amd import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2010_10039_amd import hf  # noqa: E402
from paper_2010_10039_amd import serve as S  # noqa: E402


def _requests(nreq, seed, qps, min_bytes, max_bytes):
    trace = W.served_requests(nreq, seed=seed, qps=qps, min_bytes=min_bytes, max_bytes=max_bytes, device="cuda")
    reqs = []
    for i, (t, x, A, kind) in enumerate(trace):
        reqs.append(S.Request(i, x.numel(), x.element_size(), A, t, chunk=4096, sym=x))
    torch.cuda.synchronize()
    return reqs


def _alone(req):
    """The request encoded by itself with plain calls."""
    e = hf.Encoder(req.n, req.alphabet, req.chunk, req.r)
    e.run(req.sym)
    torch.cuda.synchronize()
    hf.raise_on_status(e.status, "alone")
    return e


def test_served_mix_equals_alone_and_oracle():
    reqs = _requests(36, seed=2000, qps=40_000.0, min_bytes=2.0 ** 16, max_bytes=2.0 ** 23)
    loop = S.serve(reqs, capacity=2 << 30, slots=3, max_batch=8, keep_results=True)
    torch.cuda.synchronize()
    assert len(loop.finished) == len(reqs) and not loop.rejected
    assert loop.max_busy > 1, "batches should overlap on the device"
    assert loop.max_batch_seen > 1, "requests should share a batch"
    assert any(r.alphabet > S.BATCH_MAX_ALPHABET for r in reqs)
    for r in reqs:
        assert r.status == 0, (r.rid, r.status)
        res = r.result
        e = _alone(r)
        nbits = int(e.offsets[-1].item())
        nw = (nbits + 31) // 32
        assert torch.equal(res.hist, e.hist), r.rid
        for f in ("cl", "cw", "first", "entry", "info"):
            assert torch.equal(getattr(res.book, f), getattr(e.book, f)), (r.rid, f)
        assert torch.equal(res.offsets, e.offsets), r.rid
        assert torch.equal(res.out[:nw], e.out[:nw]), r.rid
        # and the oracle
        x = r.sym.cpu().numpy()
        x = x.view(np.uint16) if x.dtype == np.int16 else x
        ref = oracle.codebook(oracle.histogram(x, r.alphabet))
        words, offs, tb = oracle.encode(x, ref, r.chunk)
        assert tb == nbits, r.rid
        assert np.array_equal(res.offsets.cpu().numpy().view(np.uint64), offs), r.rid
        assert np.array_equal(res.out[:nw].cpu().numpy().view(np.uint32), words[:nw]), r.rid
        loop.release(r)
    assert loop.arena.used == 0


def test_served_latencies_are_recorded():
    reqs = _requests(12, seed=3000, qps=2000.0, min_bytes=2.0 ** 16, max_bytes=2.0 ** 22)
    t0 = time.perf_counter()
    loop = S.serve(reqs, capacity=1 << 30, slots=2, max_batch=4)
    wall = time.perf_counter() - t0
    lat = [r.latency for r in loop.finished]
    assert len(lat) == 12 and all(0 < v < wall for v in lat)
    assert all(r.status == 0 for r in loop.finished)
    assert loop.arena.used == 0


def test_served_mix_with_solo_and_512MiB_requests():
    """Small batched requests mixed with requests of at least 32 MiB (which
    the loop launches alone) and one of 512 MiB: each result equals the same
    request encoded alone and the oracle's stream."""
    small = _requests(12, seed=4000, qps=20_000.0, min_bytes=2.0 ** 16, max_bytes=2.0 ** 22)
    big = _requests(3, seed=4100, qps=20_000.0, min_bytes=2.0 ** 25, max_bytes=2.0 ** 26)
    huge = _requests(1, seed=4200, qps=20_000.0, min_bytes=2.0 ** 29, max_bytes=2.0 ** 29)
    reqs = sorted(small + big + huge, key=lambda r: r.arrival)
    for i, r in enumerate(reqs):
        r.rid = i
    assert sum(r.nbytes >= 32 << 20 for r in reqs) >= 4 and max(r.nbytes for r in reqs) >= (512 << 20) - 2
    loop = S.serve(reqs, capacity=6 << 30, slots=4, max_batch=8, keep_results=True)
    torch.cuda.synchronize()
    assert len(loop.finished) == len(reqs) and not loop.rejected
    for r in reqs:
        assert r.status == 0, (r.rid, r.status)
        res = r.result
        e = _alone(r)
        nbits = int(e.offsets[-1].item())
        nw = (nbits + 31) // 32
        assert torch.equal(res.hist, e.hist), r.rid
        assert torch.equal(res.offsets, e.offsets), r.rid
        assert torch.equal(res.out[:nw], e.out[:nw]), r.rid
        x = r.sym.cpu().numpy()
        x = x.view(np.uint16) if x.dtype == np.int16 else x
        ref = oracle.codebook(oracle.histogram(x, r.alphabet))
        words, offs, tb = oracle.encode(x, ref, r.chunk)
        assert tb == nbits, r.rid
        assert np.array_equal(res.offsets.cpu().numpy().view(np.uint64), offs), r.rid
        assert np.array_equal(res.out[:nw].cpu().numpy().view(np.uint32), words[:nw]), r.rid
        del e
        loop.release(r)
    assert loop.arena.used == 0
