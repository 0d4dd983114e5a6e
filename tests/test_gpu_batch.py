"""Parity of batched encoding (hf_encode_batch) with the CPU oracle.

Every stream of a batch must come out exactly as the oracle encodes it
alone: histogram, book, every output word and every chunk offset, whatever
the other streams are (sizes, widths, alphabets, reduction factors)."""
import os

import numpy as np
import pytest

import oracle
from paper_2010_10039_amd import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2010_10039_amd import hf  # noqa: E402

SENTINEL = 0x5A5A5A5A


def _np(t: torch.Tensor) -> np.ndarray:
    a = t.cpu().numpy()
    return a.view(np.uint16) if a.dtype == np.int16 else a


def _dev(x: np.ndarray) -> torch.Tensor:
    return torch.from_numpy(x.view(np.int16) if x.dtype == np.uint16 else x).cuda()


def run_batch(xs, alphabets, chunks=4096, rs=0):
    syms = [_dev(x) for x in xs]
    enc = hf.BatchEncoder(syms, alphabets, chunks, rs)
    for o in enc.outs:
        o.fill_(SENTINEL)
    for f in enc.offsets:
        f.fill_(-1)
    enc.run()
    torch.cuda.synchronize()
    return enc


def check_stream(enc, i, x, A, chunk):
    ref_h = oracle.histogram(x, A)
    assert np.array_equal(enc.hists[i].cpu().numpy().view(np.uint32), ref_h), i
    ref = oracle.codebook(ref_h)
    book = enc.books[i]
    assert np.array_equal(book.info.cpu().numpy().view(np.uint64), ref.info), i
    assert np.array_equal(book.cl.cpu().numpy(), ref.cl), i
    assert np.array_equal(book.cw.cpu().numpy().view(np.uint64), ref.cw), i
    assert np.array_equal(book.first.cpu().numpy().view(np.uint64), ref.first), i
    assert np.array_equal(book.entry.cpu().numpy().view(np.uint32), ref.entry), i
    assert np.array_equal(book.rev.cpu().numpy().view(np.uint32)[:ref.m], ref.rev[:ref.m]), i
    words, offs, tb = oracle.encode(x, ref, chunk)
    nw = (tb + 31) // 32
    got = enc.outs[i].cpu().numpy().view(np.uint32)
    assert np.array_equal(enc.offsets[i].cpu().numpy().view(np.uint64), offs), i
    assert np.array_equal(got[:nw], words[:nw]), i
    assert np.all(got[nw:] == SENTINEL), i


def _fib_stream(m, seed):
    f = [1, 1]
    while len(f) < m:
        f.append(f[-1] + f[-2])
    x = np.repeat(np.arange(m, dtype=np.uint16), f[:m])
    np.random.default_rng(seed).shuffle(x)
    return x


def test_batch_mixed_streams():
    """Uneven sizes (log-uniform), u8 and u16, alphabets 256..8192, and the
    edge streams: empty, one symbol, one distinct symbol, ragged tails, a
    33-bit longest code (the wide path) and a 29-bit one (LDS buffer path)."""
    syms, alph = W.batched_streams(20, seed=1000, min_log2=10, max_log2=20)
    xs = [_np(t) for t in syms]
    xs += [np.zeros(0, np.uint16), np.array([7], np.uint8), np.full(70_001, 3, np.uint16),
           _fib_stream(34, 1), _fib_stream(30, 2)]
    alph += [1024, 256, 4096, 64, 8192]
    rng = np.random.default_rng(5)
    xs.append(np.clip(np.rint(rng.normal(4000, 900, 262_145)), 0, 8191).astype(np.uint16))
    alph.append(8192)
    enc = run_batch(xs, alph)
    assert np.all(enc.status.cpu().numpy() == 0)
    for i, (x, A) in enumerate(zip(xs, alph)):
        check_stream(enc, i, x, A, 4096)


@pytest.mark.parametrize("r", [3, 4, 5])
def test_batch_reduction_factors_and_chunks(r):
    rng = np.random.default_rng(r)
    xs, alph, chunks, rs = [], [], [], []
    for k, (n, A, chunk) in enumerate([(300_007, 1024, 256), (1_000_001, 256, 4096), (65_537, 4096, 65536),
                                       (4096 * 40, 1024, 1024)]):
        dt = np.uint8 if A <= 256 else np.uint16
        xs.append(np.clip(np.rint(rng.normal(A / 2, 3 + 10 * k, n)), 0, A - 1).astype(dt))
        alph.append(A)
        chunks.append(chunk)
        rs.append(r if k % 2 == 0 else 0)
    enc = run_batch(xs, alph, chunks, rs)
    assert np.all(enc.status.cpu().numpy() == 0)
    for i, (x, A) in enumerate(zip(xs, alph)):
        check_stream(enc, i, x, A, chunks[i])


def test_batch_equals_single_stream_path():
    """The batch's words and offsets equal hf_encode's for each stream."""
    syms, alph = W.batched_streams(6, seed=77, min_log2=14, max_log2=21)
    xs = [_np(t) for t in syms]
    enc = run_batch(xs, alph)
    for i, (x, A) in enumerate(zip(xs, alph)):
        d = _dev(x)
        ws = hf.new_workspace(x.size, A)
        status = hf.new_status()
        hist = hf.hf_histogram(d, A, ws=ws, status=status)
        book = hf.hf_build_codebook(hist, ws=ws, status=status)
        out = torch.empty(hf.hf_bound_words(x.size, A), dtype=torch.int32, device="cuda")
        offs = torch.empty((x.size + 4095) // 4096 + 1, dtype=torch.int64, device="cuda")
        hf.hf_encode(d, book, 4096, 0, out, offs, ws, status)
        assert hf.read_status(status) == 0
        nw = (int(offs[-1].item()) + 31) // 32
        assert torch.equal(enc.offsets[i], offs)
        assert torch.equal(enc.outs[i][:nw], out[:nw])


def test_batch_errors_stay_per_stream():
    """A stream with a symbol outside its alphabet, and one with too small an
    output buffer, fail alone; their neighbours are untouched."""
    rng = np.random.default_rng(9)
    good = [np.clip(np.rint(rng.normal(512, 20, 200_003)), 0, 1023).astype(np.uint16) for _ in range(3)]
    bad_sym = good[0].copy()
    bad_sym[123_456] = 1500
    small = good[1].copy()
    xs = [good[0], bad_sym, good[1], small, good[2]]
    alph = [1024] * 5
    syms = [_dev(x) for x in xs]
    enc = hf.BatchEncoder(syms, alph, 4096, 0)
    enc.descs[3].out_capacity_words = 100
    for o in enc.outs:
        o.fill_(SENTINEL)
    enc.run()
    st = enc.status.cpu().numpy()
    assert st[1] == hf.HF_ERR_SYMBOL
    assert st[3] == hf.HF_ERR_CAPACITY
    assert st[0] == st[2] == st[4] == 0
    for i in (0, 2, 4):
        check_stream(enc, i, xs[i], 1024, 4096)


def test_batch_repeat_is_deterministic():
    syms, alph = W.batched_streams(8, seed=31, min_log2=12, max_log2=19)
    xs = [_np(t) for t in syms]
    enc = run_batch(xs, alph)
    first = [o.clone() for o in enc.outs]
    enc.run()
    enc.run()
    torch.cuda.synchronize()
    for a, b in zip(first, enc.outs):
        assert torch.equal(a, b)


def test_batch_full_size_sample():
    """A 64-stream batch at full per-stream sizes (up to 2^26 symbols),
    compared with the oracle on every 8th stream."""
    syms, alph = W.batched_streams(64, seed=1000, device="cuda")
    enc = hf.BatchEncoder(syms, alph, 4096, 0)
    for o in enc.outs:
        o.fill_(SENTINEL)
    enc.run()
    torch.cuda.synchronize()
    assert np.all(enc.status.cpu().numpy() == 0)
    for i in range(0, 64, 8):
        check_stream(enc, i, _np(syms[i]), alph[i], 4096)


def test_batch_full_512_streams():
    """The whole batched workload: 512 streams of 2^16 to 2^26 symbols with
    the autotuner's chunk size and reduction factor per stream, every 4th
    stream compared with the oracle (the others decode back to their input)."""
    from paper_2010_10039_amd import autotune

    syms, alph = W.batched_streams(512, seed=1000, device="cuda")
    tuner = autotune.Autotuner.load(os.path.join(os.path.dirname(autotune.__file__), "tuning_mi355x.json"))
    picks = [tuner.choose(t.element_size(), A, None) for t, A in zip(syms, alph)]
    enc = hf.BatchEncoder(syms, alph, [c.chunk for c in picks], [c.r for c in picks])
    for o in enc.outs:
        o.fill_(SENTINEL)
    enc.run()
    torch.cuda.synchronize()
    assert np.all(enc.status.cpu().numpy() == 0)
    for i in range(0, 512, 4):
        check_stream(enc, i, _np(syms[i]), alph[i], picks[i].chunk)
    for i in range(512):
        if i % 4 and syms[i].numel():
            r = hf.hf_decode_check(enc.outs[i], enc.offsets[i], syms[i], picks[i].chunk, enc.books[i])
            assert r.cpu().tolist() == [0, syms[i].numel()], i
