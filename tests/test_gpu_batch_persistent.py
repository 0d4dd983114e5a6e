"""Parity of the persistent batched launch (hf_encode_batch_persistent): one
kernel that takes every stage of every stream from a device work queue.

Every stream must come out exactly as the oracle encodes it alone, and
exactly as the staged batch (hf_encode_batch, one launch per stage) encodes
it: histogram, book, every output word and every chunk offset."""
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

pytest.skip("hf_encode_batch_persistent is switched off: its kernel's first run made a GPU memory fault "
            "(test_persistent_mixed_streams) whose cause is not found yet; it returns HF_ERR_LAUNCH",
            allow_module_level=True)

SENTINEL = 0x5A5A5A5A


def _np(t: torch.Tensor) -> np.ndarray:
    a = t.cpu().numpy()
    return a.view(np.uint16) if a.dtype == np.int16 else a


def _dev(x: np.ndarray) -> torch.Tensor:
    return torch.from_numpy(x.view(np.int16) if x.dtype == np.uint16 else x).cuda()


def run(syms, alphabets, chunks=4096, rs=0, persistent=True):
    enc = hf.BatchEncoder(syms, alphabets, chunks, rs)
    for o in enc.outs:
        o.fill_(SENTINEL)
    for f in enc.offsets:
        f.fill_(-1)
    enc.run(persistent=persistent)
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


def assert_same(a, b):
    """Two batch encoders hold identical results for every stream."""
    for i in range(len(a.outs)):
        assert torch.equal(a.outs[i], b.outs[i]), i
        assert torch.equal(a.offsets[i], b.offsets[i]), i
        assert torch.equal(a.hists[i], b.hists[i]), i
        for f in ("cl", "cw", "first", "entry", "info"):
            assert torch.equal(getattr(a.books[i], f), getattr(b.books[i], f)), (i, f)


def _fib_stream(m, seed):
    f = [1, 1]
    while len(f) < m:
        f.append(f[-1] + f[-2])
    x = np.repeat(np.arange(m, dtype=np.uint16), f[:m])
    np.random.default_rng(seed).shuffle(x)
    return x


def test_persistent_mixed_streams():
    """Uneven sizes, u8 and u16, alphabets 64..8192, and the edge streams:
    empty, one symbol, one distinct symbol, a 33-bit longest code (wide
    path), a 29-bit one, books above the launch's 1024-symbol LDS tree."""
    syms, alph = W.batched_streams(20, seed=1000, min_log2=10, max_log2=20)
    xs = [_np(t) for t in syms]
    xs += [np.zeros(0, np.uint16), np.array([7], np.uint8), np.full(70_001, 3, np.uint16),
           _fib_stream(34, 1), _fib_stream(30, 2)]
    alph += [1024, 256, 4096, 64, 8192]
    rng = np.random.default_rng(5)
    xs.append(np.clip(np.rint(rng.normal(4000, 900, 262_145)), 0, 8191).astype(np.uint16))
    alph.append(8192)
    xs.append(rng.integers(0, 3000, 400_003).astype(np.uint16))  # ~3000 used: tree in the workspace
    alph.append(4096)
    enc = run([_dev(x) for x in xs], alph)
    assert np.all(enc.status.cpu().numpy() == 0)
    for i, (x, A) in enumerate(zip(xs, alph)):
        check_stream(enc, i, x, A, 4096)


@pytest.mark.parametrize("r", [3, 4, 5])
def test_persistent_reduction_factors_and_chunks(r):
    rng = np.random.default_rng(r)
    xs, alph, chunks, rs = [], [], [], []
    for k, (n, A, chunk) in enumerate([(300_007, 1024, 256), (1_000_001, 256, 4096), (65_537, 4096, 65536),
                                       (4096 * 40, 1024, 1024), (2_000_003, 8192, 16384)]):
        dt = np.uint8 if A <= 256 else np.uint16
        xs.append(np.clip(np.rint(rng.normal(A / 2, 3 + 10 * k, n)), 0, A - 1).astype(dt))
        alph.append(A)
        chunks.append(chunk)
        rs.append(r if k % 2 == 0 else 0)
    enc = run([_dev(x) for x in xs], alph, chunks, rs)
    assert np.all(enc.status.cpu().numpy() == 0)
    for i, (x, A) in enumerate(zip(xs, alph)):
        check_stream(enc, i, x, A, chunks[i])


def test_persistent_errors_stay_per_stream():
    """A stream with a symbol outside its alphabet and one with too small an
    output buffer fail alone; their neighbours are untouched."""
    rng = np.random.default_rng(9)
    good = [np.clip(np.rint(rng.normal(512, 20, 200_003)), 0, 1023).astype(np.uint16) for _ in range(3)]
    bad_sym = good[0].copy()
    bad_sym[123_456] = 1500
    xs = [good[0], bad_sym, good[1], good[1].copy(), good[2]]
    enc = hf.BatchEncoder([_dev(x) for x in xs], [1024] * 5, 4096, 0)
    enc.descs[3].out_capacity_words = 100
    for o in enc.outs:
        o.fill_(SENTINEL)
    enc.run(persistent=True)
    st = enc.status.cpu().numpy()
    assert st[1] == hf.HF_ERR_SYMBOL
    assert st[3] == hf.HF_ERR_CAPACITY
    assert st[0] == st[2] == st[4] == 0
    for i in (0, 2, 4):
        check_stream(enc, i, xs[i], 1024, 4096)


def test_persistent_equals_staged_and_repeats():
    """64 streams of 2^12 to 2^22 symbols: the persistent launch, twice in a
    row on the same workspace, equals the staged launches bit for bit."""
    syms, alph = W.batched_streams(64, seed=4242, min_log2=12, max_log2=22, device="cuda")
    staged = run(syms, alph, persistent=False)
    fused = run(syms, alph, persistent=True)
    assert np.all(fused.status.cpu().numpy() == 0)
    assert_same(staged, fused)
    fused.run(persistent=True)
    torch.cuda.synchronize()
    assert_same(staged, fused)


def test_persistent_full_512_streams():
    """The whole batched workload (512 streams of 2^16 to 2^26 symbols, the
    autotuner's chunk size and reduction factor per stream) in one launch:
    every stream equals the staged batch, every 16th equals the oracle."""
    from paper_2010_10039_amd import autotune

    syms, alph = W.batched_streams(512, seed=1000, device="cuda")
    tuner = autotune.Autotuner.load(os.path.join(os.path.dirname(autotune.__file__), "tuning_mi355x.json"))
    picks = [tuner.choose(t.element_size(), A, None) for t, A in zip(syms, alph)]
    chunks, rs = [c.chunk for c in picks], [c.r for c in picks]
    fused = run(syms, alph, chunks, rs, persistent=True)
    assert np.all(fused.status.cpu().numpy() == 0)
    staged = run(syms, alph, chunks, rs, persistent=False)
    assert_same(staged, fused)
    for i in range(0, 512, 16):
        check_stream(fused, i, _np(syms[i]), alph[i], picks[i].chunk)
