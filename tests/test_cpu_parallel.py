"""The multi-core CPU baseline (libhf_cpu: thread-parallel histogram,
parallel codebook, chunk-parallel encoder) against the oracle.

The baseline is measured beside the GPU path; here it must give exactly the
oracle's histogram, codebook (lengths, codewords, First, Entry, reverse
book, info) and bitstream, for any number of threads.  Histograms cover
tie-heavy counts, exact Fibonacci counts (codes longer than 32 bits), one
and two used symbols, an empty book, and alphabets up to 65536 with rounds
long enough to take the parallel merge.
"""
import numpy as np
import pytest

import oracle
from paper_2010_10039_amd import workloads as W

hfc = pytest.importorskip("paper_2010_10039_amd.hf_cpu")


def _fib(k):
    f = [1, 1]
    while len(f) < k:
        f.append(f[-1] + f[-2])
    return f[:k]


_HISTS = []


def _hists():
    if _HISTS:
        return _HISTS
    rng = np.random.default_rng(123)
    out = []
    for A in (1, 2, 3, 7, 64, 256, 1024):
        out.append(rng.integers(0, 5, size=A).astype(np.uint32))          # tie-heavy, with zeros
        out.append(rng.integers(1, 1 << 20, size=A).astype(np.uint32))
    h = np.zeros(1024, dtype=np.uint32)
    h[[3, 500, 1000]] = [5, 5, 5]
    out.append(h)
    h = np.zeros(300, dtype=np.uint32)
    h[17] = 99                                                              # one used symbol
    out.append(h)
    out.append(np.zeros(40, dtype=np.uint32))                               # none
    f = np.zeros(64, dtype=np.uint32)
    f[5:5 + 40] = _fib(40)                                                  # 39-bit codes
    out.append(f)
    for A, kind in ((4096, "normal"), (16384, "normal"), (65536, "normal"), (65536, "uniform")):
        out.append(W.skewed_histogram(A, 1 << 24, seed=A % 7, kind=kind))
    z = (1e9 / np.arange(1, 65537) ** 1.2).astype(np.uint32)               # many long rounds
    out.append(z)
    _HISTS.extend(out)
    return _HISTS


def _same_book(got, ref):
    m = ref.m
    assert np.array_equal(got["cl"], ref.cl)
    assert np.array_equal(got["cw"], ref.cw)
    assert np.array_equal(got["first"], ref.first)
    assert np.array_equal(got["entry"], ref.entry)
    assert np.array_equal(got["rev"][:m], ref.rev[:m])
    assert np.array_equal(got["info"], ref.info)


@pytest.mark.parametrize("nthreads", [1, 2, 3, 8])
def test_codebook_equals_oracle(nthreads):
    for h in _hists():
        _same_book(hfc.codebook(h, nthreads), oracle.codebook(h))


@pytest.mark.parametrize("nthreads", [1, 4, 7])
@pytest.mark.parametrize("dtype,A", [(np.uint16, 1024), (np.uint8, 256), (np.uint16, 65536)])
def test_histogram_equals_oracle(nthreads, dtype, A):
    x = W.gaussian_codes(n=1_000_003, alphabet=A, mean=A / 2, sigma=A / 40, seed=1, dtype=dtype)
    assert np.array_equal(hfc.histogram(x, A, nthreads), oracle.histogram(x, A))
    with pytest.raises(hfc.HFCError) as e:  # a symbol outside the alphabet
        hfc.histogram(x, int(x.max()), nthreads)
    assert e.value.code == 16


@pytest.mark.parametrize("nthreads", [1, 3, 8])
@pytest.mark.parametrize("chunk", [256, 4096, 65536])
def test_encode_equals_oracle(nthreads, chunk):
    for dtype, A, sigma, n in ((np.uint16, 1024, 6.0, 777_777), (np.uint8, 256, 30.0, 300_001),
                               (np.uint16, 1024, 2.0, 5)):
        x = W.gaussian_codes(n=n, alphabet=A, mean=A / 2, sigma=sigma, seed=2, dtype=dtype)
        ref = oracle.codebook(oracle.histogram(x, A))
        words, offs, tb = oracle.encode(x, ref, chunk)
        g_words, g_offs, g_tb = hfc.encode(x, ref.cl, ref.cw, chunk, nthreads=nthreads)
        assert g_tb == tb
        assert np.array_equal(g_offs, offs)
        assert np.array_equal(g_words, words)


def test_encode_long_codes_and_errors():
    # Fibonacci counts give codes of up to 33 bits
    f = np.array(_fib(34), dtype=np.uint64)
    x = np.repeat(np.arange(34, dtype=np.uint16), np.minimum(f, 3000).astype(np.int64))
    h = np.zeros(64, dtype=np.uint32)
    h[:34] = _fib(34)
    book = oracle.codebook(h)
    assert book.lmax == 33
    rng = np.random.default_rng(4)
    rng.shuffle(x)
    words, offs, tb = oracle.encode(x, book, 256)
    g_words, g_offs, g_tb = hfc.encode(x, book.cl, book.cw, 256, nthreads=5)
    assert g_tb == tb and np.array_equal(g_offs, offs) and np.array_equal(g_words, words)
    # a symbol without a code, a symbol outside the alphabet, too little room
    y = x.copy()
    y[100] = 40
    with pytest.raises(hfc.HFCError) as e:
        hfc.encode(y, book.cl, book.cw, 256)
    assert e.value.code == 16
    y[100] = 64
    with pytest.raises(hfc.HFCError) as e:
        hfc.encode(y, book.cl, book.cw, 256)
    assert e.value.code == 16
    with pytest.raises(hfc.HFCError) as e:
        hfc.encode(x, book.cl, book.cw, 256, cap_words=(tb + 31) // 32 - 1)
    assert e.value.code == 17


def test_empty_stream():
    x = np.zeros(0, dtype=np.uint16)
    cl = np.zeros(8, dtype=np.uint8)
    words, offs, tb = hfc.encode(x, cl, np.zeros(8, dtype=np.uint64), 1024)
    assert tb == 0 and offs.tolist() == [0]
