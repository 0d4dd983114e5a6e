"""Pins of the paper-format oracle (oracle/paper_format.py).

- A worked example derived by hand from the format's definition (below).
- With no breaking group, every chunk's bits equal the dense stream's bits
  for that chunk, as the independent serial C oracle writes them.
- Round trips through the format's own decoder, with breaking groups and
  short last groups, and the breaking count against group sums.
"""
import numpy as np
import pytest

import oracle
from oracle import paper_format as pf


def test_hand_worked_example():
    # codes: 0 -> "0", 1 -> "10", 2 -> "11" + 18 zeros (20 bits)
    cl = np.array([1, 2, 20], dtype=np.uint8)
    cw = np.array([0b0, 0b10, 0b11 << 18], dtype=np.uint64)
    x = np.array([2, 2, 0, 1, 0, 0, 1, 2], dtype=np.uint16)
    words, offs, brk, bsyms = pf.encode(x, cl, cw, M=2, r=1)
    # chunk 0: group (2, 2) has 40 bits -> breaking group 0; group (0, 1) -> "010"
    # chunk 1: group (0, 0) -> "00"; group (1, 2) -> "10" + 20 bits -> 24 bits "001011" + 18 zeros
    assert list(words) == [0b010 << 29, 0b001011 << 26]
    assert list(offs) == [0, 1, 2]
    assert list(brk) == [0] and list(bsyms) == [2, 2]


def _bits(words, lo, hi):
    s = "".join(f"{int(w):032b}" for w in words)
    return s[lo:hi]


@pytest.mark.parametrize("M,r,spread", [(8, 1, 0), (10, 2, 16), (12, 3, 8), (10, 3, 5)])
def test_matches_dense_stream_without_breaking(M, r, spread):
    rng = np.random.default_rng(M + r)
    if spread:  # few symbols: short codes, no group can pass 32 bits
        x = (500 + rng.integers(0, spread, 70_001)).astype(np.uint16)
    else:
        x = np.clip(np.rint(rng.normal(512, 1.5, 70_001)), 0, 1023).astype(np.uint16)
    book = oracle.codebook(oracle.histogram(x, 1024))
    assert int(book.cl.max()) << r <= 32  # no group can break
    words, offs, brk, _ = pf.encode(x, book.cl, book.cw, M, r)
    assert brk.size == 0
    dw, doffs, total = oracle.encode(x, book, 1 << M)
    for k in range(offs.size - 1):
        nbits = int(doffs[k + 1] - doffs[k])
        assert _bits(words[int(offs[k]):int(offs[k + 1])], 0, nbits) == _bits(dw, int(doffs[k]), int(doffs[k + 1]))
        assert int(offs[k + 1] - offs[k]) == (nbits + 31) // 32


@pytest.mark.parametrize("M,r,n", [(8, 2, 5000), (10, 3, 20_011), (9, 4, 7777), (10, 5, 3000)])
def test_round_trip_with_breaking(M, r, n):
    rng = np.random.default_rng(n)
    x = np.clip(np.rint(rng.normal(512, 40, n)), 0, 1023).astype(np.uint16)
    book = oracle.codebook(oracle.histogram(x, 1024))
    words, offs, brk, bsyms = pf.encode(x, book.cl, book.cw, M, r)
    G = 1 << r
    pad = (-n) % G
    sums = np.concatenate([book.cl[x].astype(np.int64), np.zeros(pad, np.int64)]).reshape(-1, G).sum(axis=1)
    assert brk.size == int((sums > 32).sum()) and brk.size > 0
    assert np.array_equal(brk, np.flatnonzero(sums > 32).astype(np.uint64))
    got = pf.decode(words, offs, brk, bsyms, n, book.cl, book.cw, M, r, np.uint16)
    assert np.array_equal(got, x)
