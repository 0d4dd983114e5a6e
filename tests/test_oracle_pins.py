"""Pins of the CPU oracle to facts that do not come from the oracle itself.

Each test checks the oracle against something the paper, a published
standard or plain mathematics fixes: brute-force optimality, Huffman
closed forms, Shannon bounds, Kraft equality, the RFC 1951 worked example,
bit-string concatenation written out independently, and decoding with an
independent code-table walk.  A plausible mistake anywhere in the oracle (a
dropped term, a wrong index or sign, a transposed operand, a wrong tie
order) fails at least one of these.
"""
import heapq
import itertools
import math
import os
import random

import numpy as np
import pytest

import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _read_golden(name):
    rows, notes = [], []
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if not line:
                continue
            if line.startswith("#"):
                notes.append(line)
                continue
            s, l, c = line.split()
            rows.append((int(s), int(l), c))
    return rows, notes


def _cost(h, cl):
    return int(np.dot(np.asarray(h, dtype=np.int64), np.asarray(cl, dtype=np.int64)))


def _kraft_complete(cl):
    """sum 2^-l == 1, in exact integer arithmetic."""
    used = [int(l) for l in cl if l > 0]
    L = max(used)
    return sum(1 << (L - l) for l in used) == (1 << L)


# --------------------------------------------------------------------------
# Histogram (Sec. 4.1): reduces to numpy's bincount.
# --------------------------------------------------------------------------
@pytest.mark.parametrize("dtype,A", [(np.uint8, 256), (np.uint16, 1024), (np.uint16, 65536)])
def test_histogram_is_bincount(dtype, A):
    rng = np.random.default_rng(3)
    x = rng.integers(0, A, size=100_003).astype(dtype)
    h = oracle.histogram(x, A)
    assert np.array_equal(h, np.bincount(x, minlength=A).astype(np.uint32))


def test_histogram_rejects_symbol_outside_alphabet():
    x = np.array([0, 5, 1023, 1024], dtype=np.uint16)
    with pytest.raises(oracle.OracleError) as e:
        oracle.histogram(x, 1024)
    assert e.value.code == oracle.ERR_SYMBOL


# --------------------------------------------------------------------------
# Code lengths: optimality and the exact tie order, by brute force.
# --------------------------------------------------------------------------
def _brute_force_candidates(hu):
    """All length vectors for weights hu that are (1) Kraft-complete and
    optimal, (2) of minimum maximum length, (3) of minimum total length, and
    (4) non-increasing along the (weight, symbol) order.  Enumerates length
    multisets; for a fixed multiset the optimal assignment is the monotone one
    (rearrangement inequality), so no optimal vector is missed."""
    m = len(hu)
    order = sorted(range(m), key=lambda s: (hu[s], s))
    best = None
    pool = []
    for ms in itertools.combinations_with_replacement(range(1, m), m):
        K = m - 1
        if sum(1 << (K - l) for l in ms) != (1 << K):
            continue
        lengths = sorted(ms, reverse=True)  # longest to lightest
        vec = [0] * m
        for r, s in enumerate(order):
            vec[s] = lengths[r]
        c = _cost(hu, vec)
        if best is None or c < best:
            best, pool = c, [vec]
        elif c == best:
            pool.append(vec)
    mx = min(max(v) for v in pool)
    pool = [v for v in pool if max(v) == mx]
    sm = min(sum(v) for v in pool)
    return best, [v for v in pool if sum(v) == sm]


def test_lengths_unique_min_variance_optimum_brute_force():
    """Huffman's code is optimal; with leaf-first ties (Sec. 4.2.1's 'combine
    everything lighter than the two smallest' order) it is also the
    minimum-maximum, minimum-total-length optimal code, and equal weights get
    non-increasing lengths in symbol order.  Brute force finds exactly one
    such vector on every tie-heavy tiny histogram; the oracle must return it."""
    rng = random.Random(11)
    for _ in range(400):
        m = rng.randint(2, 9)
        hu = [rng.choice([1, 1, 2, 2, 3, 4, 5, 8, 13]) for _ in range(m)]
        pad = rng.randint(0, 3)  # unused symbols interleaved
        h = []
        slots = []
        for v in hu:
            h.append(v)
            slots.append(len(h) - 1)
            for _ in range(rng.randint(0, pad)):
                h.append(0)
        cl, wsum = oracle.code_lengths(np.array(h, dtype=np.uint32))
        best, cands = _brute_force_candidates(hu)
        assert len(cands) == 1
        got = [int(cl[s]) for s in slots]
        assert got == cands[0], (hu, got, cands)
        assert _cost(hu, got) == best == wsum
        assert all(cl[i] == 0 for i in range(len(h)) if h[i] == 0)


def _textbook_huffman_cost(h):
    """Sum of merged weights of the textbook algorithm (any tie order)."""
    heap = [int(v) for v in h if v > 0]
    if len(heap) == 1:
        return heap[0]
    heapq.heapify(heap)
    cost = 0
    while len(heap) > 1:
        a = heapq.heappop(heap)
        b = heapq.heappop(heap)
        cost += a + b
        heapq.heappush(heap, a + b)
    return cost


def test_cost_matches_textbook_huffman_and_internal_weights():
    rng = np.random.default_rng(5)
    for trial in range(200):
        A = int(rng.integers(2, 400))
        kind = trial % 3
        if kind == 0:
            h = rng.integers(0, 50, size=A)
        elif kind == 1:
            h = rng.geometric(0.05, size=A) * (rng.random(A) < 0.7)
        else:
            h = np.rint(1e5 * np.exp(-0.5 * ((np.arange(A) - A / 2) / max(1.0, A / 20)) ** 2))
        h = h.astype(np.uint32)
        if h.sum() == 0:
            h[0] = 1
        cl, wsum = oracle.code_lengths(h)
        assert _cost(h, cl) == wsum == _textbook_huffman_cost(h)


# --------------------------------------------------------------------------
# Closed forms.
# --------------------------------------------------------------------------
@pytest.mark.parametrize("k", [1, 2, 5, 10])
def test_uniform_power_of_two(k):
    cl, _ = oracle.code_lengths(np.full(1 << k, 7, dtype=np.uint32))
    assert np.all(cl == k)


def test_dyadic_probabilities_give_minus_log2():
    # p_s = 2^-l_s with lengths 1,2,3,4,5,6,6
    lengths = [1, 2, 3, 4, 5, 6, 6]
    h = np.array([1 << (6 - l) for l in lengths], dtype=np.uint32)
    perm = np.random.default_rng(1).permutation(len(h))
    cl, _ = oracle.code_lengths(h[perm])
    assert list(cl) == [lengths[p] for p in perm]


@pytest.mark.parametrize("m", [3, 10, 25, 40])
def test_fibonacci_weights(m):
    """Weights F_1..F_m give lengths (m-1, m-1, m-2, ..., 1): the deepest
    possible tree; m = 40 yields 39-bit codes."""
    fib = [1, 1]
    while len(fib) < m:
        fib.append(fib[-1] + fib[-2])
    h = np.array(fib[:m], dtype=np.uint32)
    cl, _ = oracle.code_lengths(h)
    expect = [m - 1] + [m - i for i in range(1, m)]
    assert list(cl) == expect


def test_degenerate_alphabets():
    cl, w = oracle.code_lengths(np.zeros(16, dtype=np.uint32))
    assert not cl.any() and w == 0
    h = np.zeros(16, dtype=np.uint32)
    h[9] = 100
    cl, w = oracle.code_lengths(h)
    assert cl[9] == 1 and cl.sum() == 1 and w == 100
    h[3] = 1
    cl, _ = oracle.code_lengths(h)
    assert cl[3] == 1 and cl[9] == 1 and cl.sum() == 2


def test_shannon_bounds():
    rng = np.random.default_rng(9)
    for _ in range(100):
        A = int(rng.integers(2, 2000))
        h = rng.integers(0, 1000, size=A).astype(np.uint32)
        h[int(rng.integers(0, A))] += 1
        if np.count_nonzero(h) < 2:
            h[(int(np.flatnonzero(h)[0]) + 1) % A] = 1
        b = oracle.codebook(h)
        n = int(h.sum())
        p = h[h > 0] / n
        H = float(-(p * np.log2(p)).sum())
        beta = b.total_bits / n
        assert H - 1e-12 <= beta < H + 1


# --------------------------------------------------------------------------
# Canonical codes (Sec. 4.2.2).
# --------------------------------------------------------------------------
def _bits(code, l):
    return format(int(code), f"0{l}b") if l else ""


def test_canonical_matches_rfc1951_complement():
    """Per length, the ones-first code set is the bitwise complement of the
    RFC 1951 canonical code set (codes built in reverse per level, then
    inverted, Algorithm 1 / Sec. 4.2.2); within a length codes ascend with
    the symbol id."""
    rfc, _ = _read_golden("rfc1951_canonical_example.txt")
    cl = np.array([l for _, l, _ in rfc], dtype=np.uint8)
    b = oracle.canonical(cl)
    for l in sorted(set(cl.tolist())):
        ours = {_bits(b.cw[s], l) for s, ll, _ in rfc if ll == l}
        comp = {"".join("1" if ch == "0" else "0" for ch in c) for _, ll, c in rfc if ll == l}
        assert ours == comp
    hand, _ = _read_golden("ones_first_canonical_example.txt")
    for s, l, c in hand:
        assert int(cl[s]) == l and _bits(b.cw[s], l) == c
    assert list(b.first[1:5]) == [2, 3, 1, 0]
    assert list(b.entry[1:6]) == [0, 0, 1, 6, 8]
    assert list(b.rev[:8]) == [5, 0, 1, 2, 3, 4, 6, 7]
    assert list(b.info) == [8, 4, 0, 2]


def test_hand_encoded_stream():
    hand, _ = _read_golden("ones_first_canonical_example.txt")
    cl = np.array([l for _, l, _ in hand], dtype=np.uint8)
    b = oracle.canonical(cl)
    out, off, tb = oracle.encode(np.array([5, 0, 7], dtype=np.uint16), b, chunk=2)
    assert tb == 9 and list(out) == [0xC8800000] and list(off) == [0, 5, 9]


def _prefix_free(codes):
    s = sorted(codes)
    return all(not s[i + 1].startswith(s[i]) for i in range(len(s) - 1))


def test_kraft_prefix_free_and_monotone_on_random_books():
    rng = np.random.default_rng(17)
    for trial in range(150):
        A = int(rng.integers(2, 3000))
        h = (rng.pareto(1.2, size=A) * 10).astype(np.uint32) * (rng.random(A) < 0.8)
        if np.count_nonzero(h) < 2:
            h[:2] = [1, 2]
        h = h.astype(np.uint32)
        b = oracle.codebook(h)
        used = np.flatnonzero(b.cl)
        assert _kraft_complete(b.cl)
        codes = [_bits(b.cw[s], b.cl[s]) for s in used]
        assert _prefix_free(codes)
        # lengths non-increasing along the (weight, symbol) order
        order = sorted(used, key=lambda s: (h[s], s))
        assert all(b.cl[order[i]] >= b.cl[order[i + 1]] for i in range(len(order) - 1))
        # ones-first: every l-bit prefix of a longer code is < first[l]
        for s in used:
            for l in range(1, int(b.cl[s])):
                assert (int(b.cw[s]) >> (int(b.cl[s]) - l)) < int(b.first[l])
        # rev lists symbols by (length, symbol)
        want = sorted(used, key=lambda s: (b.cl[s], s))
        assert list(b.rev[: b.m]) == want


# --------------------------------------------------------------------------
# Bitstream (Sec. 4.3, Merge) and chunk offsets (Table 1).
# --------------------------------------------------------------------------
def _pack_string(bitstr):
    bitstr = bitstr + "0" * (-len(bitstr) % 32)
    return np.array([int(bitstr[i:i + 32], 2) for i in range(0, len(bitstr), 32)], dtype=np.uint32)


@pytest.mark.parametrize("seed,A,n,chunk", [(0, 1024, 5000, 256), (1, 256, 7777, 1024),
                                            (2, 37, 3001, 512), (3, 1024, 1, 256)])
def test_encode_equals_string_concatenation(seed, A, n, chunk):
    rng = np.random.default_rng(seed)
    x = np.clip(np.rint(rng.normal(A / 2, A / 30, size=n)), 0, A - 1).astype(np.uint16)
    b = oracle.codebook(oracle.histogram(x, A))
    out, off, tb = oracle.encode(x, b, chunk)
    s = "".join(_bits(b.cw[v], b.cl[v]) for v in x)
    assert tb == len(s) == b.total_bits
    assert np.array_equal(out, _pack_string(s))
    per = [int(b.cl[x[i:i + chunk]].astype(np.int64).sum()) for i in range(0, n, chunk)]
    assert list(off) == [0] + list(np.cumsum(per))


def test_decode_roundtrip_and_independent_table_walk():
    rng = np.random.default_rng(4)
    x = rng.zipf(1.3, size=20000).clip(1, 255).astype(np.uint8)
    b = oracle.codebook(oracle.histogram(x, 256))
    out, off, tb = oracle.encode(x, b, 1024)
    dec, end = oracle.decode(out, tb, x.size, b, dtype=np.uint8)
    assert end == tb and np.array_equal(dec, x)
    # independent decoder: walk the bits against a code -> symbol dictionary
    table = {_bits(b.cw[s], b.cl[s]): s for s in np.flatnonzero(b.cl)}
    bits = "".join(format(int(w), "032b") for w in out)[:tb]
    got, cur = [], ""
    for ch in bits:
        cur += ch
        if cur in table:
            got.append(table[cur])
            cur = ""
    assert cur == "" and np.array_equal(np.array(got, dtype=np.uint8), x)
    # restart at every chunk offset
    for k in range(len(off) - 1):
        lo, hi = k * 1024, min(x.size, (k + 1) * 1024)
        d, e = oracle.decode(out, tb, hi - lo, b, dtype=np.uint8, start=int(off[k]))
        assert e == off[k + 1] and np.array_equal(d, x[lo:hi])


def test_decode_rejects_invalid_code():
    h = np.zeros(8, dtype=np.uint32)
    h[2] = 10
    b = oracle.codebook(h)  # single symbol: code "0"; bit 1 is not a code
    with pytest.raises(oracle.OracleError):
        oracle.decode(np.array([0x80000000], dtype=np.uint32), 32, 1, b)


def test_bitstream_independent_of_chunk_size():
    x = np.random.default_rng(8).integers(0, 300, size=50_000).astype(np.uint16)
    b = oracle.codebook(oracle.histogram(x, 300))
    ref, ref_off, ref_tb = oracle.encode(x, b, 256)
    for c in (512, 1024, 4096, 65536):
        out, off, tb = oracle.encode(x, b, c)
        assert tb == ref_tb and np.array_equal(out, ref)
        assert np.array_equal(off[:-1], ref_off[:-1:c // 256]) and off[-1] == ref_tb


def test_long_codes_over_32_bits_roundtrip():
    fib = [1, 1]
    while len(fib) < 40:
        fib.append(fib[-1] + fib[-2])
    h = np.array(fib, dtype=np.uint32)
    b = oracle.codebook(h)
    assert b.lmax == 39
    x = np.array([0, 1, 39, 2, 0, 38, 1, 1, 0], dtype=np.uint16)
    out, off, tb = oracle.encode(x, b, 256)
    assert tb == int(b.cl[x].astype(np.int64).sum())
    dec, _ = oracle.decode(out, tb, x.size, b)
    assert np.array_equal(dec, x)
    s = "".join(_bits(b.cw[v], b.cl[v]) for v in x)
    assert np.array_equal(out, _pack_string(s))


def test_encode_rejects_symbol_without_code():
    h = np.array([3, 0, 5], dtype=np.uint32)
    b = oracle.codebook(h)
    with pytest.raises(oracle.OracleError) as e:
        oracle.encode(np.array([0, 1], dtype=np.uint16), b, 256)
    assert e.value.code == oracle.ERR_SYMBOL


def test_canonical_incomplete_lengths_stay_prefix_free():
    """The First construction (ceil of half the next level's slots) keeps an
    incomplete length set (Kraft sum < 1) prefix-free and decodable; rounding
    down instead would make the 1-bit code a prefix of the 2-bit one."""
    for lengths in ([1, 2], [2, 3, 3, 3], [1, 3, 3, 4], [3, 3, 3, 3, 5, 5, 5]):
        cl = np.array(lengths, dtype=np.uint8)
        b = oracle.canonical(cl)
        codes = [_bits(b.cw[s], cl[s]) for s in range(len(lengths))]
        assert _prefix_free(codes), (lengths, codes)
        x = np.arange(len(lengths), dtype=np.uint16).repeat(3)
        out, _, tb = oracle.encode(x, b, 256)
        dec, _ = oracle.decode(out, tb, x.size, b)
        assert np.array_equal(dec, x)
