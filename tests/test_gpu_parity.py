"""Parity of the HIP path (through the C ABI) with the CPU oracle.

All of this is integer work, so every comparison is bit-exact: histogram
bins, code lengths, codewords, First/Entry/rev tables, info, every output
word and every chunk offset.  Inputs are seeded; sizes span many tiles with
ragged tails; the full-size workloads are compared whole (the oracle
finishes them in seconds)."""
import functools

import numpy as np
import pytest

import oracle
from paper_2010_10039_amd import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2010_10039_amd import hf  # noqa: E402  (raises if libhf.so is missing)

SENTINEL = 0x5A5A5A5A


def _dev(x: np.ndarray) -> torch.Tensor:
    if x.dtype == np.uint16:
        return torch.from_numpy(x.view(np.int16)).cuda()
    return torch.from_numpy(x).cuda()


def _u64(t):
    return t.cpu().numpy().view(np.uint64)


def _u32(t):
    return t.cpu().numpy().view(np.uint32)


def slab_ranges(n: int, nslabs: int):
    """Slab g covers 4096-symbol blocks [g*nb/S, (g+1)*nb/S) (include/hf.h)."""
    nb = (n + 4095) // 4096
    cut = [min(n, (g * nb // nslabs) * 4096) for g in range(nslabs + 1)]
    return list(zip(cut[:-1], cut[1:]))


def gpu_hist(x: np.ndarray, A: int, offset: int = 0, nslabs: int = 0):
    """Histogram of x on the GPU; `offset` > 0 places x at a misaligned
    address inside a larger buffer; nslabs > 0 also returns per-slab counts."""
    buf = np.zeros(x.size + offset, dtype=x.dtype)
    buf[offset:] = x
    d = _dev(buf)[offset:]
    status = hf.new_status()
    sh = torch.full((max(1, nslabs) * A,), -1, dtype=torch.int32, device="cuda") if nslabs else None
    h = hf.hf_histogram(d, A, nslabs=nslabs, slab_hist=sh, status=status)
    assert hf.read_status(status) == 0
    h = h.cpu().numpy().view(np.uint32)
    if nslabs:
        return h, sh.cpu().numpy().view(np.uint32).reshape(nslabs, A)
    return h


def gpu_book(h: np.ndarray):
    A = h.size
    hd = torch.from_numpy(h.view(np.int32)).cuda()
    ws = hf.new_workspace(1, A)
    status = hf.new_status()
    book = hf.hf_build_codebook(hd, ws=ws, status=status)
    code = hf.read_status(status)
    return book, code


def assert_book_equal(book, ref: oracle.Codebook):
    m = ref.m
    assert np.array_equal(_u64(book.info), ref.info)
    assert np.array_equal(book.cl.cpu().numpy(), ref.cl)
    assert np.array_equal(_u64(book.cw), ref.cw)
    assert np.array_equal(_u64(book.first), ref.first)
    assert np.array_equal(_u32(book.entry), ref.entry)
    assert np.array_equal(_u32(book.rev)[:m], ref.rev[:m])


def gpu_encode(x: np.ndarray, book, chunk: int, r: int = 0, cap_words: int | None = None,
               nslabs: int = 0, slab_hist: np.ndarray | None = None):
    d = _dev(x)
    n = x.size
    cap = cap_words if cap_words is not None else hf.hf_bound_words(n, book.alphabet)
    out = torch.full((cap + 64,), SENTINEL, dtype=torch.int32, device="cuda")
    nch = (n + chunk - 1) // chunk
    offsets = torch.full((nch + 1,), -1, dtype=torch.int64, device="cuda")
    ws = hf.new_workspace(n, book.alphabet, chunk)
    status = hf.new_status()
    sh = None if slab_hist is None else torch.from_numpy(slab_hist.reshape(-1).view(np.int32)).cuda()
    hf.hf_encode(d, book, chunk, r, out[:cap], offsets, ws, status, nslabs=nslabs, slab_hist=sh)
    code = hf.read_status(status)
    return _u32(out), _u64(offsets), code


def check_pipeline(x: np.ndarray, A: int, chunk: int, r: int = 0, slab_counts=None):
    """GPU histogram (with per-slab counts when the alphabet allows),
    codebook, and encoding both from those counts and without them, each
    compared with the oracle."""
    ref_h = oracle.histogram(x, A)
    nslabs = hf.hf_slab_count(x.size, A)
    if nslabs:
        h, sh = gpu_hist(x, A, nslabs=nslabs)
        for g, (lo, hi) in enumerate(slab_ranges(x.size, nslabs)):
            assert np.array_equal(sh[g], oracle.histogram(x[lo:hi], A)), g
    else:
        h, sh = gpu_hist(x, A), None
    assert np.array_equal(h, ref_h)
    ref = oracle.codebook(ref_h)
    book, code = gpu_book(h)
    assert code == 0
    assert_book_equal(book, ref)
    ref_words, ref_offs, tb = oracle.encode(x, ref, chunk)
    nw = (tb + 31) // 32
    variants = [(nslabs, sh)] if nslabs else []
    nb = (x.size + 4095) // 4096
    for s in (slab_counts or [0, 1, min(3, nb), min(nb, 16384)]):
        variants.append((s, None))
    for s, part in variants:
        words, offs, code = gpu_encode(x, book, chunk, r, nslabs=s, slab_hist=part)
        assert code == 0
        assert np.array_equal(offs, ref_offs), (s, part is not None)
        assert np.array_equal(words[:nw], ref_words[:nw]), (s, part is not None)
        assert np.all(words[nw:] == SENTINEL)  # nothing written past the stream
    return book, words, offs, tb


# ---------------------------------------------------------------------------
# histogram
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("n,A,dtype,offset", [
    (1, 16, np.uint16, 0), (7, 256, np.uint8, 3), (1000, 1024, np.uint16, 1),
    (1_000_003, 1024, np.uint16, 0), (2_000_001, 256, np.uint8, 5),
    (300_001, 65536, np.uint16, 0), (300_001, 20000, np.uint16, 2), (0, 64, np.uint16, 0)])
def test_histogram_parity(n, A, dtype, offset):
    rng = np.random.default_rng(n + A)
    x = np.clip(np.rint(rng.normal(A / 2, max(1.0, A / 16), size=n)), 0, A - 1).astype(dtype)
    assert np.array_equal(gpu_hist(x, A, offset), oracle.histogram(x, A))


@pytest.mark.parametrize("n,nslabs", [(1, 1), (4097, 2), (1_000_003, 7), (1_000_003, 245), (3 << 20, 768)])
def test_histogram_slab_counts(n, nslabs):
    rng = np.random.default_rng(n)
    x = np.clip(np.rint(rng.normal(512, 30, size=n)), 0, 1023).astype(np.uint16)
    h, sh = gpu_hist(x, 1024, nslabs=nslabs)
    assert np.array_equal(h, oracle.histogram(x, 1024))
    for g, (lo, hi) in enumerate(slab_ranges(n, nslabs)):
        assert np.array_equal(sh[g], oracle.histogram(x[lo:hi], 1024)), g


@pytest.mark.parametrize("n,A,dtype", [(1, 16, np.uint16), (1_000_003, 1024, np.uint16),
                                       (2_000_001, 256, np.uint8), (300_001, 4096, np.uint16),
                                       (300_001, 8192, np.uint16)])
def test_histogram_with_workspace(n, A, dtype):
    """With a workspace (and no per-slab buffer of the caller's) the counts
    per slab go to the workspace and are reduced there; above 4096 symbols
    the global atomics path is used."""
    rng = np.random.default_rng(n + A + 7)
    x = np.clip(np.rint(rng.normal(A / 2, max(1.0, A / 20), size=n)), 0, A - 1).astype(dtype)
    d = _dev(x)
    ws = hf.new_workspace(n, A)
    status = hf.new_status()
    h = hf.hf_histogram(d, A, ws=ws, status=status)
    assert hf.read_status(status) == 0
    assert np.array_equal(h.cpu().numpy().view(np.uint32), oracle.histogram(x, A))


def test_histogram_peaked_single_bin():
    x = np.full(3_000_017, 511, dtype=np.uint16)
    x[::1000] = 3
    assert np.array_equal(gpu_hist(x, 1024), oracle.histogram(x, 1024))


def test_histogram_flags_out_of_range_symbol():
    x = np.zeros(100_000, dtype=np.uint16)
    x[77_777] = 1024
    d = _dev(x)
    status = hf.new_status()
    hf.hf_histogram(d, 1024, status=status)
    assert hf.read_status(status) == hf.HF_ERR_SYMBOL


# ---------------------------------------------------------------------------
# codebook
# ---------------------------------------------------------------------------
def _fib(m):
    f = [1, 1]
    while len(f) < m:
        f.append(f[-1] + f[-2])
    return f[:m]


def _hist_cases():
    rng = np.random.default_rng(123)
    cases = {}
    cases["empty"] = np.zeros(64, np.uint32)
    h = np.zeros(64, np.uint32); h[17] = 5; cases["one"] = h
    h = np.zeros(64, np.uint32); h[3] = 5; h[60] = 1; cases["two"] = h
    cases["uniform1024"] = np.full(1024, 9, np.uint32)
    cases["ties"] = rng.choice(np.array([0, 1, 1, 2, 3, 3, 8]), size=1024).astype(np.uint32)
    cases["gauss"] = oracle.histogram(W.gaussian_codes(n=1 << 16, seed=5), 1024)
    cases["zipf256"] = oracle.histogram(W.zipf_bytes(n=1 << 18, seed=6), 256)
    h = np.zeros(1024, np.uint32); h[100:140] = _fib(40); cases["fib40_codes_over_32_bits"] = h
    h = np.zeros(256, np.uint32); h[:46] = _fib(46); cases["fib46"] = h
    cases["m4096"] = (rng.integers(1, 1000, size=4096)).astype(np.uint32)
    h = rng.integers(1, 1000, size=4097).astype(np.uint32); cases["m4097_global"] = h
    cases["normal65536"] = W.skewed_histogram(65536, 3_000_000, seed=7)
    cases["uniform65536"] = W.skewed_histogram(65536, 65536 * 3, kind="uniform")
    h = rng.integers(0, 3, size=8192).astype(np.uint32) * rng.integers(1, 1 << 20, size=8192).astype(np.uint32)
    cases["sparse8192"] = h
    # books of up to 256 used symbols take the 32-bit register path: used
    # counts around every 64-element register boundary, with geometric,
    # random and tied counts, scattered over the alphabet
    for mm in (2, 3, 63, 64, 65, 127, 128, 129, 191, 192, 193, 255, 256, 257):
        for kind in ("geom", "rand", "ties"):
            h = np.zeros(4096 if mm > 200 else 1024, np.uint32)
            pos = np.sort(rng.choice(h.size, size=mm, replace=False))
            if kind == "geom":
                v = np.maximum(1, (1e9 * 0.93 ** np.arange(mm))).astype(np.uint32)
                rng.shuffle(v)
            elif kind == "rand":
                v = rng.integers(1, 1 << 24, size=mm).astype(np.uint32)
            else:
                v = rng.choice(np.array([1, 2, 2, 5, 5, 5], np.uint32), size=mm)
            h[pos] = v
            cases[f"m{mm}_{kind}"] = h
    # 1024 < m <= 4096: tree in LDS, rounds merged by the whole workgroup
    cases["m2000_ties"] = np.concatenate([rng.choice(np.array([1, 2, 2, 3, 7], np.uint32), size=2000),
                                          np.zeros(96, np.uint32)])
    cases["m3000_geom"] = np.maximum(1, (1e9 * 0.995 ** np.arange(3000))).astype(np.uint32)
    # more than 4096 used: tree in the workspace; Zipf counts up to 2^28 take
    # seven 4-bit sort passes; geometric counts need more rounds than are
    # recorded (depths by pointer jumping)
    p = np.arange(1, 65537, dtype=np.float64) ** -1.05
    cases["zipf65536"] = np.maximum(1, np.round(p / p.sum() * (1 << 28))).astype(np.uint32)
    h = np.zeros(16384, np.uint32)
    h[rng.choice(16384, size=6000, replace=False)] = np.maximum(1, (1e9 * 0.9975 ** np.arange(6000))).astype(np.uint32)
    cases["m6000_geom_global"] = h
    # alphabets above 8192: the grid-wide sort, lengths and codewords when more
    # than 4096 symbols are used, else the single-workgroup build
    h = np.zeros(16384, np.uint32)
    h[rng.choice(16384, size=4097, replace=False)] = rng.integers(1, 1000, size=4097)
    cases["multi_m4097_a16384"] = h
    h = np.zeros(32768, np.uint32)
    h[rng.choice(32768, size=4096, replace=False)] = rng.integers(1, 1000, size=4096)
    cases["multi_fallback_m4096_a32768"] = h
    h = np.zeros(10000, np.uint32)
    h[rng.choice(10000, size=9000, replace=False)] = rng.integers(1, 1 << 20, size=9000)
    cases["multi_a10000_m9000"] = h
    h = np.zeros(16384, np.uint32)
    h[rng.choice(16384, size=6000, replace=False)] = rng.integers(1, 1 << 31, size=6000)
    cases["multi_counts_to_2^31"] = h
    h = np.zeros(20000, np.uint32)
    pos = rng.choice(20000, size=4200, replace=False)
    h[pos[:40]] = _fib(40)
    h[pos[40:]] = 1
    cases["multi_fib40_long_codes"] = h
    h = np.zeros(65536, np.uint32)
    h[rng.choice(65536, size=5000, replace=False)] = rng.choice(np.array([1, 2, 2, 3, 7], np.uint32), size=5000)
    cases["multi_ties_m5000_a65536"] = h
    cases["multi_empty_a16384"] = np.zeros(16384, np.uint32)
    h = np.zeros(65536, np.uint32); h[40000] = 7; cases["multi_one_a65536"] = h
    h = np.zeros(65536, np.uint32); h[3] = 1; h[65535] = 2; cases["multi_two_a65536"] = h
    # the sum of counts just below / at 2^32 - 1 (register path / general path)
    h = np.zeros(1024, np.uint32); h[:200] = 1; h[500] = 0xFFFFFFFE - 200 - 7; h[501:508] = 1
    assert int(h.sum(dtype=np.uint64)) == 0xFFFFFFFE
    cases["total_2^32-2"] = h
    h = h.copy(); h[502] += 1
    cases["total_2^32-1"] = h
    return cases


HISTS = _hist_cases()


@pytest.mark.parametrize("name", sorted(HISTS))
def test_codebook_parity(name):
    h = HISTS[name]
    ref = oracle.codebook(h)
    book, code = gpu_book(h)
    assert code == 0
    assert_book_equal(book, ref)


@pytest.mark.parametrize("name", ["m63_geom", "m231", "m3000_geom", "sparse8192", "m6000_geom_global", "zipf65536"])
def test_codebook_traced_equals_untraced(name):
    """The traced build is the same build: same book, and phase clocks that
    rise through the phases of the single-workgroup build (none for books
    built over the grid: alphabets above 8192 with more than 4096 used)."""
    if name == "m231":
        h = oracle.histogram(W.gaussian_codes(n=1 << 20, sigma=8.0, seed=3), 1024)
    else:
        h = HISTS[name]
    ref = oracle.codebook(h)
    hd = torch.from_numpy(h.view(np.int32)).cuda()
    ws = hf.new_workspace(1, h.size)
    status = hf.new_status()
    book = hf.Codebook.empty(h.size, "cuda")
    stamps = torch.zeros(9, dtype=torch.int64, device="cuda")
    hf.hf_build_codebook_traced(hd, book, ws, status, stamps)
    torch.cuda.synchronize()
    assert hf.read_status(status) == 0
    assert_book_equal(book, ref)
    t = stamps.cpu().numpy()
    if h.size > 8192 and ref.m > 4096:
        assert np.all(t == 0)
    else:
        assert np.all(t > 0) and np.all(np.diff(t) >= 0), t


def _random_small_books(count, seed):
    """Seeded books of 2..256 used symbols, scattered over alphabets up to
    1024 (one in five up to 65536), with counts that are tiny and tied, uniform, exponential, geometric,
    all equal, drawn from a few values, or large enough that merged weights
    pass 2^25 (the 64-bit merge keys): every round shape of the one-wave
    construction (one run only, runs of at most 32 each, of at most 64 each,
    and longer runs merged through LDS, then a queue that fits a register
    again)."""
    rng = np.random.default_rng(seed)
    books = []
    while len(books) < count:
        kind = len(books) % 7
        mm = int(rng.integers(2, 257))
        A = int(rng.integers(mm, 1025)) if len(books) % 5 else int(rng.integers(4097, 65537))
        h = np.zeros(A, np.int64)
        pos = rng.choice(A, size=mm, replace=False)
        if kind == 0:
            v = rng.integers(1, 5, mm)
        elif kind == 1:
            v = rng.integers(1, 1 << 24, mm)
        elif kind == 2:
            v = np.maximum(1, np.round(rng.exponential(50, mm))).astype(np.int64)
        elif kind == 3:
            v = np.maximum(1, (1e7 * 0.93 ** np.arange(mm))).astype(np.int64)
        elif kind == 4:
            v = np.full(mm, 7)
        elif kind == 5:
            v = rng.choice([1, 2, 2, 5, 5, 5, 9], size=mm)
        else:
            v = rng.integers(1, 0xFFFFFFF0 // (mm + 1), mm)
        h[pos] = v
        books.append(h.astype(np.uint32))
    return books


def test_codebook_parity_random_small_books():
    for i, h in enumerate(_random_small_books(280, seed=77)):
        ref = oracle.codebook(h)
        book, code = gpu_book(h)
        assert code == 0, i
        assert_book_equal(book, ref)


# ---------------------------------------------------------------------------
# encoding
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("n", [1, 255, 256, 4095, 4097, 70_001, 1 << 20])
def test_encode_small_and_ragged(n):
    x = W.gaussian_codes(n=n, seed=n)
    check_pipeline(x, 1024, 256)


@pytest.mark.parametrize("r", [1, 2, 3, 4, 5, 6])
def test_encode_independent_of_r(r):
    x = W.gaussian_codes(n=300_007, sigma=20.0, seed=3)
    check_pipeline(x, 1024, 1024, r)


@pytest.mark.parametrize("chunk", [256, 1024, 4096, 65536])
def test_encode_independent_of_chunk(chunk):
    x = W.zipf_bytes(n=1_000_003, seed=2)
    check_pipeline(x, 256, chunk)


def test_encode_single_symbol_stream():
    x = np.full(100_000, 7, dtype=np.uint16)
    book, words, offs, tb = check_pipeline(x, 16, 4096)
    assert tb == x.size


def _fib_stream(nfib: int, base: int, seed: int) -> np.ndarray:
    """Symbols base..base+nfib-1 with exactly F_1..F_nfib occurrences each,
    shuffled: the deepest Huffman tree, codes of nfib-1 bits."""
    counts = np.array(_fib(nfib), dtype=np.int64)
    x = np.repeat(np.arange(base, base + nfib, dtype=np.uint16), counts)
    np.random.default_rng(seed).shuffle(x)
    return x


@pytest.mark.parametrize("nfib,A,base,mode", [(29, 1024, 200, "split tables, 28-bit codes"),
                                              (30, 1024, 200, "split tables, 29-bit codes"),
                                              (32, 4096, 4000, "split tables, 31-bit codes"),
                                              (30, 8192, 5000, "codebook from global memory, 29-bit codes"),
                                              (27, 32768, 20000, "L2 packed table, 26-bit codes"),
                                              (30, 32768, 20000, "codebook from global memory, 29-bit codes"),
                                              (33, 1024, 200, "codebook from global memory, 32-bit codes"),
                                              (34, 1024, 200, "codes over 32 bits, bits ORed into the output")])
def test_encode_long_codes(nfib, A, base, mode):
    x = _fib_stream(nfib, base, nfib)
    ref_h = oracle.histogram(x, A)
    ref = oracle.codebook(ref_h)
    assert ref.lmax == nfib - 1
    book, code = gpu_book(ref_h)
    assert code == 0
    assert_book_equal(book, ref)
    rw, ro, tb = oracle.encode(x, ref, 4096)
    for r in (2, 4, 6):
        words, offs, code = gpu_encode(x, book, 4096, r)
        assert code == 0, mode
        assert np.array_equal(offs, ro), mode
        assert np.array_equal(words[: rw.size], rw), mode
        assert np.all(words[rw.size:] == SENTINEL)


@pytest.mark.parametrize("nfib,mode", [(20, "packed table"), (30, "split tables"),
                                       (33, "codebook from global memory"), (34, "codes over 32 bits")])
def test_encode_flags_slab_counts_of_other_symbols(nfib, mode):
    """Per-slab counts that are not the symbols' (here: those of another
    shuffle of the same multiset, so every slab has the right size but the
    wrong bits) place later slabs wrongly; every mode must flag it, and
    nothing may be written past the capacity."""
    x = _fib_stream(nfib, 200, 1)
    other = _fib_stream(nfib, 200, 2)
    A = 1024
    S = hf.hf_slab_count(x.size, A)
    assert S >= 2
    part = np.stack([oracle.histogram(other[lo:hi], A) for lo, hi in slab_ranges(x.size, S)])
    book, code = gpu_book(oracle.histogram(x, A))
    assert code == 0
    rw, _, tb = oracle.encode(x, oracle.codebook(oracle.histogram(x, A)), 4096)
    cap = rw.size
    words, offs, code = gpu_encode(x, book, 4096, 4, cap_words=cap, nslabs=S, slab_hist=part)
    assert code == hf.HF_ERR_SYMBOL, mode
    assert np.all(words[cap:] == SENTINEL), mode


def test_encode_large_alphabet_global_table():
    x = np.clip(np.rint(np.random.default_rng(4).normal(30000, 3000, size=500_001)), 0, 65535).astype(np.uint16)
    check_pipeline(x, 65536, 4096)


def test_encode_capacity_error_writes_nothing_past_capacity():
    x = W.gaussian_codes(n=200_000, seed=1)
    ref = oracle.codebook(oracle.histogram(x, 1024))
    book, _ = gpu_book(oracle.histogram(x, 1024))
    cap = ref.total_bits // 64  # half of what is needed
    words, offs, code = gpu_encode(x, book, 4096, cap_words=cap)
    assert code == hf.HF_ERR_CAPACITY
    assert np.all(words[cap:] == SENTINEL)


def test_encode_flags_symbol_without_code():
    x = W.gaussian_codes(n=50_000, seed=1)
    book, _ = gpu_book(oracle.histogram(x, 1024))
    y = x.copy()
    y[12345] = 1000  # no code in this book
    _, _, code = gpu_encode(y, book, 4096)
    assert code == hf.HF_ERR_SYMBOL


@pytest.mark.parametrize("A", [16384, 65536])
def test_encode_l2_table_flags_symbol_without_code(A):
    x = np.clip(np.rint(np.random.default_rng(8).normal(A / 2, A / 16, size=400_003)), 0, A - 1).astype(np.uint16)
    book, _ = gpu_book(oracle.histogram(x, A))
    assert int(book.info[1].item()) <= 27
    y = x.copy()
    y[123_457] = A - 1 if not np.any(x == A - 1) else 0  # no code in this book
    assert not np.any(x == y[123_457])
    _, _, code = gpu_encode(y, book, 4096)
    assert code == hf.HF_ERR_SYMBOL


@pytest.mark.parametrize("at", [5, 700_000, 2_178_307])  # first tile, middle, last symbol
def test_encode_split_tables_flag_symbol_without_code(at):
    x = _fib_stream(30, 200, 3)
    book, _ = gpu_book(oracle.histogram(x, 1024))
    assert int(book.info[1].item()) == 29
    y = x.copy()
    y[at % y.size] = 900  # no code in this book
    _, _, code = gpu_encode(y, book, 4096)
    assert code == hf.HF_ERR_SYMBOL


def test_encode_deterministic_across_runs():
    x = W.zipf_bytes(n=3_000_000, seed=11)
    book, _ = gpu_book(oracle.histogram(x, 256))
    a = gpu_encode(x, book, 4096)
    for _ in range(3):
        b = gpu_encode(x, book, 4096)
        assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


# ---------------------------------------------------------------------------
# decode check
# ---------------------------------------------------------------------------
def test_decode_check_accepts_and_rejects():
    x = W.gaussian_codes(n=500_000, sigma=10.0, seed=8)
    d = _dev(x)
    enc = hf.Encoder(x.size, 1024, 4096)
    out, offs = enc.run(d)
    res = hf.hf_decode_check(out, offs, d, 4096, enc.book)
    assert res.cpu().tolist() == [0, x.size]
    assert hf.read_status(enc.status) == 0
    bad = out.clone()
    bad[1000] ^= 1 << 7
    status = hf.new_status()
    res = hf.hf_decode_check(bad, offs, d, 4096, enc.book, status=status)
    r = res.cpu().tolist()
    assert r[0] > 0 and r[1] < x.size
    assert hf.read_status(status) == hf.HF_ERR_MISMATCH


# ---------------------------------------------------------------------------
# full-size workloads, whole-output comparison
# ---------------------------------------------------------------------------
def _full(x, A, chunk):
    book, words, offs, tb = check_pipeline(x, A, chunk)
    d = _dev(x)
    res = hf.hf_decode_check(torch.from_numpy(words.view(np.int32)).cuda(),
                             torch.from_numpy(offs.view(np.int64)).cuda(), d, chunk, book)
    assert res.cpu().tolist() == [0, x.size]


def test_full_gaussian_1M_u16():
    _full(W.make("gaussian_1M_u16_A1024"), 1024, 4096)


def test_full_lorenzo_512cube_u16():
    _full(W.make("lorenzo3d_512cube_u16_A1024"), 1024, 4096)


def test_full_zipf_100M_u8():
    _full(W.make("zipf_100M_u8_A256"), 256, 4096)


@functools.lru_cache(maxsize=1)
def _zipf_full():
    return W.make("zipf_100M_u8_A256")


@pytest.mark.parametrize("chunk", [1 << 10, 1 << 11, 1 << 13, 1 << 14, 1 << 15, 1 << 16])
def test_full_zipf_100M_u8_chunk_sweep(chunk):
    """The 10^8-byte text-like stream at every chunk size of the sweep
    (2^12 is covered above): the GPU path, with the library's default slabs
    and reduction factor, against the oracle's words and offsets."""
    x = _zipf_full()
    d = _dev(x)
    enc = hf.Encoder(x.size, 256, chunk)
    out, offs = enc.run(d)
    torch.cuda.synchronize()
    hf.raise_on_status(enc.status, "encode")
    ref = oracle.codebook(oracle.histogram(x, 256))
    ref_words, ref_offs, tb = oracle.encode(x, ref, chunk)
    nw = (tb + 31) // 32
    assert np.array_equal(_u64(offs), ref_offs)
    assert np.array_equal(_u32(out[:nw]), ref_words[:nw])
