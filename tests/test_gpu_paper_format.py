"""Parity of hf_encode_paper (the paper's ReduceShuffleMerge<M, r> format
with breaking groups in a side channel) with oracle/paper_format.py.

Integer work: words, chunk word offsets, breaking group indices and their
symbols are compared bit-exactly.  The device codebook is the oracle's own
book, so the comparison does not depend on the GPU codebook builder.  The
full-size Lorenzo stream is checked on sampled chunks, which the oracle
encodes one by one (a chunk's output depends only on its own symbols).
"""
import numpy as np
import pytest

import oracle
from oracle import paper_format as pf
from paper_2010_10039_amd import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2010_10039_amd import hf  # noqa: E402  (raises if libhf.so is missing)


def dev_book(ref) -> "hf.Codebook":
    A = ref.cl.size
    return hf.Codebook(A, torch.from_numpy(ref.cl.copy()).cuda(), torch.from_numpy(ref.cw.view(np.int64).copy()).cuda(),
                       torch.from_numpy(ref.first.view(np.int64).copy()).cuda(),
                       torch.from_numpy(ref.entry.view(np.int32).copy()).cuda(),
                       torch.from_numpy(ref.rev.view(np.int32).copy()).cuda(),
                       torch.from_numpy(ref.info.view(np.int64).copy()).cuda())


def dev_sym(x: np.ndarray):
    return torch.from_numpy(x.view(np.int16) if x.dtype == np.uint16 else x).cuda()


def run(x, ref, M, r, **kw):
    status = hf.new_status()
    out, offs, bg, bs, nb = hf.hf_encode_paper(dev_sym(x), dev_book(ref), M, r, status=status, **kw)
    code = hf.read_status(status)
    return code, out, offs, bg, bs, nb


def check(x, M, r, alphabet=None):
    ref = oracle.codebook(oracle.histogram(x, alphabet or (1024 if x.dtype == np.uint16 else 256)))
    code, out, offs, bg, bs, nb = run(x, ref, M, r)
    assert code == 0
    w, o, b, s = pf.encode(x, ref.cl, ref.cw, M, r)
    got_o = offs.cpu().numpy().view(np.uint64)
    assert np.array_equal(got_o, o)
    assert np.array_equal(out[: int(o[-1])].cpu().numpy().view(np.uint32), w)
    k = int(nb.item())
    assert k == b.size
    assert np.array_equal(bg[:k].cpu().numpy().view(np.uint64), b)
    got_s = bs[: k << r].cpu().numpy()
    assert np.array_equal(got_s.view(x.dtype) if x.dtype == np.uint16 else got_s, s)
    return b.size


@pytest.mark.parametrize("M,r", [(8, 1), (9, 2), (10, 2), (10, 3), (12, 3), (12, 4), (11, 5)])
@pytest.mark.parametrize("sigma", [2.0, 40.0])
def test_matches_oracle(M, r, sigma):
    x = W.gaussian_codes(n=100_003, alphabet=1024, sigma=sigma, seed=int(sigma) + M)
    nbreak = check(x, M, r)
    if sigma == 40.0 and r >= 3:
        assert nbreak > 0  # the side channel is exercised


def test_bytes():
    x = W.zipf_bytes(n=1_000_001, seed=3)
    check(x, 10, 3)


@pytest.mark.parametrize("M,r", [(10, 1), (12, 2)])
def test_large_alphabet(M, r):
    """An alphabet above the LDS copy's 4096 symbols: the book is read from
    global memory (wide Gaussian codes: some 6600 used symbols up to 9483,
    8.3 bits a symbol on average, so that groups both fit and break)."""
    x = W.gaussian_codes(n=300_007, alphabet=16384, sigma=2000.0, seed=4)
    nbreak = check(x, M, r, 16384)
    assert 0 < nbreak < (x.size >> r)


@pytest.mark.parametrize("M,r", [(10, 1), (12, 1), (10, 2)])
def test_long_codes_with_lds_book(M, r):
    """Codes of up to 27 bits in an alphabet the workgroups copy to LDS,
    merged into words that they nearly fill.  The book is the oracle's for
    Fibonacci counts on 45 symbols and 1 on the rest (lengths 2..27); the
    stream draws the 45 symbols uniformly, so at r = 1 about 1800 groups
    fit with a code over 25 bits."""
    A = 1024
    h = np.ones(A, np.uint64)
    f = [1, 2]
    while len(f) < 45:
        f.append(f[-1] + f[-2])
    h[:45] = f[::-1]
    ref = oracle.codebook(h)
    assert ref.cl.max() > 25
    x = np.random.default_rng(1).integers(0, 45, 200_003).astype(np.uint16)
    code, out, offs, bg, bs, nb = run(x, ref, M, r)
    assert code == 0
    w, o, b, s = pf.encode(x, ref.cl, ref.cw, M, r)
    assert np.array_equal(offs.cpu().numpy().view(np.uint64), o)
    assert np.array_equal(out[: int(o[-1])].cpu().numpy().view(np.uint32), w)
    k = int(nb.item())
    assert k == b.size
    assert np.array_equal(bg[:k].cpu().numpy().view(np.uint64), b)
    assert np.array_equal(bs[: k << r].cpu().numpy().view(np.uint16), s)


def test_capacity_errors_write_nothing_past_capacity():
    x = W.gaussian_codes(n=50_000, alphabet=1024, sigma=40.0, seed=1)
    ref = oracle.codebook(oracle.histogram(x, 1024))
    w, o, b, s = pf.encode(x, ref.cl, ref.cw, 10, 4)
    assert b.size > 4
    bg = torch.full((b.size,), -7, dtype=torch.int64, device="cuda")
    bs = torch.full((b.size << 4,), -7, dtype=torch.int16, device="cuda")
    code, *_ = run(x, ref, 10, 4, break_groups=bg[:3], break_syms=bs[: 3 << 4])
    assert code == hf.HF_ERR_CAPACITY
    assert (bg[3:] == -7).all() and (bs[3 << 4:] == -7).all()
    # a real stream (few breaking groups at r = 2, sigma = 8), one word short
    x = W.gaussian_codes(n=50_000, alphabet=1024, sigma=8.0, seed=1)
    ref = oracle.codebook(oracle.histogram(x, 1024))
    w, o, b, s = pf.encode(x, ref.cl, ref.cw, 10, 2)
    assert int(o[-1]) > 1000
    out = torch.full((int(o[-1]) + 8,), -7, dtype=torch.int32, device="cuda")
    code, *_ = run(x, ref, 10, 2, out=out[: int(o[-1]) - 1])
    assert code == hf.HF_ERR_CAPACITY
    assert (out == -7).all()


def test_symbol_without_code():
    x = W.gaussian_codes(n=10_000, alphabet=1024, sigma=3.0, seed=2)
    ref = oracle.codebook(oracle.histogram(x, 1024))
    y = x.copy()
    y[5000] = 5  # count 0 in the book: no code
    code, *_ = run(y, ref, 10, 2)
    assert code == hf.HF_ERR_SYMBOL


def test_empty():
    ref = oracle.codebook(oracle.histogram(np.zeros(4, np.uint16), 1024))
    offs = torch.full((1,), 9, dtype=torch.int64, device="cuda")
    nb = torch.full((1,), 9, dtype=torch.int64, device="cuda")
    code, out, offs, bg, bs, nb = run(np.zeros(0, np.uint16), ref, 10, 3, offsets=offs, nbreak=nb)
    assert code == 0 and int(offs[0]) == 0 and int(nb[0]) == 0


def test_full_size_lorenzo_sampled_chunks():
    x = W.make("lorenzo3d_512cube_u16_A1024")
    ref = oracle.codebook(oracle.histogram(x, 1024))
    M, r = 10, 3
    code, out, offs, bg, bs, nb = run(x, ref, M, r)
    assert code == 0
    C = 1 << M
    o = offs.cpu().numpy().view(np.uint64)
    k_all = int(nb.item())
    groups = bg[:k_all].cpu().numpy().view(np.uint64)
    assert np.all(np.diff(groups.astype(np.int64)) > 0)
    rng = np.random.default_rng(0)
    nch = (x.size + C - 1) // C
    for k in list(rng.integers(0, nch, 40)) + [0, nch - 1]:
        xs = x[k * C:(k + 1) * C]
        w, oo, b, s = pf.encode(xs, ref.cl, ref.cw, M, r)
        assert int(o[k + 1] - o[k]) == int(oo[-1])
        assert np.array_equal(out[int(o[k]):int(o[k + 1])].cpu().numpy().view(np.uint32), w)
        g0 = (k * C) >> r
        mine = groups[(groups >= g0) & (groups < g0 + (C >> r))] - g0
        assert np.array_equal(mine, b)


@pytest.fixture(scope="module")
def long_stream():
    """20 M Lorenzo codes (a ragged length) with a wide Gaussian segment
    spliced into the middle, and the oracle's book for them."""
    n = 20_000_003
    x = W.make("lorenzo3d_512cube_u16_A1024")[:n].copy()
    wide = W.gaussian_codes(n=1 << 20, alphabet=1024, sigma=40.0, seed=9)
    x[n // 2:n // 2 + wide.size] = wide
    return x, oracle.codebook(oracle.histogram(x, 1024))


@pytest.mark.parametrize("M,r", [(8, 1), (10, 2), (11, 3), (12, 4), (9, 5)])
def test_long_ragged_stream_sampled_chunks(long_stream, M, r):
    """A stream long enough that every workgroup encodes many tiles in turn:
    sampled chunks (the first, the last, two in the wide segment, random
    ones) against the oracle: words, chunk offsets, breaking groups and
    their symbols."""
    x, ref = long_stream
    n = x.size
    code, out, offs, bg, bs, nb = run(x, ref, M, r)
    assert code == 0
    C, G = 1 << M, 1 << r
    o = offs.cpu().numpy().view(np.uint64)
    nch = (n + C - 1) // C
    assert o.size == nch + 1 and np.all(np.diff(o.astype(np.int64)) >= 0)
    k_all = int(nb.item())
    groups = bg[:k_all].cpu().numpy().view(np.uint64)
    syms = bs[: k_all << r].cpu().numpy().view(np.uint16).reshape(k_all, G)
    assert np.all(np.diff(groups.astype(np.int64)) > 0)
    rng = np.random.default_rng(M * 10 + r)
    mid = (n // 2 + (1 << 19)) // C  # inside the wide segment
    for k in list(rng.integers(0, nch, 24)) + [0, mid, mid + 1, nch - 1]:
        xs = x[k * C:(k + 1) * C]
        w, oo, b, s = pf.encode(xs, ref.cl, ref.cw, M, r)
        assert int(o[k + 1] - o[k]) == int(oo[-1])
        assert np.array_equal(out[int(o[k]):int(o[k + 1])].cpu().numpy().view(np.uint32), w)
        g0 = (k * C) >> r
        sel = (groups >= g0) & (groups < g0 + ((xs.size + G - 1) >> r))
        assert np.array_equal(groups[sel] - g0, b)
        assert np.array_equal(syms[sel].reshape(-1), s.reshape(-1))
        if k == mid and r >= 2:
            assert b.size > 0  # the side channel is exercised inside the long stream
