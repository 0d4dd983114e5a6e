"""Parity of the GPU decoder (hf_decode) with the CPU oracle.

The decoder is fed the oracle's own stream, offsets and codebook, so it is
checked independently of the GPU encoder: every decoded symbol must equal
the input and the oracle's serial decode.  Then the GPU encoder's output
round-trips, and streams that are no valid encoding raise HF_ERR_STREAM."""
import functools

import numpy as np
import pytest

import oracle
from paper_2010_10039_amd import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2010_10039_amd import hf  # noqa: E402


def _t(a: np.ndarray, dtype) -> torch.Tensor:
    return torch.from_numpy(np.ascontiguousarray(a).view(dtype)).cuda()


def dev_book(ref: oracle.Codebook, A: int) -> hf.Codebook:
    rev = np.zeros(A, np.uint32)
    rev[: ref.rev.size] = ref.rev[:A]
    return hf.Codebook(A, _t(ref.cl, np.uint8), _t(ref.cw.astype(np.uint64), np.int64),
                       _t(ref.first.astype(np.uint64), np.int64), _t(ref.entry.astype(np.uint32), np.int32),
                       _t(rev, np.int32), _t(ref.info.astype(np.uint64), np.int64))


def gpu_decode(words, offs, n, x_dtype, chunk, book):
    dt = torch.uint8 if x_dtype == np.uint8 else torch.int16
    w = _t(words if words.size else np.zeros(1, np.uint32), np.int32)
    o = _t(offs.astype(np.uint64), np.int64)
    status = hf.new_status()
    out = torch.full((max(n, 1),), 0x5A, dtype=dt, device="cuda")
    hf.hf_decode(w, o, n, dt, chunk, book, out=out[:n] if n else out[:0], status=status)
    code = hf.read_status(status)
    got = out[:n].cpu().numpy()
    return (got.view(np.uint16) if x_dtype == np.uint16 else got), code


def check(x: np.ndarray, A: int, chunk: int):
    ref = oracle.codebook(oracle.histogram(x, A))
    words, offs, tb = oracle.encode(x, ref, chunk)
    got, code = gpu_decode(words, offs, x.size, x.dtype, chunk, dev_book(ref, A))
    assert code == 0
    assert np.array_equal(got, x)
    if x.size:
        serial, end = oracle.decode(words, tb, x.size, ref, dtype=x.dtype)
        assert end == tb and np.array_equal(got, serial)
    return ref


def _fib_stream(nfib: int, base: int, seed: int) -> np.ndarray:
    f = [1, 1]
    while len(f) < nfib:
        f.append(f[-1] + f[-2])
    x = np.repeat(np.arange(base, base + nfib, dtype=np.uint16), f[:nfib])
    np.random.default_rng(seed).shuffle(x)
    return x


@pytest.mark.parametrize("chunk", [256, 1024, 4096, 65536])
def test_decode_gaussian_chunks(chunk):
    check(W.gaussian_codes(n=(1 << 20) + 77, seed=3), 1024, chunk)


@pytest.mark.parametrize("n", [1, 255, 256, 4097, 70_001])
def test_decode_small_and_ragged(n):
    check(W.gaussian_codes(n=n, seed=n), 1024, 256)


def test_decode_empty_stream():
    x = np.zeros(0, np.uint16)
    book = dev_book(oracle.codebook(np.zeros(1024, np.uint32)), 1024)
    got, code = gpu_decode(np.zeros(0, np.uint32), np.zeros(1, np.uint64), 0, np.uint16, 4096, book)
    assert code == 0 and got.size == 0


def test_decode_one_distinct_symbol():
    check(np.full(100_003, 9, np.uint16), 64, 4096)


def test_decode_zipf_bytes():
    check(W.zipf_bytes(n=3_000_001, seed=4), 256, 4096)


def test_decode_lorenzo_codes():
    ref = check(W.make("lorenzo3d_512cube_u16_A1024", scale=6), 1024, 4096)
    assert ref.lmax > 12  # codes beyond one table lookup


@pytest.mark.parametrize("nfib", [20, 30, 34])  # codes of 19, 29 and 33 bits
def test_decode_long_codes(nfib):
    ref = check(_fib_stream(nfib, 200, nfib), 1024, 4096)
    assert ref.lmax == nfib - 1


def test_decode_large_alphabet():
    x = np.clip(np.rint(np.random.default_rng(4).normal(30000, 3000, size=500_001)), 0, 65535).astype(np.uint16)
    check(x, 65536, 1024)


@pytest.mark.parametrize("shift", [1, 3])  # output 2 or 6 bytes past a 16-byte boundary: element stores
def test_decode_unaligned_output(shift):
    x = W.gaussian_codes(n=100_000, seed=12)
    ref = oracle.codebook(oracle.histogram(x, 1024))
    words, offs, tb = oracle.encode(x, ref, 1024)
    buf = torch.zeros(x.size + 8, dtype=torch.int16, device="cuda")
    status = hf.new_status()
    hf.hf_decode(_t(words, np.int32), _t(offs.astype(np.uint64), np.int64), x.size, torch.int16, 1024,
                 dev_book(ref, 1024), out=buf[shift:shift + x.size], status=status)
    assert hf.read_status(status) == 0
    got = buf.cpu().numpy().view(np.uint16)
    assert np.array_equal(got[shift:shift + x.size], x)
    assert np.all(got[:shift] == 0) and np.all(got[shift + x.size:] == 0)


def test_decode_gpu_encoder_round_trip():
    x = W.gaussian_codes(n=3_000_017, seed=11)
    enc = hf.Encoder(x.size, 1024, 4096, 0)
    d = torch.from_numpy(x.view(np.int16)).cuda()
    enc.run(d)
    status = hf.new_status()
    out = hf.hf_decode(enc.out, enc.offsets, x.size, torch.int16, 4096, enc.book, status=status)
    torch.cuda.synchronize()
    hf.raise_on_status(enc.status, "encode")
    hf.raise_on_status(status, "decode")
    assert torch.equal(out, d)


def test_decode_flags_invalid_stream():
    """A one-symbol book has the single code 0: a stream of ones is no
    encoding; offsets that do not match the stream fail too."""
    x = np.full(5000, 3, np.uint16)
    ref = oracle.codebook(oracle.histogram(x, 16))
    book = dev_book(ref, 16)
    words = np.full(200, 0xFFFFFFFF, np.uint32)
    offs = np.array([0, 4096, 5000], np.uint64)
    _, code = gpu_decode(words, offs, x.size, np.uint16, 4096, book)
    assert code == hf.HF_ERR_STREAM
    words, offs, tb = oracle.encode(x, ref, 4096)
    bad = offs.copy()
    bad[1] += 1
    _, code = gpu_decode(words, bad, x.size, np.uint16, 4096, book)
    assert code == hf.HF_ERR_STREAM


def test_decode_fixed_length_code():
    """256 equally frequent bytes: every code is 8 bits, so a lane that starts
    off a code boundary never resynchronises; lane regions are multiples of
    the gcd of the code lengths, which keeps every start on a boundary."""
    x = np.tile(np.arange(256, dtype=np.uint8), 4001)
    np.random.default_rng(5).shuffle(x)
    ref = check(x, 256, 4096)
    assert set(np.unique(ref.cl[ref.cl > 0]).tolist()) == {8}


def test_decode_even_lengths_only():
    """Code lengths 2 and 4 only (gcd 2)."""
    h = np.array([4] * 3 + [1] * 4, np.uint32) * 1000
    x = np.repeat(np.arange(7, dtype=np.uint16), h)
    np.random.default_rng(6).shuffle(x)
    ref = check(x, 16, 4096)
    assert set(np.unique(ref.cl[ref.cl > 0]).tolist()) == {2, 4}


def test_decode_near_fixed_length_code():
    """Mostly 8-bit codes with a few 7- and 9-bit ones: lanes resynchronise
    slowly, so the restart rounds run long chains."""
    rng = np.random.default_rng(7)
    p = np.ones(256)
    p[:8] = 2.5
    p /= p.sum()
    x = rng.choice(256, size=2_000_003, p=p).astype(np.uint8)
    ref = check(x, 256, 4096)
    assert ref.cl[ref.cl > 0].min() < 8 < ref.cl.max()


@functools.lru_cache(maxsize=1)
def _lorenzo_full():
    return W.make("lorenzo3d_512cube_u16_A1024")


@pytest.mark.parametrize("chunk", [1024, 4096, 65536])
def test_decode_full_lorenzo_stream(chunk):
    """The whole 134 M-symbol Lorenzo code stream, against the input and the
    oracle's serial decode."""
    check(_lorenzo_full(), 1024, chunk)
