"""hf_encode_noalloc (the encoder with the library's fixed device scratch in
place of a workspace) against hf_encode on the same symbols and codebook:
every output word and chunk offset must be equal, on calls made back to
back, each later one on a smaller stream (the scratch keeps the previous
call's contents), and both must equal the oracle's stream."""
import numpy as np
import pytest

import oracle
from paper_2010_10039_amd import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2010_10039_amd import hf  # noqa: E402


def _dev(x: np.ndarray) -> torch.Tensor:
    return torch.from_numpy(x.view(np.int16) if x.dtype == np.uint16 else x).cuda()


def _book(d: torch.Tensor, A: int) -> hf.Codebook:
    return hf.hf_build_codebook(hf.hf_histogram(d, A))


def _compare(x: np.ndarray, A: int, chunk: int, r: int):
    d = _dev(x)
    book = _book(d, A)
    n = x.size
    nch = (n + chunk - 1) // chunk
    words = hf.hf_bound_words(n, A)
    ref_out, ref_offs = hf.hf_encode(d, book, chunk, r)
    # output buffers pre-filled with a sentinel: words past the stream stay as they were
    out = torch.full((words,), 0x5A5A5A5A, dtype=torch.int32, device="cuda")
    offs = torch.full((nch + 1,), -1, dtype=torch.int64, device="cuda")
    status = hf.new_status()
    hf.hf_encode_noalloc(d, book, out, offs, status, chunk, r)
    torch.cuda.synchronize()
    assert hf.read_status(status) == 0
    tb = int(offs[-1].item())
    nw = (tb + 31) // 32
    assert torch.equal(offs, ref_offs)
    assert torch.equal(out[:nw], ref_out[:nw])
    assert bool((out[nw:] == 0x5A5A5A5A).all())
    ref = oracle.codebook(oracle.histogram(x, A))
    o_words, o_offs, o_tb = oracle.encode(x, ref, chunk)
    assert o_tb == tb
    assert np.array_equal(offs.cpu().numpy().view(np.uint64), o_offs)
    assert np.array_equal(out[:nw].cpu().numpy().view(np.uint32), o_words[:nw])


def test_noalloc_matches_encode_on_successive_calls():
    # a large stream, then smaller ones with other widths, alphabets and chunks
    _compare(W.make("lorenzo3d_512cube_u16_A1024", scale=3), 1024, 4096, 0)
    _compare(W.zipf_bytes(n=1_000_003, seed=2), 256, 1024, 3)
    _compare(W.gaussian_codes(n=70_001, sigma=3.0, seed=5), 1024, 256, 5)


def test_noalloc_large_alphabet_table_then_smaller():
    # alphabets above 8192 keep their packed table in the scratch too
    x = np.clip(np.rint(np.random.default_rng(3).normal(30000, 2500, size=2_000_001)), 0, 65535).astype(np.uint16)
    _compare(x, 65536, 4096, 4)
    _compare(x[:12_345], 65536, 1024, 4)


def test_noalloc_empty_stream():
    d = torch.zeros(0, dtype=torch.int16, device="cuda")
    book = _book(torch.zeros(1, dtype=torch.int16, device="cuda"), 1024)
    out = torch.zeros(1, dtype=torch.int32, device="cuda")
    offs = torch.full((1,), -1, dtype=torch.int64, device="cuda")
    status = hf.new_status()
    hf.hf_encode_noalloc(d, book, out, offs, status, 4096, 0)
    torch.cuda.synchronize()
    assert hf.read_status(status) == 0 and int(offs[0].item()) == 0
