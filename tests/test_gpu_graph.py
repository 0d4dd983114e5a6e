"""The whole path (histogram, codebook, encode) captured as one HIP graph:
every replay equals the eager pass bit for bit, also with other eager work
and synchronizations between the replays."""
import numpy as np
import pytest

import oracle
from paper_2010_10039_amd import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2010_10039_amd import hf  # noqa: E402


def _dev(x):
    return torch.from_numpy(x.view(np.int16) if x.dtype == np.uint16 else x).cuda()


def _snapshot(enc, nw):
    """The pass's results: the stream's words (the encoder writes no word
    past them), offsets, histogram and book."""
    return [t.clone() for t in (enc.out[:nw], enc.offsets, enc.hist, enc.book.cl, enc.book.cw, enc.book.info)]


@pytest.mark.parametrize("workload", ["gaussian", "zipf_bytes"])
def test_graph_replays_equal_eager(workload):
    if workload == "gaussian":
        x, A = W.gaussian_codes(n=1 << 20, alphabet=1024, sigma=2.0, seed=0), 1024
    else:
        x, A = W.zipf_bytes(n=3_000_017, seed=4), 256
    d = _dev(x)
    enc = hf.Encoder(x.size, A, 4096, 0)
    enc.run(d)
    torch.cuda.synchronize()
    # the eager pass equals the oracle
    ref = oracle.codebook(oracle.histogram(x, A))
    words, offs, tb = oracle.encode(x, ref, 4096)
    nw = (tb + 31) // 32
    eager = _snapshot(enc, nw)
    assert np.array_equal(enc.out[:nw].cpu().numpy().view(np.uint32), words[:nw])
    assert np.array_equal(enc.offsets.cpu().numpy().view(np.uint64), offs)

    g = enc.capture(d)
    # other eager work on other buffers between the replays
    y = W.gaussian_codes(n=300_001, alphabet=1024, sigma=9.0, seed=3)
    other = hf.Encoder(y.size, 1024, 4096, 0)
    dy = _dev(y)
    for k in range(4):
        for t in (enc.out, enc.offsets, enc.hist):
            t.fill_(-1)
        enc.book.cl.fill_(255)
        torch.cuda.synchronize()
        g.replay()
        other.run(dy)
        torch.cuda.synchronize()
        for a, b in zip(_snapshot(enc, nw), eager):
            assert torch.equal(a, b), k
    assert hf.read_status(enc.status) == 0
    assert hf.read_status(other.status) == 0
