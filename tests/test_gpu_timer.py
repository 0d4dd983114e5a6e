"""The stage timer (hf_time_next_main_kernel): the armed events are recorded
around the timed stage's main kernel(s), within the bracketing step, and
the outputs are unchanged by timing."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2010_10039_amd import hf  # noqa: E402
from paper_2010_10039_amd import workloads as W  # noqa: E402


def _events(k):
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(k)]
    for e in ev:
        e.record()
    torch.cuda.synchronize()
    return ev


def test_stage_timers_inside_the_step():
    x = W.gaussian_codes(n=(1 << 22) + 123, alphabet=1024)
    d = torch.from_numpy(x.view(np.int16)).cuda()
    enc = hf.Encoder(x.size, 1024, 4096, 4)
    enc.run(d)
    torch.cuda.synchronize()
    ref_out, ref_off = enc.out.clone(), enc.offsets.clone()
    s0, s1, h0, h1, c0, c1, e0, e1 = _events(8)
    s0.record()
    enc.run(d, timers={"hist": (h0, h1), "codebook": (c0, c1), "encode": (e0, e1)})
    s1.record()
    torch.cuda.synchronize()
    hf.raise_on_status(enc.status, "timed")
    step = s0.elapsed_time(s1)
    for a, b in ((h0, h1), (c0, c1), (e0, e1)):
        dt = a.elapsed_time(b)
        assert 0 < dt <= step
        assert s0.elapsed_time(a) >= 0 and b.elapsed_time(s1) >= 0
    # stage order within the step
    assert h1.elapsed_time(c0) >= 0 and c1.elapsed_time(e0) >= 0
    assert torch.equal(enc.out, ref_out) and torch.equal(enc.offsets, ref_off)


def test_batch_encode_timer():
    syms, alph = W.batched_streams(12, seed=5, min_log2=14, max_log2=19, device="cuda")
    enc = hf.BatchEncoder(syms, alph, 4096, 0)
    enc.run()
    torch.cuda.synchronize()
    ref = [o.clone() for o in enc.outs]
    s0, s1, e0, e1 = _events(4)
    s0.record()
    hf.hf_time_next_main_kernel(e0, e1)
    enc.run()
    s1.record()
    torch.cuda.synchronize()
    assert np.all(enc.status.cpu().numpy() == 0)
    dt = e0.elapsed_time(e1)
    assert 0 < dt <= s0.elapsed_time(s1)
    for a, b in zip(ref, enc.outs):
        assert torch.equal(a, b)
