"""Parity of the fused quantizing front end (hf_lorenzo_histogram, through
the C ABI) with its CPU oracle (oracle/lorenzo.py).

Codes, histograms and per-slab counts are integers: every comparison is
bit-exact.  The float step (prequantization) is taken in float32 on both
sides, so it decides the same integers.  Shapes cover the vector path
(nx % 8 == 0, aligned), the element path (odd rows, misaligned buffers),
1D and 2D fields, fields with one row per plane, the longest row the LDS
ring takes, many slabs with ragged ends, radii from 1 to 8192, huge finite
values, exact ties, non-finite values (refused with HF_ERR_VALUE on every
path, as the oracle refuses them), the empty field, chained slabs (four slabs one plane apart per
workgroup, short last chains), and the full 512^3 benchmark field.  The encoder
fed with the fused per-slab counts must produce the very stream the plain
histogram path produces, and that stream must decode to the oracle's codes.
"""
import numpy as np
import pytest

from oracle import lorenzo as lz
from paper_2010_10039_amd import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2010_10039_amd import hf  # noqa: E402  (raises if libhf.so is missing)


def _inv(eb: float) -> float:
    return float(np.float32(1.0 / (2.0 * eb)))


def run_gpu(x: np.ndarray, inv: float, radius: int, nslabs: int = 0, x_off: int = 0, c_off: int = 0):
    """Front end on the GPU.  x_off / c_off place the field / codes that many
    elements into larger buffers (misaligned starts)."""
    nz, ny, nx = x.shape
    n = x.size
    A = 2 * radius
    xb = torch.zeros(n + x_off, dtype=torch.float32, device="cuda")
    xb[x_off:] = torch.from_numpy(x.reshape(-1)).cuda()
    xd = xb[x_off:]
    cb = torch.full((n + c_off,), -1, dtype=torch.int16, device="cuda")
    cd = cb[c_off:]
    hist = torch.full((A,), -1, dtype=torch.int32, device="cuda")
    sh = torch.full((max(1, nslabs) * A,), -1, dtype=torch.int32, device="cuda") if nslabs else None
    status = hf.new_status()
    hf.hf_lorenzo_histogram(xd, (nz, ny, nx), inv, radius, cd, hist, nslabs, sh, status)
    torch.cuda.synchronize()
    assert hf.read_status(status) == hf.HF_OK
    codes = cd.cpu().numpy().view(np.uint16)
    h = hist.cpu().numpy().view(np.uint32)
    rows = sh.cpu().numpy().view(np.uint32).reshape(nslabs, A) if nslabs else None
    return codes, h, rows


def check(x: np.ndarray, inv: float, radius: int, nslabs: int = 0, **kw):
    codes, h, rows = run_gpu(x, inv, radius, nslabs, **kw)
    want = lz.lorenzo_codes(x, inv, radius)
    bad = np.flatnonzero(codes != want)
    assert bad.size == 0, f"{bad.size} codes differ, first at {bad[0]}: {codes[bad[0]]} vs {want[bad[0]]}"
    assert np.array_equal(h, lz.histogram(want, 2 * radius))
    if nslabs:
        assert np.array_equal(rows, lz.slab_histograms(want, 2 * radius, nslabs))
    return want


SHAPES = [
    ((8, 16, 512), 3),     # vector path, several slabs
    ((5, 7, 96), 1),       # vector path, one block
    ((3, 33, 257), 7),     # odd rows: element path, 7 slabs of whole blocks
    ((1, 1, 100003), 5),   # 1D: no ring, ragged last slab
    ((1, 300, 300), 4),    # 2D
    ((40, 1, 1000), 9),    # one row per plane
    ((2, 3, 8192), 12),    # the longest row the ring takes
    ((17, 19, 64), 2),     # planes not a multiple of the step
    ((1, 1, 1), 1),        # a single value
]


@pytest.mark.parametrize("shape,nslabs", SHAPES)
def test_shapes_match_oracle(shape, nslabs):
    x = W.random_field(shape, seed=sum(shape))
    eb = 1e-3 * max(float(x.max() - x.min()), 1.0)
    check(x, _inv(eb), 512, nslabs)
    check(x, _inv(eb), 512, 0)  # no per-slab counts: global atomics


# Equal slabs of whole 2048-value steps that tile the planes take the chained
# kernel (four slabs one plane apart per workgroup, plane-back values passed
# in LDS); the last chain is short when the plane count is not a multiple of 4.
CHAINS = [
    ((7, 64, 128), 14, 512),   # 2 slabs per plane, 2 chains, the second with 3 planes
    ((7, 64, 128), 7, 512),    # 1 slab per plane
    ((9, 32, 256), 18, 512),   # last chain of a single plane
    ((4, 8, 512), 4, 512),     # exactly one chain
    ((6, 32, 256), 12, 2048),  # alphabet 4096
    ((7, 64, 128), 0, 512),    # no per-slab counts: counts added with atomics
]


@pytest.mark.parametrize("shape,nslabs,radius", CHAINS)
def test_chained_slabs_match_oracle(shape, nslabs, radius):
    x = W.random_field(shape, seed=sum(shape) + nslabs, noise_rel_std=0.02)
    eb = 1e-3 * float(x.max() - x.min())
    check(x, _inv(eb), radius, nslabs)


@pytest.mark.parametrize("radius", [1, 2, 3, 64, 2048])
def test_radii_with_slabs(radius):
    x = W.random_field((6, 20, 136), seed=radius, noise_rel_std=0.05)
    eb = 2e-3 * float(x.max() - x.min())
    want = check(x, _inv(eb), radius, nslabs=2)
    if radius <= 3:
        assert (want == 0).any()  # outliers exercised


@pytest.mark.parametrize("radius", [4096, 8192])
def test_large_alphabets_without_slabs(radius):
    x = W.random_field((4, 50, 200), seed=radius, noise_rel_std=0.3)
    eb = 1e-5 * float(x.max() - x.min())
    want = check(x, _inv(eb), radius)
    assert (want == 0).any() and np.unique(want).size > 100


@pytest.mark.parametrize("x_off,c_off", [(1, 0), (0, 1), (3, 5), (4, 8)])
def test_misaligned_buffers(x_off, c_off):
    x = W.random_field((4, 24, 512), seed=7)
    eb = 1e-3 * float(x.max() - x.min())
    check(x, _inv(eb), 512, nslabs=2, x_off=x_off, c_off=c_off)


def test_huge_values_and_ties():
    rng = np.random.default_rng(9)
    x = rng.normal(0, 3, size=(4, 8, 64)).astype(np.float32)
    flat = x.reshape(-1)
    flat[11::89] = 1e30
    flat[13::83] = -1e30
    flat[17::79] = 3e38  # the float32 product overflows to +inf and clamps
    k = rng.integers(-50, 50, size=flat.size // 7)
    flat[1::7][: k.size] = ((k + 0.5) / 4.0).astype(np.float32)  # exact ties at inv = 4
    check(x, 4.0, 512, nslabs=1)
    check(x, 4.0, 8, nslabs=1)


# (shape, nslabs, where): the vector path, the element path (odd rows), the
# chained path (equal slabs tiling the planes), and the unchained vector path
# without per-slab counts; `where` puts the one bad value first, inside, or
# last in the field.
@pytest.mark.parametrize("shape,nslabs", [((4, 8, 64), 1), ((3, 5, 37), 1), ((8, 32, 256), 16), ((4, 24, 512), 0)])
@pytest.mark.parametrize("bad", [np.nan, np.inf, -np.inf])
@pytest.mark.parametrize("where", ["first", "middle", "last"])
def test_non_finite_values_are_refused(shape, nslabs, bad, where):
    """The oracle refuses a field holding a NaN or an infinity
    (lorenzo.NonFiniteInput); the kernel must raise HF_ERR_VALUE."""
    x = W.random_field(shape, seed=3)
    flat = x.reshape(-1)
    flat[{"first": 0, "middle": flat.size // 2 + 3, "last": flat.size - 1}[where]] = bad
    inv = _inv(1e-3 * float(np.nanmax(x[np.isfinite(x)]) - np.nanmin(x[np.isfinite(x)])))
    with pytest.raises(lz.NonFiniteInput):
        lz.lorenzo_codes(x, inv, 512)
    A = 1024
    xd = torch.from_numpy(flat).cuda()
    cd = torch.empty(x.size, dtype=torch.int16, device="cuda")
    hist = torch.empty(A, dtype=torch.int32, device="cuda")
    sh = torch.empty(max(1, nslabs) * A, dtype=torch.int32, device="cuda") if nslabs else None
    status = hf.new_status()
    hf.hf_lorenzo_histogram(xd, x.shape, inv, 512, cd, hist, nslabs, sh, status)
    assert hf.read_status(status) == hf.HF_ERR_VALUE


def test_empty_field_zeroes_histogram():
    hist = torch.full((1024,), 7, dtype=torch.int32, device="cuda")
    xd = torch.zeros(1, dtype=torch.float32, device="cuda")
    cd = torch.zeros(1, dtype=torch.int16, device="cuda")
    hf.hf_lorenzo_histogram(xd[:0], (0, 4, 8), 1.0, 512, cd[:0], hist)
    assert int(hist.abs().sum()) == 0


def test_repeated_calls_reuse_buffers():
    """Two calls into the same buffers, the second on a smaller field: every
    output is rewritten, none accumulates."""
    x1 = W.random_field((6, 32, 256), seed=1)
    x2 = W.random_field((2, 32, 256), seed=2)
    inv = _inv(1e-3 * float(x1.max() - x1.min()))
    A = 1024
    xd = torch.from_numpy(x1.reshape(-1)).cuda()
    cd = torch.empty(x1.size, dtype=torch.int16, device="cuda")
    hist = torch.empty(A, dtype=torch.int32, device="cuda")
    sh = torch.empty(3 * A, dtype=torch.int32, device="cuda")
    for x in (x1, x2):
        xd[: x.size] = torch.from_numpy(x.reshape(-1)).cuda()
        nb = (x.size + 4095) // 4096
        hf.hf_lorenzo_histogram(xd[: x.size], x.shape, inv, 512, cd[: x.size], hist, min(3, nb), sh[: min(3, nb) * A])
        want = lz.lorenzo_codes(x, inv, 512)
        assert np.array_equal(cd[: x.size].cpu().numpy().view(np.uint16), want)
        assert np.array_equal(hist.cpu().numpy().view(np.uint32), lz.histogram(want, A))
        rows = sh[: min(3, nb) * A].cpu().numpy().view(np.uint32).reshape(-1, A)
        assert np.array_equal(rows, lz.slab_histograms(want, A, min(3, nb)))


def test_feeds_encoder_like_the_plain_histogram():
    """Codes and per-slab counts from the front end encode to exactly the
    stream that hf_histogram's counts give, and it decodes to the oracle's
    codes."""
    x, eb = W.lorenzo_field(dim=96, seed=5)
    inv = _inv(eb)
    n, A, chunk = x.size, 1024, 4096
    S = hf.hf_slab_count(n, A)
    xd = torch.from_numpy(x.reshape(-1)).cuda()
    codes, hist = hf.hf_lorenzo_histogram(xd, x.shape, inv, 512)
    sh_f = torch.empty(S * A, dtype=torch.int32, device="cuda")
    codes2, hist2 = hf.hf_lorenzo_histogram(xd, x.shape, inv, 512, nslabs=S, slab_hist=sh_f)
    assert torch.equal(codes, codes2) and torch.equal(hist, hist2)
    sh_h = torch.empty(S * A, dtype=torch.int32, device="cuda")
    status = hf.new_status()
    ws = hf.new_workspace(n, A, chunk)
    hist3 = hf.hf_histogram(codes, A, nslabs=S, slab_hist=sh_h, ws=ws, status=status)
    assert torch.equal(hist, hist3) and torch.equal(sh_f, sh_h)
    book = hf.hf_build_codebook(hist, ws=ws, status=status)
    out1, off1 = hf.hf_encode(codes, book, chunk, ws=ws, status=status, nslabs=S, slab_hist=sh_f)
    out1, off1 = out1.clone(), off1.clone()
    out2, off2 = hf.hf_encode(codes, book, chunk, ws=ws, status=status, nslabs=S, slab_hist=sh_h)
    assert hf.read_status(status) == 0
    assert torch.equal(off1, off2)
    nwords = (int(off1[-1]) + 31) // 32
    assert torch.equal(out1[:nwords], out2[:nwords])
    dec = hf.hf_decode(out1, off1, n, torch.int16, chunk, book)
    want = lz.lorenzo_codes(x, inv, 512)
    assert np.array_equal(dec.cpu().numpy().view(np.uint16), want)


def test_full_size_benchmark_field():
    """The 512^3 field of the benchmark, in the launch configuration the
    benchmark uses (per-slab counts, the encoder's slab count), compared
    whole."""
    x, eb = W.lorenzo_field(dim=512, seed=0)
    inv = _inv(eb)
    S = hf.hf_slab_count(x.size, 1024)
    check(x, inv, 512, nslabs=S)
