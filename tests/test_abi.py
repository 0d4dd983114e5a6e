"""Host-side checks of libhf that need no GPU: the library loads, exports
every entry point include/hf.h declares, rejects bad arguments before any
device work, and implements the paper's reduction-factor rule."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hf.h")
LIB = os.path.join(ROOT, "paper_2010_10039_amd", "libhf.so")


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\*?\s*(hf_[a-z_0-9]+)\s*\(", text, flags=re.M)
    return sorted(set(names))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.fail("libhf.so is not built (python -m paper_2010_10039_amd.build)")
    return ctypes.CDLL(LIB)


def test_header_declares_the_boundary():
    names = _declared_functions()
    for want in ("hf_histogram", "hf_build_codebook", "hf_encode", "hf_decode", "hf_decode_check",
                 "hf_lorenzo_histogram", "hf_workspace_bytes", "hf_decode_workspace_bytes", "hf_bound_words",
                 "hf_encode_noalloc", "hf_encode_batch_persistent"):
        assert want in names


def test_library_exports_every_declared_symbol(lib):
    missing = [n for n in _declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_bound_words(lib):
    lib.hf_bound_words.restype = ctypes.c_uint64
    lib.hf_bound_words.argtypes = [ctypes.c_uint64, ctypes.c_uint32]
    # ceil(log2 A) + 1 bits per symbol, plus one word
    assert lib.hf_bound_words(1 << 20, 1024) == ((1 << 20) * 11 + 31) // 32 + 1
    assert lib.hf_bound_words(100, 256) == (100 * 9 + 31) // 32 + 1
    assert lib.hf_bound_words(7, 1) == (7 + 31) // 32 + 1


def test_workspace_grows_with_n_and_large_alphabets(lib):
    f = lib.hf_workspace_bytes
    f.restype = ctypes.c_size_t
    f.argtypes = [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32]
    assert f(1 << 27, 1024, 4096) > f(1 << 20, 1024, 4096) >= 256
    assert f(1000, 65536, 4096) > f(1000, 1024, 4096)


def test_reduction_factor_rule_matches_table4(lib):
    """floor(log2 beta) + r + 1 = log2 32 (Sec. 4.3).  Table 4 lists the
    average bitwidth and the reduction factor used per dataset; the rule
    reproduces it for the five byte datasets (Nyx-Quant's r = 3 was chosen
    empirically over the rule's 4, Sec. 4.3 / Table 3)."""
    lib.hf_reduction_factor.restype = ctypes.c_uint32
    lib.hf_reduction_factor.argtypes = [ctypes.c_double]
    table4 = [(5.1639, 2), (5.2124, 2), (4.0165, 2), (2.7307, 3), (4.1428, 2)]
    for beta, r in table4:
        assert lib.hf_reduction_factor(beta) == r
    assert lib.hf_reduction_factor(1.0272) == 4
    assert lib.hf_reduction_factor(40.0) == 1  # clamped


def test_host_argument_checks_return_before_device_work(lib):
    P = ctypes.c_void_p
    U32, U64, SZ = ctypes.c_uint32, ctypes.c_uint64, ctypes.c_size_t
    lib.hf_histogram.argtypes = [P, U64, U32, U32, P, U32, P, P, SZ, P, P]
    d = P(0x1000)
    # sym_bytes 3, alphabet 0, uint8 with alphabet > 256, n >= 2^32
    assert lib.hf_histogram(d, 10, 3, 16, d, 0, None, None, 0, d, None) == 1
    assert lib.hf_histogram(d, 10, 2, 0, d, 0, None, None, 0, d, None) == 1
    assert lib.hf_histogram(d, 10, 1, 300, d, 0, None, None, 0, d, None) == 1
    assert lib.hf_histogram(d, 1 << 32, 2, 16, d, 0, None, None, 0, d, None) == 1
    # misaligned 16-bit symbols
    assert lib.hf_histogram(P(0x1001), 10, 2, 16, d, 0, None, None, 0, d, None) == 1
    # per-slab counts: need 1 <= nslabs <= blocks and alphabet <= 4096
    assert lib.hf_histogram(d, 10_000, 2, 16, d, 0, d, None, 0, d, None) == 1
    assert lib.hf_histogram(d, 10_000, 2, 16, d, 4, d, None, 0, d, None) == 1
    assert lib.hf_histogram(d, 10_000, 2, 8192, d, 2, d, None, 0, d, None) == 1
    lib.hf_status_string.restype = ctypes.c_char_p
    assert b"argument" in lib.hf_status_string(1)


class _Book(ctypes.Structure):
    _fields_ = [("alphabet", ctypes.c_uint32)] + [(k, ctypes.c_void_p) for k in ("cl", "cw", "first", "entry", "rev",
                                                                                 "info")]


def test_decoder_argument_checks(lib):
    P = ctypes.c_void_p
    U32, U64, SZ = ctypes.c_uint32, ctypes.c_uint64, ctypes.c_size_t
    lib.hf_decode.argtypes = [P, P, U64, U32, U32, ctypes.POINTER(_Book), P, P, SZ, P, P]
    lib.hf_decode_workspace_bytes.restype = SZ
    need = lib.hf_decode_workspace_bytes()
    assert need == 4 << 12
    d, ws = P(0x1000), P(0x100000)
    book = _Book(1024, *([0x2000] * 6))
    # chunk not a power of two / out of range, bad width, missing buffers
    assert lib.hf_decode(d, d, 100, 2, 1000, ctypes.byref(book), d, ws, need, d, None) == 1
    assert lib.hf_decode(d, d, 100, 2, 128, ctypes.byref(book), d, ws, need, d, None) == 1
    assert lib.hf_decode(d, d, 100, 3, 4096, ctypes.byref(book), d, ws, need, d, None) == 1
    assert lib.hf_decode(d, d, 100, 2, 4096, ctypes.byref(book), None, ws, need, d, None) == 1
    assert lib.hf_decode(d, None, 100, 2, 4096, ctypes.byref(book), d, ws, need, d, None) == 1
    # workspace missing, too small, misaligned
    assert lib.hf_decode(d, d, 100, 2, 4096, ctypes.byref(book), d, None, need, d, None) == 2
    assert lib.hf_decode(d, d, 100, 2, 4096, ctypes.byref(book), d, ws, need - 1, d, None) == 2
    assert lib.hf_decode(d, d, 100, 2, 4096, ctypes.byref(book), d, P(0x100004), need, d, None) == 2
    lib.hf_status_string.restype = ctypes.c_char_p
    assert b"decode" in lib.hf_status_string(21)


def test_front_end_argument_checks(lib):
    P = ctypes.c_void_p
    U32, F = ctypes.c_uint32, ctypes.c_float
    f = lib.hf_lorenzo_histogram
    f.argtypes = [P, U32, U32, U32, F, U32, P, P, U32, P, P, P]
    x, c, h, sh, st = P(0x10000), P(0x20000), P(0x30000), P(0x40000), P(0x50000)
    ok = dict(x=x, nz=8, ny=16, nx=512, r=100.0, radius=512, c=c, h=h, s=0, sh=None, st=st)

    def call(**kw):
        a = dict(ok, **kw)
        return f(a["x"], a["nz"], a["ny"], a["nx"], a["r"], a["radius"], a["c"], a["h"], a["s"], a["sh"], a["st"],
                 None)

    assert call(st=None) == 1                                              # the status word is required
    assert call(radius=0) == 1 and call(radius=8193) == 1
    assert call(r=0.0) == 1 and call(r=-1.0) == 1 and call(r=float("inf")) == 1 and call(r=float("nan")) == 1
    assert call(h=None) == 1 and call(x=None) == 1 and call(c=None) == 1
    assert call(x=P(0x10002)) == 1 and call(c=P(0x20001)) == 1            # misaligned
    assert call(nz=1 << 12, ny=1 << 10, nx=1 << 10) == 1                   # n = 2^32
    assert call(nz=1, ny=2, nx=8193) == 1                                  # row longer than the LDS ring
    assert call(sh=sh, s=0) == 1 and call(sh=sh, s=17) == 1                # 16 blocks of 4096
    assert call(sh=sh, s=4, radius=4096) == 1                              # alphabet 8192 > 4096 with slabs


def test_paper_format_argument_checks(lib):
    P = ctypes.c_void_p
    U32, U64, SZ = ctypes.c_uint32, ctypes.c_uint64, ctypes.c_size_t
    f = lib.hf_encode_paper
    f.argtypes = [P, U64, U32, ctypes.POINTER(_Book), U32, U32, P, U64, P, P, P, U64, P, P, SZ, P, P]
    lib.hf_paper_workspace_bytes.argtypes = [U64, U32]
    lib.hf_paper_workspace_bytes.restype = SZ
    need = lib.hf_paper_workspace_bytes(100000, 10)
    assert need >= ((100000 + 1023) // 1024) * 16 and lib.hf_paper_workspace_bytes(100000, 13) == 0
    d, ws = P(0x1000), P(0x100000)
    book = _Book(1024, *([0x2000] * 6))

    def call(M=10, r=3, sb=2, cap=10, bg=d, bs=d, w=ws, nbytes=need, sym=d):
        return f(sym, 100000, sb, ctypes.byref(book), M, r, d, 100000, d, bg, bs, cap, d, w, nbytes, d, None)

    assert call(M=7) == 1 and call(M=13) == 1 and call(r=0) == 1 and call(r=6) == 1
    assert call(sb=3) == 1 and call(sym=P(0x1001)) == 1 and call(bg=None) == 1 and call(bs=None) == 1
    assert call(w=None) == 2 and call(nbytes=need - 1) == 2 and call(w=P(0x100010)) == 2


def test_slab_count_bounds(lib):
    lib.hf_slab_count.restype = ctypes.c_uint32
    lib.hf_slab_count.argtypes = [ctypes.c_uint64, ctypes.c_uint32]
    assert lib.hf_slab_count(0, 1024) == 0
    assert lib.hf_slab_count(1 << 20, 65536) == 0  # no per-slab counts for large alphabets
    assert 1 <= lib.hf_slab_count(5000, 1024) <= 2  # at most one slab per 4096-symbol block
    assert 1 <= lib.hf_slab_count(1 << 27, 1024) <= (1 << 27) // 4096


def test_batch_descriptor_checks(lib):
    """hf_batch_workspace_bytes is 0 for an invalid descriptor, and
    hf_encode_batch rejects it before launching anything."""
    from paper_2010_10039_amd import hf

    def desc(**kw):
        d = hf.hf_stream_desc()
        d.sym, d.n, d.sym_bytes, d.chunk_symbols = 0x1000, 1000, 2, 4096
        d.hist, d.out, d.out_capacity_words, d.chunk_bit_offsets = 0, 0x2000, 1000, 0x3000
        b = hf.hf_codebook()
        b.alphabet = 1024
        b.cl = b.cw = b.first = b.entry = b.rev = b.info = 0x4000
        d.book = b
        for k, v in kw.items():
            if k == "alphabet":
                d.book.alphabet = v
            else:
                setattr(d, k, v)
        return d

    f = lib.hf_batch_workspace_bytes
    f.restype = ctypes.c_size_t
    f.argtypes = [ctypes.POINTER(hf.hf_stream_desc), ctypes.c_uint32]
    ok = (hf.hf_stream_desc * 2)(desc(), desc(n=5_000_000, sym_bytes=1, alphabet=256, reduce_log2=3))
    assert f(ok, 2) >= 256
    bad = [dict(alphabet=8193), dict(sym_bytes=1, alphabet=300), dict(chunk_symbols=1000),
           dict(chunk_symbols=128), dict(reduce_log2=2), dict(reduce_log2=6), dict(reserved=1),
           dict(n=1 << 32), dict(sym=0x1001), dict(chunk_bit_offsets=0)]
    g = lib.hf_encode_batch
    g.restype = ctypes.c_int
    g.argtypes = [ctypes.POINTER(hf.hf_stream_desc), ctypes.c_uint32, ctypes.c_void_p, ctypes.c_size_t,
                  ctypes.c_void_p, ctypes.c_void_p]
    for kw in bad:
        arr = (hf.hf_stream_desc * 2)(desc(), desc(**kw))
        assert f(arr, 2) == 0, kw
        assert g(arr, 2, ctypes.c_void_p(0x10000), 1 << 20, ctypes.c_void_p(0x20000), None) == 1, kw


def test_binding_refuses_host_tensors():
    """The Python binding passes device addresses only: a host tensor is
    refused before any library call (its address would be dereferenced by a
    kernel)."""
    torch = pytest.importorskip("torch")
    from paper_2010_10039_amd import hf

    x = torch.zeros(1000, dtype=torch.int16)
    with pytest.raises(ValueError, match="GPU tensors only"):
        hf._dptr(x)
    with pytest.raises(ValueError, match="GPU tensors only"):
        hf.hf_histogram(x, 1024, status=torch.zeros(1, dtype=torch.int32))


def test_codebook_argument_checks(lib):
    """hf_build_codebook and its traced variant reject bad arguments before
    any device work; alphabets above 4096 need the workspace, and above 8192
    the larger one of the grid-wide steps."""
    P, SZ = ctypes.c_void_p, ctypes.c_size_t
    for f in (lib.hf_build_codebook, lib.hf_build_codebook_traced):
        traced = f is lib.hf_build_codebook_traced
        f.argtypes = [P, ctypes.POINTER(_Book), P, SZ, P] + ([P] if traced else []) + [P]

        def call(hist, book, ws, ws_bytes, status, stamps=P(0x9000)):
            args = [hist, ctypes.byref(book), ws, ws_bytes, status] + ([stamps] if traced else []) + [None]
            return f(*args)

        d, ws = P(0x1000), P(0x100000)
        assert call(None, _Book(1024, *([0x2000] * 6)), None, 0, d) == 1       # no histogram
        assert call(d, _Book(0, *([0x2000] * 6)), None, 0, d) == 1             # alphabet 0
        assert call(d, _Book(65537, *([0x2000] * 6)), None, 0, d) == 1         # alphabet > 65536
        assert call(d, _Book(1024, *([0x2000] * 6)), None, 0, None) == 1       # no status word
        assert call(d, _Book(8192, *([0x2000] * 6)), None, 0, d) == 2          # tree in the workspace
        lib.hf_workspace_bytes.restype = SZ
        lib.hf_workspace_bytes.argtypes = [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32]
        small, big = lib.hf_workspace_bytes(1, 8192, 4096), lib.hf_workspace_bytes(1, 65536, 4096)
        assert big > small > 0
        assert call(d, _Book(65536, *([0x2000] * 6)), ws, big - 256, d) == 2  # too small for the grid-wide steps
        assert call(d, _Book(65536, *([0x2000] * 6)), P(0x100004), big, d) == 2  # misaligned
        if traced:
            assert call(d, _Book(1024, *([0x2000] * 6)), None, 0, d, stamps=None) == 1  # no stamp array
