"""Python binding of libhf (include/hf.h): argument marshalling only.

Every function here has the name of the C entry point it calls.  Device
buffers are torch tensors on a ROCm device; calls enqueue work on torch's
current stream and return without synchronizing.  Every step of the encoding
runs in the HIP kernels of libhf.so; if the library is not built, importing
this module raises.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import torch

_LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libhf.so")

HF_OK = 0
HF_ERR_ARG = 1
HF_ERR_WORKSPACE = 2
HF_ERR_LAUNCH = 3
HF_ERR_SYMBOL = 16
HF_ERR_CAPACITY = 17
HF_ERR_CODELEN = 18
HF_ERR_MISMATCH = 19
HF_ERR_INTERNAL = 20
HF_ERR_STREAM = 21
HF_ERR_VALUE = 22
MAX_CODELEN = 64

if not os.path.exists(_LIB_PATH):
    raise ImportError(
        f"{_LIB_PATH} is not built; run `python -m paper_2010_10039_amd.build` "
        "(the encoder has no CPU fallback)")

_lib = ctypes.CDLL(_LIB_PATH)


class hf_codebook(ctypes.Structure):
    _fields_ = [
        ("alphabet", ctypes.c_uint32),
        ("cl", ctypes.c_void_p),
        ("cw", ctypes.c_void_p),
        ("first", ctypes.c_void_p),
        ("entry", ctypes.c_void_p),
        ("rev", ctypes.c_void_p),
        ("info", ctypes.c_void_p),
    ]


_P = ctypes.c_void_p
_U32 = ctypes.c_uint32
_U64 = ctypes.c_uint64
_SZ = ctypes.c_size_t

_lib.hf_workspace_bytes.argtypes = [_U64, _U32, _U32]
_lib.hf_workspace_bytes.restype = _SZ
_lib.hf_bound_words.argtypes = [_U64, _U32]
_lib.hf_bound_words.restype = _U64
_lib.hf_reduction_factor.argtypes = [ctypes.c_double]
_lib.hf_reduction_factor.restype = _U32
_lib.hf_status_string.argtypes = [_U32]
_lib.hf_status_string.restype = ctypes.c_char_p
_lib.hf_time_next_main_kernel.argtypes = [_P, _P]
_lib.hf_time_next_main_kernel.restype = ctypes.c_int
_lib.hf_slab_count.argtypes = [_U64, _U32]
_lib.hf_slab_count.restype = _U32
_lib.hf_histogram.argtypes = [_P, _U64, _U32, _U32, _P, _U32, _P, _P, _SZ, _P, _P]
_lib.hf_histogram.restype = ctypes.c_int
_lib.hf_build_codebook.argtypes = [_P, ctypes.POINTER(hf_codebook), _P, _SZ, _P, _P]
_lib.hf_build_codebook.restype = ctypes.c_int
_lib.hf_build_codebook_traced.argtypes = [_P, ctypes.POINTER(hf_codebook), _P, _SZ, _P, _P, _P]
_lib.hf_build_codebook_traced.restype = ctypes.c_int
_lib.hf_encode.argtypes = [_P, _U64, _U32, ctypes.POINTER(hf_codebook), _U32, _U32, _U32, _P, _P, _U64,
                           _P, _P, _SZ, _P, _P]
_lib.hf_encode.restype = ctypes.c_int
_lib.hf_encode_noalloc.argtypes = [_P, _U64, _U32, ctypes.POINTER(hf_codebook), _U32, _U32, _U32, _P, _P, _U64,
                                   _P, _P, _P]
_lib.hf_encode_noalloc.restype = ctypes.c_int
_lib.hf_decode_check.argtypes = [_P, _P, _U64, _U32, _U32, ctypes.POINTER(hf_codebook), _P, _P, _P, _P]
_lib.hf_decode_check.restype = ctypes.c_int
_lib.hf_lorenzo_histogram.argtypes = [_P, _U32, _U32, _U32, ctypes.c_float, _U32, _P, _P, _U32, _P, _P, _P]
_lib.hf_lorenzo_histogram.restype = ctypes.c_int
_lib.hf_paper_workspace_bytes.argtypes = [_U64, _U32]
_lib.hf_paper_workspace_bytes.restype = _SZ
_lib.hf_encode_paper.argtypes = [_P, _U64, _U32, ctypes.POINTER(hf_codebook), _U32, _U32, _P, _U64, _P, _P, _P,
                                 _U64, _P, _P, _SZ, _P, _P]
_lib.hf_encode_paper.restype = ctypes.c_int
_lib.hf_decode_workspace_bytes.argtypes = []
_lib.hf_decode_workspace_bytes.restype = _SZ
_lib.hf_decode.argtypes = [_P, _P, _U64, _U32, _U32, ctypes.POINTER(hf_codebook), _P, _P, _SZ, _P, _P]
_lib.hf_decode.restype = ctypes.c_int


class HFError(RuntimeError):
    def __init__(self, code: int, where: str):
        super().__init__(f"{where}: {hf_status_string(code)} ({code})")
        self.code = code


def library_path() -> str:
    return _LIB_PATH


def hf_status_string(code: int) -> str:
    return _lib.hf_status_string(code).decode()


def _check(rc: int, where: str) -> None:
    if rc != HF_OK:
        raise HFError(rc, where)


def _stream() -> ctypes.c_void_p:
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dptr(t: torch.Tensor) -> int:
    """Device address of a GPU tensor; host tensors are refused here, since
    the kernels would dereference their addresses on the device."""
    if not t.is_cuda:
        raise ValueError(f"libhf takes GPU tensors only, got a {t.device} tensor of shape {tuple(t.shape)}")
    return t.data_ptr()


def _ptr(t: torch.Tensor | None) -> ctypes.c_void_p:
    return ctypes.c_void_p(0 if t is None else _dptr(t))


def _sym_bytes(sym: torch.Tensor) -> int:
    if sym.element_size() not in (1, 2) or sym.is_floating_point():
        raise TypeError(f"symbols must be 8- or 16-bit integers, got {sym.dtype}")
    if not sym.is_contiguous():
        raise ValueError("symbols must be contiguous")
    return sym.element_size()


def hf_workspace_bytes(n: int, alphabet: int, chunk_symbols: int = 4096) -> int:
    return int(_lib.hf_workspace_bytes(n, alphabet, chunk_symbols))


def hf_bound_words(n: int, alphabet: int) -> int:
    return int(_lib.hf_bound_words(n, alphabet))


def hf_slab_count(n: int, alphabet: int) -> int:
    return int(_lib.hf_slab_count(n, alphabet))


def hf_reduction_factor(beta: float) -> int:
    return int(_lib.hf_reduction_factor(beta))


def hf_time_next_main_kernel(before: torch.cuda.Event | None, after: torch.cuda.Event | None) -> None:
    """Arm the one-shot timer around the next call's main kernel (this thread)."""
    b = ctypes.c_void_p(before.cuda_event) if before is not None else ctypes.c_void_p(0)
    a = ctypes.c_void_p(after.cuda_event) if after is not None else ctypes.c_void_p(0)
    _check(_lib.hf_time_next_main_kernel(b, a), "hf_time_next_main_kernel")


def new_status(device=None) -> torch.Tensor:
    return torch.zeros(1, dtype=torch.int32, device=device or "cuda")


def new_workspace(n: int, alphabet: int, chunk_symbols: int = 4096, device=None) -> torch.Tensor:
    nbytes = hf_workspace_bytes(n, alphabet, chunk_symbols)
    return torch.empty(nbytes, dtype=torch.uint8, device=device or "cuda")


def read_status(status: torch.Tensor) -> int:
    """Synchronizes with the stream and returns the device status word."""
    return int(status.item())


def raise_on_status(status: torch.Tensor, where: str = "device") -> None:
    code = read_status(status)
    if code != HF_OK:
        raise HFError(code, where)


@dataclass
class Codebook:
    """Device arrays of one codebook (see hf_codebook in include/hf.h)."""

    alphabet: int
    cl: torch.Tensor      # uint8[A]
    cw: torch.Tensor      # int64[A] (bit pattern of uint64)
    first: torch.Tensor   # int64[65]
    entry: torch.Tensor   # int32[65]
    rev: torch.Tensor     # int32[A]
    info: torch.Tensor    # int64[4]: m, Lmax, total_bits, min_len

    @staticmethod
    def empty(alphabet: int, device=None) -> "Codebook":
        d = device or "cuda"
        return Codebook(
            alphabet,
            torch.zeros(alphabet, dtype=torch.uint8, device=d),
            torch.zeros(alphabet, dtype=torch.int64, device=d),
            torch.zeros(MAX_CODELEN + 1, dtype=torch.int64, device=d),
            torch.zeros(MAX_CODELEN + 1, dtype=torch.int32, device=d),
            torch.zeros(alphabet, dtype=torch.int32, device=d),
            torch.zeros(4, dtype=torch.int64, device=d),
        )

    def struct(self) -> hf_codebook:
        return hf_codebook(self.alphabet, _dptr(self.cl), _dptr(self.cw), _dptr(self.first), _dptr(self.entry),
                           _dptr(self.rev), _dptr(self.info))


def hf_histogram(sym: torch.Tensor, alphabet: int, hist: torch.Tensor | None = None,
                 nslabs: int = 0, slab_hist: torch.Tensor | None = None,
                 ws: torch.Tensor | None = None, status: torch.Tensor | None = None) -> torch.Tensor:
    """Histogram of `sym`; with `slab_hist` (int32[nslabs * alphabet]) also
    the per-slab counts for hf_encode."""
    sb = _sym_bytes(sym)
    if hist is None:
        hist = torch.empty(alphabet, dtype=torch.int32, device=sym.device)
    if status is None:
        status = new_status(sym.device)
    _check(_lib.hf_histogram(_ptr(sym), sym.numel(), sb, alphabet, _ptr(hist), nslabs, _ptr(slab_hist),
                             _ptr(ws), 0 if ws is None else ws.numel(), _ptr(status), _stream()),
           "hf_histogram")
    return hist


def hf_lorenzo_histogram(field: torch.Tensor, dims, inv_2eb: float, radius: int,
                         codes: torch.Tensor | None = None, hist: torch.Tensor | None = None,
                         nslabs: int = 0, slab_hist: torch.Tensor | None = None,
                         status: torch.Tensor | None = None):
    """Quantization codes (int16 tensor holding uint16) of the float32 field
    of shape dims = (nz, ny, nx) and their histogram (int32[2 radius]); with
    `slab_hist` (int32[nslabs * 2 radius]) also the per-slab counts for
    hf_encode.  A NaN or infinite value raises HF_ERR_VALUE in `status`.
    Returns (codes, hist)."""
    if field.dtype != torch.float32 or not field.is_contiguous():
        raise TypeError("the field must be a contiguous float32 tensor")
    nz, ny, nx = (int(v) for v in dims)
    if field.numel() != nz * ny * nx:
        raise ValueError(f"field has {field.numel()} elements, dims {dims} need {nz * ny * nx}")
    if codes is None:
        codes = torch.empty(field.numel(), dtype=torch.int16, device=field.device)
    if hist is None:
        hist = torch.empty(2 * radius, dtype=torch.int32, device=field.device)
    if status is None:
        status = new_status(field.device)
    _check(_lib.hf_lorenzo_histogram(_ptr(field), nz, ny, nx, float(inv_2eb), radius, _ptr(codes), _ptr(hist),
                                     nslabs, _ptr(slab_hist), _ptr(status), _stream()), "hf_lorenzo_histogram")
    return codes, hist


def hf_build_codebook(hist: torch.Tensor, book: Codebook | None = None, ws: torch.Tensor | None = None,
                      status: torch.Tensor | None = None) -> Codebook:
    if book is None:
        book = Codebook.empty(hist.numel(), hist.device)
    if status is None:
        status = new_status(hist.device)
    if ws is None:  # alphabets above 4096 build the tree in device memory
        ws = new_workspace(1, hist.numel(), device=hist.device)
    s = book.struct()
    _check(_lib.hf_build_codebook(_ptr(hist), ctypes.byref(s), _ptr(ws), 0 if ws is None else ws.numel(),
                                  _ptr(status), _stream()), "hf_build_codebook")
    return book


CODEBOOK_PHASES = ("histogram", "compaction", "sort", "rounds", "depths", "lengths", "first_entry", "codewords")


def hf_build_codebook_traced(hist: torch.Tensor, book: Codebook, ws: torch.Tensor, status: torch.Tensor,
                             stamps: torch.Tensor) -> Codebook:
    """hf_build_codebook with the single-workgroup build's phase clocks
    written to `stamps` (int64[9] on the device, zeroed by the caller)."""
    if stamps.dtype != torch.int64 or stamps.numel() < 9:
        raise ValueError("stamps must be an int64 tensor of at least 9 elements")
    s = book.struct()
    _check(_lib.hf_build_codebook_traced(_ptr(hist), ctypes.byref(s), _ptr(ws), ws.numel(), _ptr(status),
                                         _ptr(stamps), _stream()), "hf_build_codebook_traced")
    return book


def hf_encode(sym: torch.Tensor, book: Codebook, chunk_symbols: int = 4096, reduce_log2: int = 0,
              out: torch.Tensor | None = None, offsets: torch.Tensor | None = None,
              ws: torch.Tensor | None = None, status: torch.Tensor | None = None,
              nslabs: int = 0, slab_hist: torch.Tensor | None = None):
    """Returns (out words as int32 tensor, chunk bit offsets as int64 tensor)."""
    sb = _sym_bytes(sym)
    n = sym.numel()
    nch = (n + chunk_symbols - 1) // chunk_symbols
    if out is None:
        out = torch.empty(max(1, hf_bound_words(n, book.alphabet)), dtype=torch.int32, device=sym.device)
    if offsets is None:
        offsets = torch.empty(nch + 1, dtype=torch.int64, device=sym.device)
    if ws is None:
        ws = new_workspace(n, book.alphabet, chunk_symbols, sym.device)
    if status is None:
        status = new_status(sym.device)
    s = book.struct()
    _check(_lib.hf_encode(_ptr(sym), n, sb, ctypes.byref(s), chunk_symbols, reduce_log2, nslabs,
                          _ptr(slab_hist), _ptr(out), out.numel(), _ptr(offsets), _ptr(ws), ws.numel(),
                          _ptr(status), _stream()),
           "hf_encode")
    return out, offsets


def hf_encode_noalloc(sym: torch.Tensor, book: Codebook, out: torch.Tensor, offsets: torch.Tensor,
                      status: torch.Tensor, chunk_symbols: int = 4096, reduce_log2: int = 0, nslabs: int = 0,
                      slab_hist: torch.Tensor | None = None) -> None:
    """hf_encode with the library's fixed device scratch in place of a
    workspace: every buffer is the caller's, nothing is allocated."""
    s = book.struct()
    _check(_lib.hf_encode_noalloc(_ptr(sym), sym.numel(), _sym_bytes(sym), ctypes.byref(s), chunk_symbols,
                                  reduce_log2, nslabs, _ptr(slab_hist), _ptr(out), out.numel(), _ptr(offsets),
                                  _ptr(status), _stream()),
           "hf_encode_noalloc")


def hf_decode_check(out: torch.Tensor, offsets: torch.Tensor, sym: torch.Tensor, chunk_symbols: int,
                    book: Codebook, result: torch.Tensor | None = None,
                    status: torch.Tensor | None = None) -> torch.Tensor:
    """Returns int64[2] = (mismatches, first mismatching index or n)."""
    sb = _sym_bytes(sym)
    if result is None:
        result = torch.empty(2, dtype=torch.int64, device=sym.device)
    if status is None:
        status = new_status(sym.device)
    s = book.struct()
    _check(_lib.hf_decode_check(_ptr(out), _ptr(offsets), sym.numel(), sb, chunk_symbols, ctypes.byref(s),
                                _ptr(sym), _ptr(result), _ptr(status), _stream()), "hf_decode_check")
    return result


def hf_paper_workspace_bytes(n: int, chunk_log2: int) -> int:
    return int(_lib.hf_paper_workspace_bytes(n, chunk_log2))


def hf_encode_paper(sym: torch.Tensor, book: Codebook, chunk_log2: int, reduce_log2: int,
                    out: torch.Tensor | None = None, offsets: torch.Tensor | None = None,
                    break_groups: torch.Tensor | None = None, break_syms: torch.Tensor | None = None,
                    nbreak: torch.Tensor | None = None, ws: torch.Tensor | None = None,
                    status: torch.Tensor | None = None):
    """The paper's format (include/hf.h, hf_encode_paper).  Returns (words,
    chunk word offsets, breaking group indices, their symbols, count), all
    device tensors; the side channel holds break_groups.numel() groups."""
    sb = _sym_bytes(sym)
    n = sym.numel()
    nch = (n + (1 << chunk_log2) - 1) >> chunk_log2
    dev = sym.device
    if out is None:
        out = torch.empty(max(1, n), dtype=torch.int32, device=dev)  # at most 32 bits a symbol
    if offsets is None:
        offsets = torch.empty(nch + 1, dtype=torch.int64, device=dev)
    if break_groups is None:
        break_groups = torch.empty(max(1, (n + (1 << reduce_log2) - 1) >> reduce_log2), dtype=torch.int64,
                                   device=dev)
    if break_syms is None:
        break_syms = torch.empty(break_groups.numel() << reduce_log2, dtype=sym.dtype, device=dev)
    if nbreak is None:
        nbreak = torch.empty(1, dtype=torch.int64, device=dev)
    if ws is None:
        ws = torch.empty(max(256, hf_paper_workspace_bytes(n, chunk_log2)), dtype=torch.uint8, device=dev)
    if status is None:
        status = new_status(dev)
    s = book.struct()
    _check(_lib.hf_encode_paper(_ptr(sym), n, sb, ctypes.byref(s), chunk_log2, reduce_log2, _ptr(out), out.numel(),
                                _ptr(offsets), _ptr(break_groups), _ptr(break_syms), break_groups.numel(),
                                _ptr(nbreak), _ptr(ws), ws.numel(), _ptr(status), _stream()), "hf_encode_paper")
    return out, offsets, break_groups, break_syms, nbreak


def hf_decode_workspace_bytes() -> int:
    return int(_lib.hf_decode_workspace_bytes())


def hf_decode(words: torch.Tensor, offsets: torch.Tensor, n: int, dtype: torch.dtype, chunk_symbols: int,
              book: Codebook, out: torch.Tensor | None = None, ws: torch.Tensor | None = None,
              status: torch.Tensor | None = None) -> torch.Tensor:
    """Decodes n symbols (dtype torch.uint8 or torch.int16 holding uint16)
    from a stream and its chunk offsets; returns `out`."""
    if dtype not in (torch.uint8, torch.int16):
        raise TypeError(f"symbols must be uint8 or int16 (holding uint16), got {dtype}")
    sb = 1 if dtype == torch.uint8 else 2
    if out is None:
        out = torch.empty(n, dtype=dtype, device=words.device)
    if ws is None:
        ws = torch.empty(hf_decode_workspace_bytes(), dtype=torch.uint8, device=words.device)
    if status is None:
        status = new_status(words.device)
    s = book.struct()
    _check(_lib.hf_decode(_ptr(words), _ptr(offsets), n, sb, chunk_symbols, ctypes.byref(s), _ptr(out), _ptr(ws),
                          ws.numel(), _ptr(status), _stream()), "hf_decode")
    return out


class Encoder:
    """Pre-allocated buffers for repeated hist -> codebook -> encode passes
    over streams of exactly `n` symbols (nothing is allocated per call).
    When the alphabet allows it, the histogram pass also records per-slab
    counts that let the encoder place every slab without re-reading the
    input."""

    def __init__(self, n: int, alphabet: int, chunk_symbols: int = 4096, reduce_log2: int = 0,
                 device="cuda", use_slab_hist: bool = True):
        self.n = n
        self.alphabet = alphabet
        self.chunk = chunk_symbols
        self.r = reduce_log2
        self.hist = torch.empty(alphabet, dtype=torch.int32, device=device)
        self.book = Codebook.empty(alphabet, device)
        self.ws = new_workspace(n, alphabet, chunk_symbols, device)
        self.status = new_status(device)
        self.out = torch.empty(max(1, hf_bound_words(n, alphabet)), dtype=torch.int32, device=device)
        self.offsets = torch.empty((n + chunk_symbols - 1) // chunk_symbols + 1, dtype=torch.int64,
                                   device=device)
        self.nslabs = hf_slab_count(n, alphabet) if use_slab_hist else 0
        self.slab_hist = (torch.empty(self.nslabs * alphabet, dtype=torch.int32, device=device)
                          if self.nslabs else None)

    def run(self, sym: torch.Tensor, timers=None):
        """One pass of the whole path.  `timers` (optional) maps 'hist',
        'codebook', 'encode' to (before, after) torch.cuda.Event pairs
        recorded around each stage's main kernel."""
        assert sym.numel() == self.n
        if timers and "hist" in timers:
            hf_time_next_main_kernel(*timers["hist"])
        hf_histogram(sym, self.alphabet, self.hist, self.nslabs, self.slab_hist, self.ws, self.status)
        if timers and "codebook" in timers:
            hf_time_next_main_kernel(*timers["codebook"])
        hf_build_codebook(self.hist, self.book, self.ws, self.status)
        if timers and "encode" in timers:
            hf_time_next_main_kernel(*timers["encode"])
        hf_encode(sym, self.book, self.chunk, self.r, self.out, self.offsets, self.ws, self.status,
                  self.nslabs, self.slab_hist)
        return self.out, self.offsets

    def capture(self, sym: torch.Tensor):
        """One pass of the whole path over `sym` captured as a HIP graph
        (torch.cuda.CUDAGraph): replay() then launches every kernel of the
        pass at once, which removes the per-launch host overhead that bounds
        small streams.  Every kernel writes or clears what it reads (no
        memset nodes), so each replay gives the eager result; the graph
        keeps using this encoder's buffers and `sym`'s storage."""
        assert sym.numel() == self.n
        self.run(sym)  # one eager pass first: one-time host set-up happens outside the capture
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            self.run(sym)
        return g


class hf_stream_desc(ctypes.Structure):
    _fields_ = [
        ("sym", ctypes.c_void_p),
        ("n", ctypes.c_uint64),
        ("sym_bytes", ctypes.c_uint32),
        ("chunk_symbols", ctypes.c_uint32),
        ("reduce_log2", ctypes.c_uint32),
        ("reserved", ctypes.c_uint32),
        ("hist", ctypes.c_void_p),
        ("book", hf_codebook),
        ("out", ctypes.c_void_p),
        ("out_capacity_words", ctypes.c_uint64),
        ("chunk_bit_offsets", ctypes.c_void_p),
    ]


_lib.hf_batch_workspace_bytes.argtypes = [ctypes.POINTER(hf_stream_desc), _U32]
_lib.hf_batch_workspace_bytes.restype = _SZ
_lib.hf_encode_batch.argtypes = [ctypes.POINTER(hf_stream_desc), _U32, _P, _SZ, _P, _P]
_lib.hf_encode_batch.restype = ctypes.c_int
_lib.hf_encode_batch_persistent.argtypes = [ctypes.POINTER(hf_stream_desc), _U32, _P, _SZ, _P, _P]
_lib.hf_encode_batch_persistent.restype = ctypes.c_int


def hf_batch_workspace_bytes(descs) -> int:
    return int(_lib.hf_batch_workspace_bytes(descs, len(descs)))


def hf_encode_batch(descs, ws: torch.Tensor, status: torch.Tensor) -> None:
    """Encode every stream of the ctypes hf_stream_desc array `descs`."""
    _check(_lib.hf_encode_batch(descs, len(descs), _ptr(ws), ws.numel(), _ptr(status), _stream()),
           "hf_encode_batch")


def hf_encode_batch_persistent(descs, ws: torch.Tensor, status: torch.Tensor) -> None:
    """hf_encode_batch in one persistent launch (same arguments, same results)."""
    _check(_lib.hf_encode_batch_persistent(descs, len(descs), _ptr(ws), ws.numel(), _ptr(status), _stream()),
           "hf_encode_batch_persistent")


class BatchEncoder:
    """Buffers for one batch of independent streams encoded by a single
    hf_encode_batch call: per stream a codebook, a histogram, output words
    and chunk offsets; one workspace and one status word per stream."""

    def __init__(self, syms, alphabets, chunk_symbols=4096, reduce_log2=0, device="cuda"):
        self.syms = list(syms)
        n = len(self.syms)
        self.alphabets = list(alphabets)
        chunks = chunk_symbols if isinstance(chunk_symbols, (list, tuple)) else [chunk_symbols] * n
        rs = reduce_log2 if isinstance(reduce_log2, (list, tuple)) else [reduce_log2] * n
        self.chunks = list(chunks)
        self.books, self.hists, self.outs, self.offsets = [], [], [], []
        self.descs = (hf_stream_desc * n)()
        for i, (x, A) in enumerate(zip(self.syms, self.alphabets)):
            sb = _sym_bytes(x)
            book = Codebook.empty(A, device)
            hist = torch.empty(A, dtype=torch.int32, device=device)
            out = torch.empty(max(1, hf_bound_words(x.numel(), A)), dtype=torch.int32, device=device)
            offs = torch.empty((x.numel() + chunks[i] - 1) // chunks[i] + 1, dtype=torch.int64, device=device)
            self.books.append(book)
            self.hists.append(hist)
            self.outs.append(out)
            self.offsets.append(offs)
            d = self.descs[i]
            d.sym = _dptr(x) if x.numel() else 0
            d.n = x.numel()
            d.sym_bytes = sb
            d.chunk_symbols = chunks[i]
            d.reduce_log2 = rs[i]
            d.reserved = 0
            d.hist = _dptr(hist)
            d.book = book.struct()
            d.out = _dptr(out)
            d.out_capacity_words = out.numel()
            d.chunk_bit_offsets = _dptr(offs)
        nbytes = hf_batch_workspace_bytes(self.descs)
        if nbytes == 0:
            raise HFError(HF_ERR_ARG, "BatchEncoder")
        self.ws = torch.empty(nbytes, dtype=torch.uint8, device=device)
        self.status = torch.zeros(n, dtype=torch.int32, device=device)

    def run(self, persistent: bool = False):
        """Encodes the batch: one launch per stage, or one persistent launch."""
        (hf_encode_batch_persistent if persistent else hf_encode_batch)(self.descs, self.ws, self.status)
        return self.outs, self.offsets
