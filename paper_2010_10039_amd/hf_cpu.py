"""Python binding of libhf_cpu (include/hf_cpu.h): the multi-core CPU
histogram, parallel codebook and encoder, on numpy arrays.  Argument
marshalling only; raises ImportError if the library is not built."""
from __future__ import annotations

import ctypes
import os

import numpy as np

_LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libhf_cpu.so")
if not os.path.exists(_LIB_PATH):
    raise ImportError(f"{_LIB_PATH} is not built; run `python -m paper_2010_10039_amd.build`")
_lib = ctypes.CDLL(_LIB_PATH)

_P, _U32, _U64, _I = ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int
_lib.hfc_threads.argtypes = [_I]
_lib.hfc_threads.restype = _I
_lib.hfc_histogram.argtypes = [_P, _U64, _U32, _U32, _P, _I]
_lib.hfc_histogram.restype = _I
_lib.hfc_codebook.argtypes = [_P, _U32, _P, _P, _P, _P, _P, _P, _I]
_lib.hfc_codebook.restype = _I
_lib.hfc_encode.argtypes = [_P, _U64, _U32, _U32, _P, _P, _U32, _P, _U64, _P, _I]
_lib.hfc_encode.restype = _I

MAXLEN = 64


class HFCError(RuntimeError):
    def __init__(self, code: int, where: str):
        super().__init__(f"{where}: status {code}")
        self.code = code


def _p(a: np.ndarray):
    return ctypes.c_void_p(a.ctypes.data)


def _sb(x: np.ndarray) -> int:
    if x.dtype == np.uint8:
        return 1
    if x.dtype == np.uint16:
        return 2
    raise TypeError(f"symbols must be uint8 or uint16, got {x.dtype}")


def threads(nthreads: int = 0) -> int:
    return int(_lib.hfc_threads(nthreads))


def histogram(x: np.ndarray, alphabet: int, nthreads: int = 0) -> np.ndarray:
    x = np.ascontiguousarray(x)
    h = np.empty(alphabet, dtype=np.uint32)
    rc = _lib.hfc_histogram(_p(x), x.size, _sb(x), alphabet, _p(h), nthreads)
    if rc:
        raise HFCError(rc, "hfc_histogram")
    return h


def codebook(hist: np.ndarray, nthreads: int = 0) -> dict:
    """Returns dict(cl, cw, first, entry, rev, info) as numpy arrays; rev
    entries [m, alphabet) are 0xFFFFFFFF."""
    h = np.ascontiguousarray(hist, dtype=np.uint32)
    A = h.size
    out = dict(cl=np.empty(A, np.uint8), cw=np.empty(A, np.uint64), first=np.empty(MAXLEN + 1, np.uint64),
               entry=np.empty(MAXLEN + 1, np.uint32), rev=np.full(A, 0xFFFFFFFF, np.uint32),
               info=np.empty(4, np.uint64))
    rc = _lib.hfc_codebook(_p(h), A, _p(out["cl"]), _p(out["cw"]), _p(out["first"]), _p(out["entry"]),
                           _p(out["rev"]), _p(out["info"]), nthreads)
    if rc:
        raise HFCError(rc, "hfc_codebook")
    return out


def encode(x: np.ndarray, cl: np.ndarray, cw: np.ndarray, chunk: int, cap_words: int | None = None,
           nthreads: int = 0):
    """Returns (words, chunk bit offsets, total bits)."""
    x = np.ascontiguousarray(x)
    cl = np.ascontiguousarray(cl, dtype=np.uint8)
    cw = np.ascontiguousarray(cw, dtype=np.uint64)
    nch = (x.size + chunk - 1) // chunk
    if cap_words is None:
        cap_words = (x.size * MAXLEN + 31) // 32 if x.size * MAXLEN < (1 << 31) else \
            (int(cl.astype(np.uint64)[x].sum()) + 31) // 32
    out = np.empty(max(1, cap_words), dtype=np.uint32)
    offs = np.empty(nch + 1, dtype=np.uint64)
    rc = _lib.hfc_encode(_p(x), x.size, _sb(x), cl.size, _p(cl), _p(cw), chunk, _p(out), cap_words, _p(offs),
                         nthreads)
    if rc:
        raise HFCError(rc, "hfc_encode")
    tb = int(offs[-1])
    return out[: (tb + 31) // 32], offs, tb
