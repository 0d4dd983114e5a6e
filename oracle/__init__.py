"""CPU oracle for the Huffman encoding path -- TEST INFRASTRUCTURE ONLY.

Thin numpy wrapper over ``huff_oracle.c``: a plain serial C implementation
of what the path computes (histogram, heap-built Huffman code lengths,
canonical codewords with First/Entry tables, serial bit packing, treeless
decoding).  Each routine cites the part of Tian et al., arXiv 2010.10039,
it follows; see the C file's header.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  It imports nothing from the GPU
library and the GPU library imports nothing from it.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "huff_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

OK = 0
ERR_ARG = 1
ERR_SYMBOL = 16
ERR_CAPACITY = 17
ERR_CODELEN = 18
MAXLEN = 64


def build(force: bool = True) -> str:
    """Compile ``huff_oracle.c`` into ``liboracle.so`` with gcc."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.run(
            ["gcc", "-O2", "-std=c99", "-Wall", "-Wextra", "-shared", "-fPIC", _SRC, "-o", tmp],
            check=True,
        )
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        U64 = ctypes.c_uint64
        U32 = ctypes.c_uint32
        I = ctypes.c_int
        lib.oracle_histogram.argtypes = [P, U64, I, U32, P]
        lib.oracle_code_lengths.argtypes = [P, U32, P, P]
        lib.oracle_canonical.argtypes = [P, U32, P, P, P, P, P]
        lib.oracle_codebook.argtypes = [P, U32, P, P, P, P, P, P]
        lib.oracle_encode.argtypes = [P, U64, I, U32, P, P, U64, P, U64, P, P]
        lib.oracle_decode.argtypes = [P, U64, U64, U64, P, P, P, U32, U32, I, P, P]
        for f in (lib.oracle_histogram, lib.oracle_code_lengths, lib.oracle_canonical,
                  lib.oracle_codebook, lib.oracle_encode, lib.oracle_decode):
            f.restype = ctypes.c_int
        _lib = lib
    return _lib


class OracleError(RuntimeError):
    def __init__(self, code: int, what: str):
        super().__init__(f"{what}: oracle error {code}")
        self.code = code


def _ptr(a: np.ndarray):
    return ctypes.c_void_p(a.ctypes.data)


def _sym_bytes(x: np.ndarray) -> int:
    if x.dtype == np.uint8:
        return 1
    if x.dtype == np.uint16:
        return 2
    raise TypeError(f"symbols must be uint8 or uint16, got {x.dtype}")


def histogram(x: np.ndarray, alphabet: int) -> np.ndarray:
    """h[s] = number of occurrences of s in x (Sec. 4.1)."""
    x = np.ascontiguousarray(x)
    h = np.zeros(alphabet, dtype=np.uint32)
    rc = _load().oracle_histogram(_ptr(x), x.size, _sym_bytes(x), alphabet, _ptr(h))
    if rc:
        raise OracleError(rc, "histogram")
    return h


def code_lengths(h: np.ndarray) -> tuple[np.ndarray, int]:
    """Huffman code lengths under the (weight, leaf-first, rank) tie-break.

    Returns (cl, sum of internal node weights)."""
    h = np.ascontiguousarray(h, dtype=np.uint32)
    cl = np.zeros(h.size, dtype=np.uint8)
    ws = np.zeros(1, dtype=np.uint64)
    rc = _load().oracle_code_lengths(_ptr(h), h.size, _ptr(cl), _ptr(ws))
    if rc:
        raise OracleError(rc, "code_lengths")
    return cl, int(ws[0])


@dataclass
class Codebook:
    cl: np.ndarray     # uint8[A]
    cw: np.ndarray     # uint64[A]
    first: np.ndarray  # uint64[65]
    entry: np.ndarray  # uint32[65]
    rev: np.ndarray    # uint32[A]; entries [m, A) unspecified
    info: np.ndarray   # uint64[4] = m, Lmax, total_bits, min_len

    @property
    def m(self) -> int:
        return int(self.info[0])

    @property
    def lmax(self) -> int:
        return int(self.info[1])

    @property
    def total_bits(self) -> int:
        return int(self.info[2])


def canonical(cl: np.ndarray) -> Codebook:
    """Canonical codewords and First/Entry tables from code lengths (Sec. 4.2.2)."""
    cl = np.ascontiguousarray(cl, dtype=np.uint8)
    A = cl.size
    cw = np.zeros(A, dtype=np.uint64)
    first = np.zeros(MAXLEN + 1, dtype=np.uint64)
    entry = np.zeros(MAXLEN + 1, dtype=np.uint32)
    rev = np.full(A, 0xFFFFFFFF, dtype=np.uint32)
    info = np.zeros(4, dtype=np.uint64)
    rc = _load().oracle_canonical(_ptr(cl), A, _ptr(cw), _ptr(first), _ptr(entry), _ptr(rev), _ptr(info))
    if rc:
        raise OracleError(rc, "canonical")
    return Codebook(cl, cw, first, entry, rev, info)


def codebook(h: np.ndarray) -> Codebook:
    """Code lengths + canonical codes + total bits = sum h*cl."""
    h = np.ascontiguousarray(h, dtype=np.uint32)
    A = h.size
    cl = np.zeros(A, dtype=np.uint8)
    cw = np.zeros(A, dtype=np.uint64)
    first = np.zeros(MAXLEN + 1, dtype=np.uint64)
    entry = np.zeros(MAXLEN + 1, dtype=np.uint32)
    rev = np.full(A, 0xFFFFFFFF, dtype=np.uint32)
    info = np.zeros(4, dtype=np.uint64)
    rc = _load().oracle_codebook(_ptr(h), A, _ptr(cl), _ptr(cw), _ptr(first), _ptr(entry),
                                 _ptr(rev), _ptr(info))
    if rc:
        raise OracleError(rc, "codebook")
    return Codebook(cl, cw, first, entry, rev, info)


def bound_words(total_bits: int) -> int:
    return (total_bits + 31) // 32


def encode(x: np.ndarray, book: Codebook, chunk: int) -> tuple[np.ndarray, np.ndarray, int]:
    """Serial bit packing (Sec. 4.3).  Returns (words, chunk offsets, total bits)."""
    x = np.ascontiguousarray(x)
    n = x.size
    nch = (n + chunk - 1) // chunk
    # capacity: exact size from the lengths (sum of cl over x), computed plainly
    total = int(book.cl.astype(np.uint64)[x].sum()) if n else 0
    cap = max(1, bound_words(total))
    out = np.zeros(cap, dtype=np.uint32)
    offsets = np.zeros(nch + 1, dtype=np.uint64)
    tb = np.zeros(1, dtype=np.uint64)
    rc = _load().oracle_encode(_ptr(x), n, _sym_bytes(x), book.cl.size, _ptr(book.cl), _ptr(book.cw),
                               chunk, _ptr(out), cap, _ptr(offsets), _ptr(tb))
    if rc:
        raise OracleError(rc, "encode")
    return out[: bound_words(int(tb[0]))], offsets, int(tb[0])


def decode(words: np.ndarray, nbits: int, n: int, book: Codebook, dtype=np.uint16,
           start: int = 0) -> tuple[np.ndarray, int]:
    """Treeless canonical decoding (Sec. 4.2.2).  Returns (symbols, end bit)."""
    words = np.ascontiguousarray(words, dtype=np.uint32)
    if words.size == 0:
        words = np.zeros(1, dtype=np.uint32)
    out = np.zeros(n, dtype=dtype)
    end = np.zeros(1, dtype=np.uint64)
    rc = _load().oracle_decode(_ptr(words), start, nbits, n, _ptr(book.first), _ptr(book.entry),
                               _ptr(book.rev), book.m, book.lmax, _sym_bytes(out), _ptr(out), _ptr(end))
    if rc:
        raise OracleError(rc, "decode")
    return out, int(end[0])
