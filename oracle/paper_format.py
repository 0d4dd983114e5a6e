"""CPU oracle of the paper-format encoding -- TEST INFRASTRUCTURE ONLY.

The paper's own output format (Sec. 4.3, Interface ReduceShuffleMerge<M, r>;
Sec. 5.2.2 and Table 3), read as follows (reading R17):

- the stream is cut into chunks of C = 2^M symbols and every chunk into
  groups of G = 2^r consecutive symbols (the last group of the last chunk
  may be short);
- a group's merged word is the concatenation of its codes, MSB first, of
  total length L = sum of its code lengths.  A group with L > 32 bits is a
  "breaking" group: it is filtered out of the stream and kept in a sparse
  side channel (its global group index and its raw symbols), in ascending
  group order;
- a chunk's output is the concatenation, in order, of its non-breaking
  group words, MSB first in 32-bit words, zero-padded to a whole word;
  chunk outputs follow one another word-aligned (the paper's word-aligned
  gathering), and chunk k starts at word offsets[k].

Plain Python over the groups; the codebook (cl, cw) comes from the main
oracle.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this module.
"""
from __future__ import annotations

import numpy as np


def encode(x: np.ndarray, cl: np.ndarray, cw: np.ndarray, M: int, r: int):
    """Returns (words uint32[total], offsets uint64[nchunks + 1],
    break_groups uint64[nbreak], break_syms (x's dtype)[nbreak * 2^r], with
    the symbols of a short last group padded by zeros)."""
    x = np.asarray(x).reshape(-1)
    n = x.size
    C, G = 1 << M, 1 << r
    lens = np.asarray(cl, dtype=np.int64)[x]
    codes = np.asarray(cw, dtype=np.uint64)[x]
    nch = (n + C - 1) // C
    words: list[int] = []
    offsets = [0]
    breaks: list[int] = []
    bsyms: list[np.ndarray] = []
    for k in range(nch):
        acc, nbits = 0, 0  # the chunk's bits as one integer
        lo, hi = k * C, min(n, (k + 1) * C)
        for g0 in range(lo, hi, G):
            g1 = min(hi, g0 + G)
            L = int(lens[g0:g1].sum())
            if L > 32:
                breaks.append(g0 // G)
                s = np.zeros(G, dtype=x.dtype)
                s[: g1 - g0] = x[g0:g1]
                bsyms.append(s)
                continue
            for i in range(g0, g1):
                acc = (acc << int(lens[i])) | int(codes[i])
                nbits += int(lens[i])
        nw = (nbits + 31) // 32
        acc <<= nw * 32 - nbits
        for j in range(nw):
            words.append((acc >> (32 * (nw - 1 - j))) & 0xFFFFFFFF)
        offsets.append(offsets[-1] + nw)
    return (np.array(words, dtype=np.uint32), np.array(offsets, dtype=np.uint64),
            np.array(breaks, dtype=np.uint64),
            np.concatenate(bsyms) if bsyms else np.zeros(0, dtype=x.dtype))


def decode(words: np.ndarray, offsets: np.ndarray, break_groups: np.ndarray, break_syms: np.ndarray, n: int,
           cl: np.ndarray, cw: np.ndarray, M: int, r: int, dtype) -> np.ndarray:
    """Inverse of encode with a code -> symbol dictionary (for round trips)."""
    C, G = 1 << M, 1 << r
    table = {(int(cl[s]), int(cw[s])): s for s in range(len(cl)) if cl[s]}
    brk = {int(g): i for i, g in enumerate(break_groups)}
    out = np.zeros(n, dtype=dtype)
    for k in range((n + C - 1) // C):
        bits = "".join(f"{int(w):032b}" for w in words[int(offsets[k]):int(offsets[k + 1])])
        pos = 0
        lo, hi = k * C, min(n, (k + 1) * C)
        for g0 in range(lo, hi, G):
            g1 = min(hi, g0 + G)
            if g0 // G in brk:
                i = brk[g0 // G]
                out[g0:g1] = break_syms[i * G: i * G + (g1 - g0)]
                continue
            for i in range(g0, g1):
                v, ln = 0, 0
                while (ln, v) not in table:
                    v = 2 * v + int(bits[pos])
                    pos += 1
                    ln += 1
                    if ln > 64:
                        raise ValueError("not a code")
                out[i] = table[(ln, v)]
    return out
