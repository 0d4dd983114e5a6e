"""CPU oracle of the quantizing front end -- TEST INFRASTRUCTURE ONLY.

The paper's multi-byte benchmark input (Sec. 5.1.3, Nyx-Quant) is the
stream of quantization codes that an SZ-style error-bounded compressor makes
from a float field.  The paper fixes no formula for it; the codes here follow
the usual SZ/cuSZ recipe, read as:

1. prequantization: d = rint(x * r) in float32, where r is the float32
   factor 1 / (2 eb) for an absolute error bound eb; rint rounds ties to
   even; the result is clamped to [-2^24, 2^24], which keeps every residual
   inside 32 bits.  A non-finite value (NaN or an infinity) is outside the
   domain of an error-bounded quantizer -- no finite reconstruction lies
   within eb of it -- so a field holding one is refused (NonFiniteInput);
2. 3D Lorenzo prediction: the residual e is the mixed first difference of d
   along all three axes, with d taken as 0 outside the grid;
3. codes: q = e + radius when 1 <= e + radius <= 2 radius - 1, else 0 (the
   outlier marker), over an alphabet of 2 radius symbols.

Each step is written out plainly, in numpy, in int64 for the integer steps
(no overflow is possible: |d| <= 2^24 and e sums eight such terms).  The
per-slab counts follow the slab partition of the encoder's interface (whole
4096-symbol blocks, slab g covering blocks [floor(g nb / S),
floor((g + 1) nb / S))).

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this module; it imports nothing from the GPU library.
"""
from __future__ import annotations

import numpy as np

CLAMP = float(1 << 24)
SLAB_BLOCK = 4096


class NonFiniteInput(ValueError):
    """The field holds a NaN or an infinity, which no error bound covers."""


def prequantize(x: np.ndarray, inv_2eb: float) -> np.ndarray:
    """Step 1: d = rint(x * r) computed in float32, then clamped to
    [-2^24, 2^24]; int64.  Raises NonFiniteInput if any x is NaN or infinite."""
    x = np.asarray(x, dtype=np.float32)
    if not np.all(np.isfinite(x)):
        raise NonFiniteInput(f"{int(np.count_nonzero(~np.isfinite(x)))} non-finite value(s) in the field")
    with np.errstate(over="ignore"):
        v = x * np.float32(inv_2eb)  # one correctly rounded float32 product (may overflow to +-inf)
    v = np.rint(v)                   # ties to even
    v = np.minimum(np.maximum(v, np.float32(-CLAMP)), np.float32(CLAMP))
    return v.astype(np.int64)


def lorenzo_residual(d: np.ndarray) -> np.ndarray:
    """Step 2: e = D_0 D_1 D_2 d, where D_a is the first difference along
    axis a with zero padding below index 0: (D_a d)[.., i, ..] = d[.., i, ..]
    - d[.., i - 1, ..] for i > 0 and d[.., 0, ..] itself for i = 0."""
    e = np.array(d, dtype=np.int64, copy=True)
    for axis in range(e.ndim):
        if e.shape[axis] < 2:
            continue
        hi = [slice(None)] * e.ndim
        lo = [slice(None)] * e.ndim
        hi[axis] = slice(1, None)
        lo[axis] = slice(None, -1)
        shifted = e[tuple(lo)].copy()
        e[tuple(hi)] -= shifted
    return e


def residual_codes(e: np.ndarray, radius: int) -> np.ndarray:
    """Step 3: q = e + radius inside [1, 2 radius - 1], else 0; uint16."""
    q = np.asarray(e, dtype=np.int64) + int(radius)
    q[(q < 1) | (q > 2 * int(radius) - 1)] = 0
    return q.astype(np.uint16)


def lorenzo_codes(x: np.ndarray, inv_2eb: float, radius: int) -> np.ndarray:
    """Codes of a float field of shape (nz, ny, nx) (or 1D/2D), flattened in
    C order, uint16 over the alphabet 2 radius."""
    x = np.asarray(x, dtype=np.float32)
    if x.ndim < 3:
        x = x.reshape((1,) * (3 - x.ndim) + x.shape)
    return residual_codes(lorenzo_residual(prequantize(x, inv_2eb)), radius).reshape(-1)


def histogram(codes: np.ndarray, alphabet: int) -> np.ndarray:
    """Count of every code, uint32[alphabet]."""
    return np.bincount(np.asarray(codes, dtype=np.int64).reshape(-1), minlength=alphabet).astype(np.uint32)


def slab_bounds(n: int, nslabs: int) -> list[tuple[int, int]]:
    """[begin, end) of each slab of the encoder's block partition."""
    nb = (n + SLAB_BLOCK - 1) // SLAB_BLOCK
    starts = [min((g * nb // nslabs) * SLAB_BLOCK, n) for g in range(nslabs + 1)]
    return [(starts[g], starts[g + 1]) for g in range(nslabs)]


def slab_histograms(codes: np.ndarray, alphabet: int, nslabs: int) -> np.ndarray:
    """uint32[nslabs, alphabet]: row g counts the codes of slab g."""
    codes = np.asarray(codes).reshape(-1)
    rows = [histogram(codes[lo:hi], alphabet) for lo, hi in slab_bounds(codes.size, nslabs)]
    return np.stack(rows) if rows else np.zeros((0, alphabet), dtype=np.uint32)
