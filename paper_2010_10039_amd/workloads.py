"""Seeded synthetic symbol streams shaped like the paper's workloads.

The paper evaluates on byte text (enwik8/9, Silesia), on SZ quantization
codes of a cosmology field (Nyx-Quant: 1024 symbols, 2-byte codes) and on
k-mer codes (Sec. 5.1.3).  None of those files is available, so these
generators stand in for them with the same value types, alphabet sizes and
kind of distribution.  Every generator is a pure function of its arguments
and seed.  The GPU path and the CPU oracle both consume the bytes these
functions return; nothing here performs any part of the Huffman method.
"""
from __future__ import annotations

import math

import numpy as np


def gaussian_codes(n: int = 1 << 20, alphabet: int = 1024, mean: float = 512.0,
                   sigma: float = 2.0, seed: int = 0, dtype=np.uint16) -> np.ndarray:
    """i.i.d. discrete Gaussian: clip(rint(N(mean, sigma)), 0, alphabet-1)."""
    rng = np.random.default_rng(seed)
    v = np.rint(rng.normal(mean, sigma, size=n))
    return np.clip(v, 0, alphabet - 1).astype(dtype)


def zipf_bytes(n: int = 100_000_000, s: float = 1.1, alphabet: int = 256, seed: int = 0,
               dtype=np.uint8) -> np.ndarray:
    """Zipf(s) over a random permutation of the symbol ids (text-like bytes).

    p_k is proportional to k^-s for ranks k = 1..alphabet; rank k is mapped to
    symbol perm[k-1]."""
    rng = np.random.default_rng(seed)
    perm = rng.permutation(alphabet)
    p = np.arange(1, alphabet + 1, dtype=np.float64) ** (-s)
    p /= p.sum()
    out = np.empty(n, dtype=dtype)
    step = 1 << 24
    for lo in range(0, n, step):
        hi = min(n, lo + step)
        out[lo:hi] = perm[rng.choice(alphabet, size=hi - lo, p=p)].astype(dtype)
    return out


def _smooth_field(dim: int, rng: np.random.Generator, nwaves: int = 8):
    """Sum of `nwaves` random 3D sinusoids on a dim^3 grid, in float64.

    f[i,j,k] = sum_q a_q sin(2 pi (u_q i + v_q j + w_q k) / dim + phi_q), with
    a ~ U(0.5, 1.5), (u, v, w) ~ U{1..8}^3, phi ~ U[0, 2 pi).  The angle is
    split as (u i + v j)/dim + phi and w k/dim, and sin(A + B) is expanded, so
    only dim^2 + dim transcendental evaluations are needed."""
    import torch

    a = rng.uniform(0.5, 1.5, nwaves)
    uvw = rng.integers(1, 9, size=(nwaves, 3))
    phi = rng.uniform(0.0, 2.0 * math.pi, nwaves)
    idx = np.arange(dim, dtype=np.float64)
    f = torch.zeros((dim, dim, dim), dtype=torch.float64)
    for q in range(nwaves):
        ang_ij = 2.0 * math.pi * (uvw[q, 0] * idx[:, None] + uvw[q, 1] * idx[None, :]) / dim + phi[q]
        ang_k = 2.0 * math.pi * uvw[q, 2] * idx / dim
        s_ij = torch.from_numpy(np.sin(ang_ij))[:, :, None]
        c_ij = torch.from_numpy(np.cos(ang_ij))[:, :, None]
        s_k = torch.from_numpy(np.sin(ang_k))[None, None, :]
        c_k = torch.from_numpy(np.cos(ang_k))[None, None, :]
        f.addcmul_(s_ij, c_k, value=float(a[q]))
        f.addcmul_(c_ij, s_k, value=float(a[q]))
    return f


def lorenzo_field(dim: int = 512, seed: int = 0, noise_rel_std: float = 0.01, eb_rel: float = 1e-4):
    """A dim^3 float32 field and its absolute error bound (the Nyx-like
    input of Sec. 5.1.3): 8 random sinusoids plus Gaussian noise of standard
    deviation noise_rel_std * std(field); eb = eb_rel * value range.
    Returns (x as a C-order numpy float32 array of shape (dim, dim, dim), eb)."""
    import torch

    rng = np.random.default_rng(seed)
    f = _smooth_field(dim, rng)
    sd = float(f.std())
    x = f.to(torch.float32)
    del f
    g = torch.Generator().manual_seed(int(rng.integers(0, 2**62)))
    noise = torch.randn(x.shape, generator=g, dtype=torch.float32)
    x.add_(noise, alpha=noise_rel_std * sd)
    del noise
    eb = eb_rel * float(x.max() - x.min())
    return x.numpy(), eb


def random_field(shape, seed: int = 0, nwaves: int = 6, noise_rel_std: float = 0.01) -> np.ndarray:
    """A small float32 field of any 3D shape for tests: a sum of `nwaves`
    random sinusoids over the grid (amplitudes U(0.5, 1.5), integer
    frequencies 1..4 per axis, random phases) plus Gaussian noise of standard
    deviation noise_rel_std * std.  Evaluated directly in float64, so meant
    for grids of a few million points at most."""
    rng = np.random.default_rng(seed)
    nz, ny, nx = (int(v) for v in shape)
    iz = np.arange(nz, dtype=np.float64)[:, None, None] / max(nz, 1)
    iy = np.arange(ny, dtype=np.float64)[None, :, None] / max(ny, 1)
    ix = np.arange(nx, dtype=np.float64)[None, None, :] / max(nx, 1)
    f = np.zeros((nz, ny, nx), dtype=np.float64)
    for _ in range(nwaves):
        a = rng.uniform(0.5, 1.5)
        u, v, w = rng.integers(1, 5, size=3)
        f += a * np.sin(2.0 * math.pi * (u * iz + v * iy + w * ix) + rng.uniform(0.0, 2.0 * math.pi))
    sd = float(f.std()) if f.size > 1 else 1.0
    f += rng.normal(0.0, noise_rel_std * (sd if sd > 0 else 1.0), size=f.shape)
    return f.astype(np.float32)


def lorenzo_quant_codes(dim: int = 512, seed: int = 0, noise_rel_std: float = 0.01,
                        eb_rel: float = 1e-4, radius: int = 512) -> np.ndarray:
    """Error-bounded quantization codes of a smooth 3D field (SZ-style).

    The stand-in for the paper's Nyx-Quant input (Sec. 5.1.3), made from
    lorenzo_field(dim, seed).  Each value is prequantized to
    d = rint(x / (2 eb)) in float64; the 3D Lorenzo
    predictor's residual (the mixed first difference along i, j, k with zero
    padding outside the grid) is offset by `radius`; codes outside
    [1, 2*radius - 1] become 0, SZ's outlier marker.  Returns uint16 codes in
    C order, alphabet 2*radius."""
    import torch

    xn, eb = lorenzo_field(dim, seed, noise_rel_std, eb_rel)
    x = torch.from_numpy(xn)
    d = torch.round(x.to(torch.float64) / (2.0 * eb)).to(torch.int32)
    del x, xn
    for axis in range(3):
        e = d.clone()
        sl_hi = [slice(None)] * 3
        sl_lo = [slice(None)] * 3
        sl_hi[axis] = slice(1, None)
        sl_lo[axis] = slice(None, -1)
        e[tuple(sl_hi)] -= d[tuple(sl_lo)]
        d = e
    q = d.add_(radius)
    q[(q < 1) | (q > 2 * radius - 1)] = 0
    return q.reshape(-1).to(torch.int32).numpy().astype(np.uint16)


def skewed_histogram(alphabet: int, total: int, seed: int = 0, kind: str = "normal") -> np.ndarray:
    """A histogram (not a stream) for codebook-only workloads with large
    alphabets (the paper's synthetic normally distributed histograms, Sec. 5.2.1).

    kind = "normal": counts of `total` draws from N(alphabet/2, alphabet/8)
    clipped to the alphabet; "uniform": total spread evenly."""
    rng = np.random.default_rng(seed)
    if kind == "uniform":
        h = np.full(alphabet, total // alphabet, dtype=np.uint64)
        h[: total % alphabet] += 1
        return h.astype(np.uint32)
    v = np.clip(np.rint(rng.normal(alphabet / 2, alphabet / 8, size=total)), 0, alphabet - 1)
    return np.bincount(v.astype(np.int64), minlength=alphabet).astype(np.uint32)


def batched_streams(nstreams: int = 512, seed: int = 1000, min_log2: float = 16.0, max_log2: float = 26.0,
                    alphabets=(256, 1024, 4096, 8192), sigma_range=(0.5, 50.0), device: str = "cpu"):
    """Independent streams of uneven size, each with its own alphabet and
    distribution (the batched workload).

    Stream i (seed + i): n = floor(exp(U(ln 2^min_log2, ln 2^max_log2)));
    uint8 with alphabet 256 with probability 1/2, else uint16 with an
    alphabet drawn from `alphabets`; values clip(rint(N(A/2, sigma)), 0, A-1)
    with sigma log-uniform in sigma_range.  Sizes and parameters come from
    numpy; the values are drawn by torch on `device` with a seeded generator.
    Returns (list of tensors, list of alphabets)."""
    import torch

    syms, alph = [], []
    for i in range(nstreams):
        rng = np.random.default_rng(seed + i)
        n = int(math.exp(rng.uniform(min_log2 * math.log(2), max_log2 * math.log(2))))
        if rng.random() < 0.5:
            A, dt = 256, torch.uint8
        else:
            A, dt = int(rng.choice([a for a in alphabets if a > 256] or [256])), torch.int16
        sigma = math.exp(rng.uniform(math.log(sigma_range[0]), math.log(sigma_range[1])))
        g = torch.Generator(device=device).manual_seed(seed * 7919 + i)
        v = torch.randn(n, generator=g, device=device, dtype=torch.float32) * sigma + A / 2
        v = torch.clamp(torch.round(v), 0, A - 1)
        syms.append(v.to(torch.int32).to(dt))
        alph.append(A)
    return syms, alph


def skew_normal_codes(n: int, alphabet: int, sigma: float, shape: float, generator, device="cpu"):
    """clip(rint(A/2 + sigma * y), 0, A-1) with y skew-normal of shape
    `shape`: y = d |z0| + sqrt(1 - d^2) z1, d = shape / sqrt(1 + shape^2),
    z0, z1 i.i.d. N(0, 1).  Returns int32 values."""
    import torch

    d = shape / math.sqrt(1.0 + shape * shape)
    z0 = torch.randn(n, generator=generator, device=device)
    y = torch.randn(n, generator=generator, device=device).mul_(math.sqrt(1.0 - d * d))
    y.add_(z0.abs_(), alpha=d)
    del z0
    return torch.clamp(torch.round(y.mul_(sigma).add_(alphabet / 2)), 0, alphabet - 1).to(torch.int32)


def zipf_codes(n: int, alphabet: int, s: float, generator, device="cpu"):
    """Zipf(s) over a random permutation of [0, A): rank k (1-based) has
    probability proportional to k^-s; sampled by inverting the CDF.
    Returns int32 values."""
    import torch

    k = torch.arange(1, alphabet + 1, dtype=torch.float64, device=device)
    cdf = torch.cumsum(k.pow(-s), 0)
    cdf = (cdf / cdf[-1]).to(torch.float32)
    perm = torch.randperm(alphabet, generator=generator, device=device).to(torch.int32)
    u = torch.rand(n, generator=generator, device=device)
    idx = torch.clamp(torch.searchsorted(cdf, u), max=alphabet - 1)
    return perm[idx]


def poisson_arrivals(nreq: int, qps: float, seed: int = 7) -> list:
    """Arrival times (seconds) of a Poisson process of rate qps."""
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / qps, size=nreq)).tolist()


def served_requests(nreq: int = 200, seed: int = 2000, qps: float = 2000.0, min_bytes: float = 2.0 ** 20,
                    max_bytes: float = 2.0 ** 29, device: str = "cpu"):
    """A trace of compression requests (the served workload).

    Request i (seed + i): arrival = sum of i+1 exponential gaps of mean
    1/qps seconds; size log-uniform in [min_bytes, max_bytes]; uint8 with
    alphabet 256, or uint16 with alphabet 2^k, k uniform in 10..16; half the
    requests skew-normal (shape uniform in [-8, 8], sigma log-uniform in
    [0.5, A/8]), half Zipf (s uniform in [1.05, 1.6]).  The values are drawn
    by torch on `device`.  Returns a list of (arrival_s, symbols, alphabet,
    kind)."""
    import torch

    out = []
    t = 0.0
    for i in range(nreq):
        rng = np.random.default_rng(seed + i)
        t += rng.exponential(1.0 / qps)
        nbytes = math.exp(rng.uniform(math.log(min_bytes), math.log(max_bytes)))
        if rng.random() < 0.5:
            sb, A, dt = 1, 256, torch.uint8
        else:
            sb, A, dt = 2, 1 << int(rng.integers(10, 17)), torch.int16
        n = max(1, int(nbytes) // sb)
        g = torch.Generator(device=device).manual_seed(seed * 7919 + i)
        if rng.random() < 0.5:
            sigma = math.exp(rng.uniform(math.log(0.5), math.log(A / 8)))
            v = skew_normal_codes(n, A, sigma, float(rng.uniform(-8, 8)), g, device)
            kind = "skew-normal"
        else:
            v = zipf_codes(n, A, float(rng.uniform(1.05, 1.6)), g, device)
            kind = "zipf"
        out.append((t, v.to(dt), A, kind))
    return out


WORKLOADS = {
    "gaussian_1M_u16_A1024": dict(kind="gaussian", n=1 << 20, alphabet=1024, chunk=4096),
    "lorenzo3d_512cube_u16_A1024": dict(kind="lorenzo", dim=512, alphabet=1024, chunk=4096),
    "zipf_100M_u8_A256": dict(kind="zipf", n=100_000_000, alphabet=256, chunk=4096),
}


def make(name: str, scale: int = 0) -> np.ndarray:
    """Generate a named workload.  `scale` > 0 shrinks it for quick tests:
    n is divided by 2**scale (the Lorenzo grid edge by 2**(scale/3) rounded)."""
    w = WORKLOADS[name]
    if w["kind"] == "gaussian":
        return gaussian_codes(n=max(1, w["n"] >> scale), alphabet=w["alphabet"], seed=0)
    if w["kind"] == "zipf":
        return zipf_bytes(n=max(1, w["n"] >> scale), alphabet=w["alphabet"], seed=0)
    if w["kind"] == "lorenzo":
        dim = max(8, int(round(w["dim"] / 2 ** (scale / 3))))
        return lorenzo_quant_codes(dim=dim, seed=0)
    raise KeyError(name)
