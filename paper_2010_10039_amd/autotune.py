"""Per-stream choice of the reduction factor and the chunk size.

The paper picks the reduction factor r from the average code length beta
so that 2^r merged codes fill about one 32-bit word (Sec. 4.3): r = 4 -
floor(log2 beta).  In this encoder a lane merges 2^r codes in registers
before one workgroup scan per 256 * 2^r symbols, so r trades scan and
barrier work against register pressure, and the chunk size only sets the
granularity of the offset table (8 bytes per chunk) and of later parallel
decoding.  Neither has a closed-form optimum on this hardware, so the tuner
times the encoder over a grid of (r, chunk) per bucket of (symbol width,
alphabet, beta class) on seeded synthetic streams of that bucket, and keeps
the fastest; the paper's rule is the prior used for buckets that were not
timed.  Ties within 2% go to the smaller chunk (more chunks to decode in
parallel).

Buckets:
  sym_bytes  1 or 2
  alpha      ceil(log2 A), rounded up to one of 8, 10, 12, 13, 16
  beta_cls   floor(log2 beta) clamped to [0, 4] (beta < 2: 0)
"""
from __future__ import annotations

import json
import math
import os
from dataclasses import dataclass, field

R_CHOICES = (3, 4, 5)
CHUNK_CHOICES = (1024, 4096, 16384, 65536)
ALPHA_CLASSES = (8, 10, 12, 13, 16)
BETA_CLASSES = (0, 1, 2, 3, 4)
DEFAULT_CHUNK = 4096


def alpha_class(alphabet: int) -> int:
    bits = max(1, math.ceil(math.log2(max(2, alphabet))))
    for c in ALPHA_CLASSES:
        if bits <= c:
            return c
    return ALPHA_CLASSES[-1]


def beta_class(beta: float) -> int:
    if not beta or beta < 2.0:
        return 0
    return min(4, int(math.floor(math.log2(beta))))


def paper_rule(beta: float | None) -> int:
    """The library's reduction-factor rule (hf_reduction_factor: Sec. 4.3,
    r = 4 - floor(log2 beta)), limited to the factors the batch path
    instantiates; without a beta, the middle choice."""
    if beta is None:
        return 4
    from paper_2010_10039_amd import hf

    return max(R_CHOICES[0], min(R_CHOICES[-1], hf.hf_reduction_factor(float(beta))))


def bucket_key(sym_bytes: int, alphabet: int, beta: float | None) -> str:
    b = "any" if beta is None else str(beta_class(beta))
    return f"u{8 * sym_bytes}/a{alpha_class(alphabet)}/b{b}"


@dataclass
class Choice:
    r: int
    chunk: int
    source: str  # "timed" or "rule"


@dataclass
class Autotuner:
    table: dict = field(default_factory=dict)  # bucket key -> {"r", "chunk", "times"}

    # -- lookup ----------------------------------------------------------
    def choose(self, sym_bytes: int, alphabet: int, beta: float | None = None) -> Choice:
        """Best (r, chunk) for a stream; beta may be unknown (None), then
        the bucket's choice over all beta classes is used."""
        for key in (bucket_key(sym_bytes, alphabet, beta), bucket_key(sym_bytes, alphabet, None)):
            e = self.table.get(key)
            if e:
                return Choice(int(e["r"]), int(e["chunk"]), "timed")
        return Choice(paper_rule(beta), DEFAULT_CHUNK, "rule")

    # -- persistence -----------------------------------------------------
    def save(self, path: str) -> None:
        with open(path, "w") as f:
            json.dump(self.table, f, indent=1, sort_keys=True)

    @staticmethod
    def load(path: str) -> "Autotuner":
        if not os.path.exists(path):
            return Autotuner()
        with open(path) as f:
            return Autotuner(json.load(f))

    # -- tuning ----------------------------------------------------------
    @staticmethod
    def pick(times: dict) -> tuple[int, int]:
        """Fastest (r, chunk) from {(r, chunk): seconds}; within 2% of the
        fastest, the smaller chunk, then the smaller r."""
        best = min(times.values())
        ok = [k for k, t in times.items() if t <= best * 1.02]
        return min(ok, key=lambda k: (k[1], k[0]))

    def record(self, key: str, times: dict) -> None:
        r, chunk = self.pick(times)
        self.table[key] = {"r": r, "chunk": chunk,
                           "times": {f"r{k[0]}/c{k[1]}": round(v * 1e6, 2) for k, v in sorted(times.items())}}

    def finish(self) -> None:
        """Adds the beta-independent entry of every (width, alphabet) pair:
        the (r, chunk) with the smallest sum of time ratios to each beta
        class's best."""
        groups: dict = {}
        for key, e in self.table.items():
            w, a, b = key.split("/")
            if b == "bany":
                continue
            groups.setdefault((w, a), []).append(e)
        for (w, a), entries in groups.items():
            score: dict = {}
            for e in entries:
                best = min(e["times"].values())
                for k, v in e["times"].items():
                    score[k] = score.get(k, 0.0) + v / best
            kbest = min(score, key=lambda k: (round(score[k], 3), int(k.split("/c")[1]), k))
            r = int(kbest.split("/")[0][1:])
            c = int(kbest.split("/c")[1])
            self.table[f"{w}/{a}/bany"] = {"r": r, "chunk": c, "score": round(score[kbest], 3)}


def tune(widths_alphabets=((1, 256), (2, 1024), (2, 4096), (2, 8192)), n: int = 1 << 25,
         reps: int = 5, seed: int = 4242, device: str = "cuda") -> Autotuner:
    """Times hf_encode over R_CHOICES x CHUNK_CHOICES for every bucket on a
    seeded discrete Gaussian stream whose sigma puts beta in that bucket's
    class.  Needs the GPU."""
    import torch

    from . import hf

    tuner = Autotuner()
    g = torch.Generator(device=device)
    # sigma whose discrete Gaussian has entropy near 2^c + 0.5 bits
    for sb, A in widths_alphabets:
        dt = torch.uint8 if sb == 1 else torch.int16
        for bc in BETA_CLASSES:
            target = (2 ** bc) + 0.5 if bc else 1.2
            sigma = max(0.25, 2 ** (target - 2.05))  # H(N(0, s)) ~ log2(s) + 2.05
            if A / 2 < 3 * sigma:
                continue
            g.manual_seed(seed + 97 * bc + A)
            v = torch.randn(n, generator=g, device=device) * sigma + A / 2
            x = torch.clamp(torch.round(v), 0, A - 1).to(torch.int32).to(dt)
            hist = hf.hf_histogram(x, A)
            book = hf.hf_build_codebook(hist)
            info = book.info.cpu().tolist()
            beta = info[2] / n
            key = bucket_key(sb, A, beta)
            times = {}
            status = hf.new_status(device)
            for c in CHUNK_CHOICES:
                out = torch.empty(max(1, hf.hf_bound_words(n, A)), dtype=torch.int32, device=device)
                offs = torch.empty((n + c - 1) // c + 1, dtype=torch.int64, device=device)
                ws = hf.new_workspace(n, A, c, device)
                for r in R_CHOICES:
                    hf.hf_encode(x, book, c, r, out, offs, ws, status)
                    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
                    ev[0].record()
                    for _ in range(reps):
                        hf.hf_encode(x, book, c, r, out, offs, ws, status)
                    ev[1].record()
                    ev[1].synchronize()
                    times[(r, c)] = ev[0].elapsed_time(ev[1]) / reps / 1e3
            hf.raise_on_status(status, "autotune")
            tuner.record(key, times)
    tuner.finish()
    return tuner


def main() -> None:
    import argparse
    import time

    p = argparse.ArgumentParser(description="time the encoder per bucket and write the table")
    p.add_argument("--out", default=os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuning_mi355x.json"))
    p.add_argument("--n", type=int, default=1 << 25)
    args = p.parse_args()
    t0 = time.perf_counter()
    tuner = tune(n=args.n)
    tuner.save(args.out)
    print(f"wrote {len(tuner.table)} buckets to {args.out} in {time.perf_counter() - t0:.1f}s", flush=True)
    for k in sorted(tuner.table):
        e = tuner.table[k]
        print(f"  {k}: r={e['r']} chunk={e['chunk']}", flush=True)


if __name__ == "__main__":
    main()
