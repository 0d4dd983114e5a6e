"""End-to-end Huffman encoding throughput on one MI355X.

One step = one pass of the whole path over one stream already resident in
HBM: hf_histogram -> hf_build_codebook -> hf_encode (bit-dense stream plus
chunk offsets).  The metric is input bytes per second (GB = 1e9 bytes).

Prints one JSON line with the metric, a roofline entry for the dominant
kernel (timed with HIP events around its launch, on the stream it runs on)
and the CPU oracle's throughput on the same input, timed on the host.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X published HBM3E bandwidth


def log(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=20)
    p.add_argument("--warmup", type=int, default=3)
    p.add_argument("--workload", default="lorenzo3d_512cube_u16_A1024")
    p.add_argument("--chunk", type=int, default=4096)
    p.add_argument("--reduce-log2", type=int, default=0)
    p.add_argument("--cpu-seconds", type=float, default=12.0,
                   help="approximate CPU time budget of the oracle baseline (0 = skip)")
    p.add_argument("--mode", choices=("pipeline", "copy"), default="pipeline",
                   help="copy: only time a device-to-device copy of the input (bandwidth calibration)")
    return p.parse_args()


def cpu_baseline(x: np.ndarray, A: int, chunk: int, budget_s: float):
    """The oracle (serial C: histogram, heap codebook, serial bit packer) on
    the same input, repeated over whole passes until ~budget_s has elapsed."""
    import oracle

    passes = 0
    t_total = 0.0
    while passes == 0 or (t_total < budget_s and passes < 5):
        t0 = time.perf_counter()
        h = oracle.histogram(x, A)
        book = oracle.codebook(h)
        oracle.encode(x, book, chunk)
        t_total += time.perf_counter() - t0
        passes += 1
    per_pass = t_total / passes
    return {
        "value": round(x.nbytes / per_pass / 1e9, 4),
        "unit": "GB/s",
        "cores": 1,
        "kind": "oracle",
        "sample": f"{passes} whole pass(es) of histogram+codebook+encode over the same "
                  f"{x.size} symbols, serial C, {per_pass:.2f} s per pass",
    }


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (this encoder runs each stream on a single device); "
              f"got --gpus {args.gpus}", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2010_10039_amd import hf, workloads

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    spec = workloads.WORKLOADS[args.workload]
    A = spec["alphabet"]
    t0 = time.perf_counter()
    x = workloads.make(args.workload)
    log(f"generated {args.workload}: n={x.size} bytes={x.nbytes} in {time.perf_counter() - t0:.1f}s")
    sb = x.dtype.itemsize
    d = torch.from_numpy(x.view(np.int16) if sb == 2 else x).cuda()
    n = x.size

    # calibration: a plain device-to-device copy of the same number of bytes
    dst = torch.empty_like(d)
    for _ in range(3):
        dst.copy_(d)
    c0, c1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ncopy = 10
    c0.record()
    for _ in range(ncopy):
        dst.copy_(d)
    c1.record()
    torch.cuda.synchronize()
    copy_gbs = 2 * x.nbytes / (c0.elapsed_time(c1) / ncopy * 1e-3) / 1e9
    log(f"device copy of {x.nbytes} bytes: {copy_gbs:.0f} GB/s (read + write)")
    if args.mode == "copy":
        print(json.dumps({"mode": "copy", "bytes": x.nbytes, "copy_gbs": round(copy_gbs, 1)}), flush=True)
        return
    del dst

    enc = hf.Encoder(n, A, args.chunk, args.reduce_log2)
    r_eff = args.reduce_log2 or 4
    for _ in range(args.warmup):
        enc.run(d)
    torch.cuda.synchronize()
    hf.raise_on_status(enc.status, "warmup")
    info = enc.book.info.cpu().numpy().view(np.uint64)
    m, lmax, total_bits = int(info[0]), int(info[1]), int(info[2])
    log(f"warmup done: m={m} Lmax={lmax} beta={total_bits / n:.4f}")

    stages = ("hist", "codebook", "encode")
    ev = {s: [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in range(args.steps)] for s in stages}
    for s in stages:  # materialize the event handles before handing them to libhf
        for a, b in ev[s]:
            a.record()
            b.record()
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    start.record()
    for k in range(args.steps):
        enc.run(d, timers={s: ev[s][k] for s in stages})
    stop.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    hf.raise_on_status(enc.status, "timed steps")
    ms_per_step = start.elapsed_time(stop) / args.steps
    stage_ms = {s: sum(a.elapsed_time(b) for a, b in ev[s]) / args.steps for s in stages}
    value = n * sb / (ms_per_step * 1e-3) / 1e9
    log(f"timed {args.steps} steps: {ms_per_step * 1e3:.1f} us/step (wall {wall * 1e6 / args.steps:.1f} us); "
        + ", ".join(f"{s} {stage_ms[s] * 1e3:.1f} us" for s in stages))

    # decode check of the last step's output (not timed)
    res = hf.hf_decode_check(enc.out, enc.offsets, d, args.chunk, enc.book)
    torch.cuda.synchronize()
    mism = int(res[0].item())
    if mism != 0:
        raise SystemExit(f"decode check failed: {mism} mismatching symbols")

    nch = (n + args.chunk - 1) // args.chunk
    out_bytes = (total_bits + 31) // 32 * 4
    enc_bytes = n * sb + out_bytes + (nch + 1) * 8 + A * 9
    enc_s = stage_ms["encode"] * 1e-3
    achieved = enc_bytes / enc_s / 1e9
    e2e_alg = 2 * n * sb + out_bytes + (nch + 1) * 8
    roofline = {
        "bound": "hbm",
        "kernel": "encode_kernel",
        "achieved": round(achieved, 1),
        "peak": HBM_PEAK_GBS,
        "unit": "GB/s",
        "frac": round(achieved / HBM_PEAK_GBS, 4),
        "traffic": None,
        "bytes_per_launch": enc_bytes,
        "avg_launch_us": round(stage_ms["encode"] * 1e3, 2),
    }
    cpu = None
    if args.cpu_seconds > 0:
        log("timing the CPU oracle")
        cpu = cpu_baseline(x, A, args.chunk, args.cpu_seconds)
    line = {
        "metric": "end-to-end encode GB/s of input symbols",
        "value": round(value, 2),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u16" if sb == 2 else "u8",
        "data": "synthetic",
        "config": {
            "workload": args.workload,
            "n_symbols": n,
            "alphabet": A,
            "chunk_symbols": args.chunk,
            "reduce_log2": r_eff,
            "used_symbols": m,
            "max_code_len": lmax,
            "avg_bits": round(total_bits / n, 4),
            "input_frac_of_hbm_peak": round(value / HBM_PEAK_GBS, 4),
            "e2e_algorithmic_frac_of_hbm_peak": round(e2e_alg / (ms_per_step * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
            "stage_us": {s: round(stage_ms[s] * 1e3, 2) for s in stages},
            "device_copy_gbs": round(copy_gbs, 1),
        },
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
