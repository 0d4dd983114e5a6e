"""The per-run JSON Lines record of bench.py (`--jsonl`): one line per run,
appended, holding the printed bench line and the sha256 of the input's
bytes.  Runs on the CPU: only the record writer is called."""
import hashlib
import importlib.util
import json
import os

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def load_bench():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_records_append_with_input_hash(tmp_path):
    bench = load_bench()
    path = str(tmp_path / "runs.jsonl")
    x = np.arange(1000, dtype=np.uint16)
    line = {"metric": "m", "value": 1.5, "config": {"workload": "w"}}
    bench.append_run_record(path, line, x, "dev0")
    bench.append_run_record(path, dict(line, value=2.5), x[::2], "dev0")
    recs = [json.loads(l) for l in open(path)]
    assert len(recs) == 2
    assert recs[0]["line"] == line and recs[1]["line"]["value"] == 2.5
    assert recs[0]["input_sha256"] == hashlib.sha256(x.tobytes()).hexdigest()
    assert recs[1]["input_sha256"] == hashlib.sha256(np.ascontiguousarray(x[::2]).tobytes()).hexdigest()
    assert recs[0]["input_dtype"] == "uint16" and recs[0]["device"] == "dev0"
    assert recs[0]["host_cores"] >= 1 and recs[0]["generator_seed"] == 0
