"""bench.py on the CPU: its command line and its names.

The benchmark's legs run only on a GPU, so a misspelt or out-of-scope name
in one of them would surface only there; every name a function of
bench.py reads must be one of its own, a module global or a builtin.
"""
import builtins
import json
import os
import subprocess
import sys
import symtable

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
BENCH = os.path.join(ROOT, "bench.py")


def test_more_than_one_gpu_is_refused_with_a_message():
    res = subprocess.run([sys.executable, BENCH, "--gpus", "2"], capture_output=True, text=True,
                         timeout=120, cwd=ROOT)
    assert res.returncode == 2
    assert "one GPU" in json.loads(res.stdout.strip().splitlines()[-1])["error"]


def test_every_flag_parses(monkeypatch):
    sys.path.insert(0, ROOT)
    import bench
    monkeypatch.setattr(sys, "argv", [
        "bench.py", "--gpus", "1", "--steps", "3", "--warmup", "1", "--no-cpu-baseline",
        "--cpu-blocks", "100", "--no-batched", "--no-precision", "--no-reuse", "--reuse-frames", "4,8",
        "--serve-max-batch", "2", "--serve-requests", "10", "--tuning-cache", "/tmp/t.json",
        "--serve-log", "/tmp/s.jsonl", "--realtime-seconds", "0", "--copy-calibration", "0",
        "--only-headline", "--support", "24"])
    a = bench.parse()
    assert a.steps == 3 and a.reuse_frames == "4,8" and a.serve_log == "/tmp/s.jsonl"
    assert a.only_headline and a.support == 24


def test_every_name_a_function_reads_is_defined():
    sys.path.insert(0, ROOT)
    import bench
    src = open(BENCH).read()
    top = symtable.symtable(src, BENCH, "exec")
    known = set(vars(bench)) | set(dir(builtins))
    missing = []

    def walk(table, path):
        for child in table.get_children():
            where = f"{path}.{child.get_name()}"
            for sym in child.get_symbols():
                if sym.is_referenced() and sym.is_global() and sym.get_name() not in known:
                    missing.append(f"{where}: {sym.get_name()}")
            walk(child, where)

    walk(top, "bench")
    assert not missing, missing
