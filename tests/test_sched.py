"""The server's scheduling policy on the CPU, with a simulated device.

`paper_2202_13926_amd/csrc/fsr_sched.h` holds the policy the server runs
(the HBM arena, request sizes and works, the choice of each batched
launch); `tests/sched/sched_sim.cpp` drives it on a virtual clock with a
Poisson stream of mixed frame sizes and checks FIFO admission, the budget,
slot reuse and coalescing of the arena, the in-flight limit, the
beside-a-running-batch rule, and the latency percentiles of continuous
batching against one request per launch.  Built with g++ and the host
sanitizers.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ is not available")
def test_scheduler_policy_with_a_simulated_device(tmp_path):
    exe = tmp_path / "sched_sim"
    subprocess.check_call(["g++", "-std=c++17", "-O1", "-g", "-Wall", "-Wextra",
                           "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                           "-I", os.path.join(ROOT, "paper_2202_13926_amd", "csrc"),
                           os.path.join(ROOT, "tests", "sched", "sched_sim.cpp"), "-o", str(exe)])
    res = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300)
    print(res.stdout)
    assert res.returncode == 0, res.stdout + res.stderr
    assert res.stdout.strip().endswith("ok")
