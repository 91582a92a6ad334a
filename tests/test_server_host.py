"""The request server's scheduler on the CPU (no GPU): server_core.cpp linked with a stub device
on a simulated clock (tests/host/server_stub.cpp), built with g++ under AddressSanitizer +
UndefinedBehaviorSanitizer and under ThreadSanitizer, and driven through the psara_server_* C
entry points: a seeded Poisson trace of 120 requests at 20/s (sides 64..512, a quarter adaptive,
injected failures at host set-up, device set-up and read-back, cancellations while queued and
while running) under continuous batching and under FIFO; cancelling frees the slot; a request
larger than the device is refused with PSARA_ENOMEM and one larger than the budget runs alone;
zero-iteration stages; destroying a busy server; the graph-cache key."""
import json
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SANITIZERS = {"asan": ["-fsanitize=address,undefined", "-fno-sanitize-recover=all"],
              "tsan": ["-fsanitize=thread"]}
SCENARIOS = ["graph_key", "zero_stage", "cancel", "oversize", "destroy_busy", "trace", "fifo"]


@pytest.fixture(scope="module")
def binaries(tmp_path_factory):
    if shutil.which("g++") is None:
        pytest.skip("no host C++ compiler")
    out = {}
    d = tmp_path_factory.mktemp("server_host")
    for name, flags in SANITIZERS.items():
        exe = str(d / f"server_stub_{name}")
        cmd = (["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-Wall", "-Werror", "-Wno-unused-variable"]
               + flags + ["-I", os.path.join(ROOT, "include"), "-I", os.path.join(ROOT, "paper_1801_02417_amd", "csrc"),
                          os.path.join(ROOT, "paper_1801_02417_amd", "csrc", "server_core.cpp"),
                          os.path.join(ROOT, "tests", "host", "server_stub.cpp"), "-o", exe, "-pthread"])
        r = subprocess.run(cmd, capture_output=True, text=True)
        assert r.returncode == 0, r.stderr
        out[name] = exe
    return out


@pytest.mark.parametrize("san", sorted(SANITIZERS))
@pytest.mark.parametrize("scenario", SCENARIOS)
def test_scheduler_under_sanitizer(binaries, san, scenario):
    env = dict(os.environ)
    env["TSAN_OPTIONS"] = "halt_on_error=1 second_deadlock_stack=1"
    env["ASAN_OPTIONS"] = "detect_leaks=1:abort_on_error=1"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
    r = subprocess.run([binaries[san], scenario], capture_output=True, text=True, timeout=600, env=env)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
    assert "ThreadSanitizer" not in r.stderr and "AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr
    line = json.loads(r.stdout.strip().splitlines()[-1])
    assert line["scenario"] == ("trace" if scenario == "fifo" else scenario)
    if scenario in ("trace", "fifo"):
        assert line["done"] + line["failed"] + line["cancelled"] == line["requests"] == 120
        assert line["peak_live"] == 1 if scenario == "fifo" else line["peak_live"] > 1
