"""AddressSanitizer / UndefinedBehaviorSanitizer builds of the host code (CPU
only): the oracle driven through its whole API on the tiny workload and on
edge cases, and the host model of the grid-wide planners on random and
extreme batches.  Any sanitizer report fails the test."""
import os
import shutil
import subprocess

import numpy as np
import pytest

import hypergen

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HERE = os.path.join(ROOT, "tests", "sanitize")
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")


def _run(exe, *args):
    r = subprocess.run([exe, *args], stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True, env=ENV,
                       timeout=600)
    assert r.returncode == 0, (r.returncode, r.stderr[-4000:])
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr[-4000:]
    assert r.stdout.startswith("ok ")
    return r.stdout


def _write_input(path, hg, model, p, k, eps):
    with open(path, "wb") as f:
        f.write(np.array([hg.n, hg.m, model], np.uint32).tobytes())
        f.write(np.array([p], np.float32).tobytes())
        f.write(np.array([k], np.uint32).tobytes())
        f.write(np.array([eps], np.float64).tobytes())
        f.write(hg.he_off.astype(np.uint32).tobytes())
        f.write(hg.he_mem.astype(np.uint32).tobytes())


def test_oracle_under_asan_ubsan(tmp_path):
    exe = str(tmp_path / "oracle_san")
    subprocess.check_call(["gcc", "-O1", "-g", "-std=c11", "-pthread", *SAN,
                           os.path.join(HERE, "oracle_driver.c"), os.path.join(ROOT, "oracle", "hyperim_oracle.c"),
                           "-o", exe, "-lm"])
    w = hypergen.workload("tiny")
    cases = [
        (w.build(), w.model, w.p, w.k, w.eps),
        (hypergen.tiny_hypergraph(5, 300, 500, 1, 8, allow_singletons=True), 1, 0.0, 5, 0.5),
        (hypergen.from_lists(6, [[], [2], [0, 1], [], [3, 4, 5], [1, 5]]), 0, 1.0, 2, 0.5),
        (hypergen.from_lists(1, [[0], []]), 0, 0.5, 1, 0.5),
    ]
    for i, (hg, model, p, k, eps) in enumerate(cases):
        path = str(tmp_path / f"in{i}.bin")
        _write_input(path, hg, model, p, k, eps)
        _run(exe, path)


def test_planner_model_under_asan_ubsan(tmp_path):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    exe = str(tmp_path / "plan_san")
    host_san = []
    for flag in SAN:
        host_san += ["-Xarch_host", flag]
    subprocess.check_call([hipcc, "-O1", "-g", "-std=c++17", "--offload-arch=gfx950", *host_san,
                           "-I", os.path.join(ROOT, "include"), "-I", os.path.join(ROOT, "paper_2406_01911_amd", "csrc"),
                           os.path.join(HERE, "plan_driver.hip"),
                           os.path.join(ROOT, "paper_2406_01911_amd", "csrc", "plan_model.hip"), "-o", exe],
                          stderr=subprocess.DEVNULL)
    _run(exe)
