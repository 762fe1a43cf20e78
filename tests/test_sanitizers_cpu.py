"""The host planner and the plan emulator built with AddressSanitizer and
UndefinedBehaviorSanitizer (g++, host code only) and run on the benchmark
workloads' plans: the greedy partition of both levels, the distributed
level and the lowering must run clean, and the results must still equal the
oracle's (emulated states within 1e-5, partitions exactly)."""
import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle
import workloads as W
from oracle import centrality as C

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
EMU = os.path.join(HERE, "emu")
PLANNER = os.path.join(ROOT, "paper_2509_14098_amd", "csrc", "planner.cpp")


@pytest.fixture(scope="module")
def sanitized(tmp_path_factory):
    if shutil.which("g++") is None:
        pytest.skip("g++ not available")
    d = tmp_path_factory.mktemp("san")
    exe = str(d / "sanemu")
    flags = ["-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
             "-fno-sanitize-recover=all"]
    srcs = [os.path.join(EMU, "sanitize_main.cpp"), os.path.join(EMU, "plan_emulator.cpp"), PLANNER]
    objs = [str(d / (os.path.basename(s) + ".o")) for s in srcs]
    procs = [subprocess.Popen(["g++", *flags, "-I", os.path.join(EMU, "shim"), "-c", s, "-o", o])
             for s, o in zip(srcs, objs)]
    assert all(p.wait() == 0 for p in procs), "sanitizer build failed"
    subprocess.check_call(["g++", *flags, "-o", exe, *objs])
    return exe, d


def run_cases(sanitized, cases):
    exe, d = sanitized
    inp, out = str(d / "cases.bin"), str(d / "out.bin")
    with open(inp, "wb") as f:
        f.write(np.int32(len(cases)).tobytes())
        for mode, n, gates, theta, k, R, LW, n_global in cases:
            th = np.zeros(0) if theta is None else np.asarray(theta, np.float64)
            f.write(np.array([mode, n, len(gates), len(th), k, R, LW, 0, n_global], np.int32).tobytes())
            f.write(np.ascontiguousarray(gates).tobytes())
            f.write(th.tobytes())
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0:halt_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([exe, inp, out], env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stderr[-4000:]
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr[-4000:]
    raw = open(out, "rb").read()
    results, pos = [], 0
    for mode, n, *_ in cases:
        if mode == 0:
            size = 8 << n
            results.append(np.frombuffer(raw[pos:pos + size], np.complex64))
            pos += size
        else:
            (np_,), pos = np.frombuffer(raw[pos:pos + 4], np.int32), pos + 4
            parts = []
            for _ in range(np_):
                mask = int(np.frombuffer(raw[pos:pos + 8], np.uint64)[0])
                ng = int(np.frombuffer(raw[pos + 8:pos + 12], np.int32)[0])
                gl = np.frombuffer(raw[pos + 12:pos + 12 + 4 * ng], np.int32).tolist()
                pos += 12 + 4 * ng
                parts.append(([q for q in range(64) if (mask >> q) & 1], gl))
            results.append(parts)
    assert pos == len(raw)
    return results


def test_emulated_plans_under_sanitizers(sanitized):
    cases, refs = [], []
    for i, (R, LW) in enumerate([(1, 6), (3, 6), (4, 8), (5, 8), (4, 9), (4, 10)]):
        n = 9 + i
        theta = np.random.default_rng(i).uniform(-3, 3, size=4)
        gates = W.random_circuit(n, 150, seed=70 + i, n_params=4)
        cases.append((0, n, gates, theta, min(n, R + LW - 1, 9), R, LW, 0))
        refs.append(oracle.apply(n, gates, theta))
    for name, n, gates in (("c1", 12, W.brickwork_c1()), ("c2-16", 16, W.brickwork_c2(n=16, layers=10)),
                           ("qft-15", 15, W.qft(15))):
        cases.append((0, n, gates, None, 10, 4, 8 if n > 12 else 6, 0))
        refs.append(oracle.apply(n, gates))
    gd = W.brickwork_c3(n=16, layers=8, seed=9)  # the distributed level: 4 emulated ranks
    cases.append((0, 16, gd, None, 8, 3, 8, 2))
    refs.append(oracle.apply(16, gd))
    for got, ref in zip(run_cases(sanitized, cases), refs):
        assert np.max(np.abs(got - ref)) < 1e-5


def test_benchmark_plans_under_sanitizers(sanitized):
    """Partition-only runs of the headline circuit (k = 10), a 5 100-gate
    34-qubit circuit (k = 12) and the 40-qubit circuit's distributed level
    over 256 ranks, against the oracle's greedy."""
    c2 = W.brickwork_c2()
    big = W.brickwork_c3(n=34, layers=100, seed=11)
    c40 = W.brickwork_c3(n=40)
    got = run_cases(sanitized, [(1, 28, c2, None, 10, 4, 9, 0), (1, 34, big, None, 12, 5, 8, 0),
                                (1, 40, c40, None, 10, 4, 9, 8)])
    assert got[0] == [(list(S), list(g)) for S, g in C.greedy_partition(28, c2, 10)]
    assert got[1] == [(list(S), list(g)) for S, g in C.greedy_partition(34, big, 12)]
    order = [g for _, gl in got[2] for g in gl if g >= 0]
    assert sorted(order) == list(range(len(c40)))
