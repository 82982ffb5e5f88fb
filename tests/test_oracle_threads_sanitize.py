"""The oracle's OpenMP mode and a sanitizer build of the oracle (CPU only).

* Threads: every destination particle's sums are formed by one thread in the
  same order, so 1 thread and several threads give bitwise equal results.
* Sanitizers: the oracle source is compiled together with a driver that calls
  every entry point, under AddressSanitizer and UndefinedBehaviorSanitizer
  (host code only), and run: it must finish without a report."""
import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle
import sph_workloads as W

HERE = os.path.dirname(os.path.abspath(__file__))


def _runs(fn):
    outs = []
    for k in (1, 4):
        oracle.set_threads(k)
        try:
            outs.append(fn())
        finally:
            oracle.set_threads(1)
    return outs


@pytest.mark.parametrize("case", ["tg", "cube", "dam3d", "brute"])
def test_threads_bitwise_equal_evaluate_and_step(case):
    if case == "tg":
        p, s = W.taylor_green(40, jitter=0.3, seed=3)
    elif case == "cube":
        p, s = W.periodic_cube(n_side=12, jitter=0.3, sigma_u=0.1, seed=4)
    elif case == "dam3d":
        p, s = W.dam_break_3d(dx=0.05)
    else:
        p, s = W.taylor_green(24, jitter=0.3, seed=5, kernel=W.QUINTIC)
    brute = case == "brute"

    def go():
        ev = oracle.evaluate(p, s.x, s.u, s.m, s.ptype, brute=brute)
        st = oracle.step(p, s.x, s.u, s.m, s.ptype, 3, want_diag=True, brute=brute)
        off, idx = oracle.neighbors(p, s.x, brute=brute)
        return ev, st, (off, idx)

    a, b = _runs(go)
    for x, y in zip(a[0], b[0]):
        assert np.array_equal(x, y)
    for k in a[1]:
        assert np.array_equal(a[1][k], b[1][k]), k
    assert np.array_equal(a[2][0], b[2][0]) and np.array_equal(a[2][1], b[2][1])


def test_threads_bitwise_equal_continuity():
    p, s = W.dam_break_2d()

    def go():
        e = oracle.step_continuity(p, s.x, s.u, s.rho, s.m, s.ptype, 5)
        c = oracle.step_continuity_pc(p, s.x, s.u, s.rho, s.m, s.ptype, 5)
        return e, c

    a, b = _runs(go)
    for r1, r2 in zip(a, b):
        for k in r1:
            assert np.array_equal(r1[k], r2[k]), k


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_oracle_under_address_and_ub_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_sanitize")
    src = os.path.join(HERE, "native", "oracle_sanitize_driver.cpp")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-ffp-contract=off",
           "-fopenmp", "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
           "-o", exe, src]
    subprocess.run(cmd, check=True, capture_output=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    env.pop("LD_PRELOAD", None)
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
    assert "all cases ok" in r.stdout
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr
