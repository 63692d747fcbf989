"""Host C++ of the library built with sanitizers and checked on the CPU: the request
server's admission pass and round precision schedule (admission.h) and the FP64
symmetric eigensolver (eigh.cpp), under AddressSanitizer + UndefinedBehaviorSanitizer;
the eigensolver's thread pool also under ThreadSanitizer, with results that must not
depend on the thread count. No GPU involved."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2604_17001_amd", "csrc")
HOST = os.path.join(ROOT, "tests", "host")
ASAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer"]

pytestmark = pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not available")


def _build(tmp_path, name, srcs, flags):
    exe = str(tmp_path / name)
    cmd = ["g++", "-std=c++17", "-O1", "-g", *flags, "-I", CSRC, *srcs, "-o", exe, "-pthread"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    return exe


def _run(cmd, env_extra=None):
    env = dict(os.environ)
    env.update(env_extra or {})
    env.setdefault("ASAN_OPTIONS", "detect_leaks=1:abort_on_error=0")
    r = subprocess.run(cmd, capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "runtime error" not in r.stderr and "Sanitizer" not in r.stderr, r.stderr
    return r.stdout


def test_admission_and_schedule_under_asan_ubsan(tmp_path):
    exe = _build(tmp_path, "sched", [os.path.join(HOST, "sched_test.cpp")], ASAN)
    assert "sched ok" in _run([exe])


@pytest.mark.parametrize("n", [1, 2, 3, 17, 64, 150])
def test_eigensolver_under_asan_ubsan(tmp_path, n):
    exe = _build(tmp_path, "eigh", [os.path.join(HOST, "eigh_test.cpp"), os.path.join(CSRC, "eigh.cpp")], ASAN)
    _run([exe, str(n)])


def test_eigensolver_threads_under_tsan_and_thread_count_invariance(tmp_path):
    exe = _build(tmp_path, "eigh_tsan", [os.path.join(HOST, "eigh_test.cpp"), os.path.join(CSRC, "eigh.cpp")],
                 ["-fsanitize=thread"])
    outs = []
    for t in (1, 3, 8):
        f = str(tmp_path / f"eig_{t}.bin")
        _run([exe, "120", f], {"ICNNM_EIG_THREADS": str(t), "TSAN_OPTIONS": "halt_on_error=1"})
        outs.append(open(f, "rb").read())
    assert outs[0] == outs[1] == outs[2]
