"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer.

Two host-only programs are compiled with g++ and run:

* the plan rules (``csrc/gp_rules.cpp``: parameter choice of section 3.5, the
  host tables, the step-3 row map and its low-rank factors of rem:step3, input
  validation) driven by ``tests/sanitize/rules_main.cpp`` over a sweep of
  d, nu, tol, length ranges, precisions and oversampling factors, with the
  geometric invariants the kernels rely on checked for every plan;
* the oracle (``oracle/oracle.cpp``) driven by ``tests/sanitize/oracle_main.cpp``,
  which cross-checks its independent forms on small inputs.

Any sanitizer report aborts the program (``-fno-sanitize-recover=all``).
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"]


def _build_and_run(tmp_path, name, sources, extra=(), env_extra=None):
    if shutil.which("g++") is None:
        pytest.skip("g++ not available")
    exe = str(tmp_path / name)
    cmd = ["g++", "-std=c++17", "-O1", "-g", *SAN, *extra, "-o", exe,
           *[os.path.join(ROOT, s) for s in sources]]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-4000:]
    env = dict(os.environ)
    env.setdefault("ASAN_OPTIONS", "detect_leaks=1:abort_on_error=0")
    env.setdefault("UBSAN_OPTIONS", "print_stacktrace=1")
    env.update(env_extra or {})
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-6000:])
    assert "runtime error" not in r.stderr, r.stderr[-6000:]
    return r.stdout


def test_plan_rules_under_sanitizers(tmp_path):
    out = _build_and_run(tmp_path, "rules_san",
                         ["tests/sanitize/rules_main.cpp", "paper_2407_03608_amd/csrc/gp_rules.cpp"],
                         extra=["-Wall", "-Wextra"])
    assert " 0 failures" in out, out


def test_oracle_under_sanitizers(tmp_path):
    out = _build_and_run(tmp_path, "oracle_san", ["tests/sanitize/oracle_main.cpp"],
                         extra=["-fopenmp"], env_extra={"OMP_NUM_THREADS": "2"})
    assert " 0 failures" in out, out
