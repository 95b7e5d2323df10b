"""Address and undefined-behaviour sanitizer runs on the CPU.

* The library's host-side logic (``csrc/host.cpp``: descriptor and rheology
  validation, the compact-layout builder, checkpoint parsing) is compiled
  with g++ -fsanitize=address,undefined together with the checks of
  ``tests/native/host_checks.cpp`` and run.
* The oracle is compiled with the same sanitizers and its pins (brute force,
  lattice, operators, residual) run against it.
* A planted out-of-bounds read in a copy of the oracle must be reported, so
  a clean run means the sanitizers were live.
"""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1610_01388_amd", "csrc")
SAN = ["-fno-omit-frame-pointer", "-fsanitize=address,undefined", "-fno-sanitize-recover=all"]
PINS = ["tests/test_oracle_bruteforce.py", "tests/test_oracle_lattice.py", "tests/test_oracle_operators.py",
        "tests/test_oracle_residual.py", "tests/test_oracle_hb.py"]

pytestmark = pytest.mark.skipif(shutil.which("gcc") is None or shutil.which("g++") is None,
                                reason="needs gcc and g++")


def _runtime_preload():
    """The sanitizer runtimes, ahead of anything already preloaded."""
    libs = []
    for name in ("libasan.so", "libubsan.so"):
        p = subprocess.check_output(["gcc", f"-print-file-name={name}"], text=True).strip()
        if not os.path.isabs(p):
            pytest.skip(f"{name} not found")
        libs.append(p)
    old = os.environ.get("LD_PRELOAD", "")
    return " ".join(libs + ([old] if old else []))


def test_host_logic_under_sanitizers(tmp_path):
    exe = tmp_path / "host_checks"
    subprocess.check_call(["g++", "-std=c++17", "-O1", "-g", "-Wall", *SAN, "-I", CSRC,
                           "-I", os.path.join(ROOT, "include"), os.path.join(CSRC, "host.cpp"),
                           os.path.join(ROOT, "tests", "native", "host_checks.cpp"), "-o", str(exe)])
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=600,
                       env=dict(os.environ, ASAN_OPTIONS="detect_leaks=1"))
    assert r.returncode == 0, r.stdout + r.stderr
    assert "host checks: ok" in r.stdout


def _oracle_so(tmp_path, src_text=None):
    src = os.path.join(ROOT, "oracle", "lbm_oracle.c")
    if src_text is not None:
        (tmp_path / "lbm_oracle.c").write_text(src_text)
        shutil.copy(os.path.join(ROOT, "oracle", "lbm_oracle.h"), tmp_path / "lbm_oracle.h")
        src = str(tmp_path / "lbm_oracle.c")
    so = tmp_path / "liboracle_san.so"
    subprocess.check_call(["gcc", "-O1", "-g", "-std=c11", "-fPIC", "-shared", *SAN, src, "-o", str(so), "-lm"])
    return so


def _run_pins(so, pins, log_dir):
    """Run pin files against the sanitized oracle; sanitizer reports go to
    files under log_dir (pytest's own output capture would swallow them when
    the process dies)."""
    log = os.path.join(str(log_dir), "san")
    env = dict(os.environ, LBM_ORACLE_LIB=str(so), LD_PRELOAD=_runtime_preload(),
               ASAN_OPTIONS=f"detect_leaks=0:verify_asan_link_order=0:log_path={log}",
               UBSAN_OPTIONS=f"print_stacktrace=1:log_path={log}")
    return subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider", *pins], cwd=ROOT,
                          env=env, capture_output=True, text=True, timeout=900)


def test_oracle_pins_under_sanitizers(tmp_path):
    r = _run_pins(_oracle_so(tmp_path), PINS, tmp_path)
    assert r.returncode == 0, r.stdout[-3000:] + r.stderr[-3000:] + _reports(tmp_path)
    assert "passed" in r.stdout
    assert _reports(tmp_path) == ""


def test_sanitizer_reports_a_planted_overflow(tmp_path):
    src = open(os.path.join(ROOT, "oracle", "lbm_oracle.c")).read()
    old = "            fbar[i] = dom->P[dom->L.opp[i] * dom->N + n];"
    assert src.count(old) == 1
    # bounce-back reads one direction array past the end of the state
    planted = src.replace(old, "            fbar[i] = dom->P[dom->L.q * dom->N + n];")
    r = _run_pins(_oracle_so(tmp_path, planted), ["tests/test_oracle_bruteforce.py"], tmp_path)
    assert r.returncode != 0
    assert "heap-buffer-overflow" in _reports(tmp_path)


def _reports(log_dir):
    out = []
    for name in sorted(os.listdir(str(log_dir))):
        if name.startswith("san."):
            out.append(open(os.path.join(str(log_dir), name)).read())
    return "".join(out)
