"""The library's host C++ under AddressSanitizer and UndefinedBehaviorSanitizer:
the ABI tests and the automatic-parameter tests (host code only: argument
checks, mesh tables, Sec. 3.5 parameters) run in a child process against a
build whose host objects carry both sanitizers, with every report fatal.
CPU only."""
import glob
import os
import subprocess
import sys
from pathlib import Path

import pytest

ROOT = Path(__file__).resolve().parents[1]
CSRC = ROOT / "paper_2212_05645_amd" / "csrc"


def _runtime():
    rt = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    return rt[-1] if rt else None


def test_host_code_under_asan_and_ubsan():
    rt = _runtime()
    if rt is None:
        pytest.skip("no AddressSanitizer runtime in this toolchain")
    from paper_2212_05645_amd import build as B
    lib = Path(B.SAN_OUT)
    newest = max(p.stat().st_mtime for p in CSRC.iterdir())
    if not lib.exists() or lib.stat().st_mtime < newest:
        B.build(sanitize=True)
    syms = subprocess.run(["nm", "-D", str(lib)], capture_output=True, text=True, check=True).stdout
    assert "__asan_report_load8" in syms and "__ubsan_handle_" in syms
    env = dict(os.environ, LD_PRELOAD=rt, AVS_LIBRARY=str(lib), PYTHONPATH=str(ROOT),
               ASAN_OPTIONS="detect_leaks=0:halt_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    probe = subprocess.run([sys.executable, "-c", "from paper_2212_05645_amd import avs; print(avs.lib._name)"],
                           cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    assert probe.returncode == 0 and probe.stdout.strip() == str(lib), probe.stderr[-2000:]
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider",
                        "tests/test_abi.py", "tests/test_auto_params.py"],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    out = r.stdout[-3000:] + r.stderr[-3000:]
    assert r.returncode == 0, out
    assert "AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr, out
    assert " passed" in r.stdout, out
