"""The host setup and the C ABI (setup.cpp, capi.cpp) under the address and
undefined-behaviour sanitizers, on the CPU: the library's host objects are
rebuilt with -fsanitize=address,undefined (kernels from the ordinary build),
and the C-ABI tests (tests/test_abi_cpu.py: setup of several workloads,
exports, the error paths and the singular block) run against that build in
a fresh process with the sanitizer runtimes preloaded.  Any report fails the
run (UBSan halts on the first error; ASan aborts)."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

pytestmark = pytest.mark.slow


def _runtime(name):
    return subprocess.check_output(["gcc", f"-print-file-name={name}"], text=True).strip()


def test_abi_tests_pass_under_asan_and_ubsan():
    sys.path.insert(0, ROOT)
    import paper_2609_14982_amd.build as libbuild
    lib = libbuild.build_sanitize()
    env = dict(os.environ)
    env["LD_PRELOAD"] = _runtime("libasan.so") + ":" + _runtime("libubsan.so")
    env["ASAN_OPTIONS"] = "detect_leaks=0:verify_asan_link_order=0"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
    env["FMBTF_LIB"] = lib
    probe = ("import paper_2609_14982_amd as fm; lib = fm.load(); "
             "print(fm.lib_path()); print(hasattr(lib, '__asan_init'), hasattr(lib, '__ubsan_handle_add_overflow'))")
    out = subprocess.run([sys.executable, "-c", probe], cwd=ROOT, env=env, capture_output=True, text=True, timeout=300)
    assert out.returncode == 0, out.stderr[-3000:]
    lines = out.stdout.split()
    assert lines[0] == lib and lines[1] == "True", out.stdout
    run = subprocess.run([sys.executable, "-m", "pytest", "tests/test_abi_cpu.py", "-q", "-x", "-p", "no:cacheprovider"],
                         cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    log = run.stdout + run.stderr
    assert run.returncode == 0, log[-4000:]
    assert "runtime error" not in log and "AddressSanitizer" not in log, log[-4000:]
