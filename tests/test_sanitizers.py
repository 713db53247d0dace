"""CPU sanitizer runs: the oracle (gcc, AddressSanitizer + UndefinedBehaviorSanitizer)
under its pins, and the host code of libsparkling.so (clang's sanitizers on
the host pass only) under the C-ABI validation tests.  Each suite runs in a
child process with the sanitizer runtime preloaded; any report aborts it."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

pytestmark = pytest.mark.slow

MAPS_CHECK = """
import sys
sys.path.insert(0, {root!r})
{load}
maps = open("/proc/self/maps").read()
assert {lib!r} in maps, "sanitized library not mapped"
assert {runtime!r} in maps, "sanitizer runtime not mapped"
print("mapped", {lib!r})
"""


def run_child(args, env_extra, timeout):
    env = dict(os.environ)
    env.update(env_extra)
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=1"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
    r = subprocess.run(args, cwd=ROOT, env=env, capture_output=True, text=True, timeout=timeout)
    assert r.returncode == 0, (r.stdout[-4000:], r.stderr[-4000:])
    assert "ERROR: AddressSanitizer" not in r.stderr and "runtime error:" not in r.stderr
    return r


def test_oracle_pins_under_asan_ubsan(tmp_path):
    import oracle
    lib = str(oracle.build_sanitized(tmp_path))
    runtime = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True,
                             text=True, check=True).stdout.strip()
    runtime = os.path.realpath(runtime)
    env = {"SPK_ORACLE_LIB": lib, "LD_PRELOAD": runtime}
    code = MAPS_CHECK.format(root=ROOT, lib=lib, runtime=runtime,
                             load="import oracle\noracle.num_threads()")
    run_child([sys.executable, "-c", code], env, 120)
    run_child([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
               "tests/test_oracle_pins.py", "tests/test_step_policy.py"], env, 900)


def test_host_library_validation_under_asan_ubsan(tmp_path):
    from paper_2108_02991_amd import build
    lib = str(build.build_sanitized(tmp_path))
    runtime = os.path.realpath(build.asan_runtime())
    env = {"SPK_LIBRARY": lib, "LD_PRELOAD": runtime}
    code = MAPS_CHECK.format(root=ROOT, lib=lib, runtime=runtime,
                             load="import paper_2108_02991_amd as spk\nspk.load_library()")
    run_child([sys.executable, "-c", code], env, 120)
    run_child([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
               "tests/test_abi_cpu.py"], env, 600)
