"""The oracle's own tests once more against an AddressSanitizer +
UndefinedBehaviorSanitizer build of the oracle (every report fatal), in a
child process that preloads libasan. Out-of-bounds reads or writes, use
after free and undefined arithmetic (signed overflow, bad shifts, invalid
enum-to-int paths) anywhere in the paths those tests drive end the child with
a report and fail this test."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _runtime(name):
    p = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True, text=True)
    path = p.stdout.strip()
    return path if os.path.isabs(path) and os.path.exists(path) else None


@pytest.mark.slow
def test_oracle_tests_under_asan_and_ubsan(tmp_path):
    asan = _runtime("libasan.so")
    if asan is None:
        pytest.skip("gcc has no libasan runtime here")
    sys.path.insert(0, ROOT)
    from oracle import oracle
    lib = oracle.build(force=True, out=str(tmp_path / "liboracle_asan.so"), sanitize=True)
    env = dict(os.environ)
    env.update(LD_PRELOAD=asan, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1", MCRT_ORACLE_LIB=lib)
    # the sanitized library is the one the child maps
    probe = ("import sys; sys.path.insert(0, %r)\n"
             "from oracle import oracle\n"
             "oracle.use_library(%r); oracle.lib()\n"
             "maps = open('/proc/self/maps').read()\n"
             "assert %r in maps and 'libasan' in maps\n" % (ROOT, lib, lib))
    subprocess.run([sys.executable, "-c", probe], env=env, check=True, timeout=120)
    r = subprocess.run(
        [sys.executable, "-m", "pytest", os.path.join(ROOT, "tests"), "-q", "-x", "-m", "not gpu",
         "-k", "oracle and not sanitized", "-n", "4", "-p", "no:cacheprovider"],
        env=env, cwd=ROOT, capture_output=True, text=True, timeout=1200)
    tail = (r.stdout + r.stderr)[-4000:]
    assert r.returncode == 0, tail
    assert " passed" in r.stdout, tail
