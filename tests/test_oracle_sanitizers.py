"""The oracle under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

Two builds of the oracle's C source:

* ASan + UBSan, as one executable with a driver that calls every entry point
  on small problems (degenerate grids, both limiters and walls, both sweep
  orders, the sampled-cell step, the Cochran-Chan and reactive liquids, the
  diagnostics): it must run clean, with every error fatal;
* UBSan as the shared library the tests load: the oracle's pin suites run
  against it in a separate process and must pass.
"""
import os
import subprocess
import sys

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
TESTS = os.path.join(ROOT, "tests")
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"]


def test_asan_ubsan_driver(tmp_path):
    exe = str(tmp_path / "oracle_san")
    subprocess.run(["gcc", "-O1", "-g", "-std=c99", "-ffp-contract=off", *SAN, "-I",
                    os.path.dirname(oracle.SOURCE), "-o", exe,
                    os.path.join(TESTS, "oracle_sanitize_driver.c"), "-lm"], check=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, r.stderr[-4000:]
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr
    assert "oracle sanitize driver: ok" in r.stdout


def test_ubsan_pins(tmp_path):
    lib = oracle.build_variant(oracle.SOURCE, str(tmp_path / "oracle_ubsan.so"),
                               ["-fsanitize=undefined", "-fno-sanitize-recover=all"])
    env = dict(os.environ, MESO_ORACLE_LIB=lib, UBSAN_OPTIONS="print_stacktrace=1")
    suites = ["test_oracle_pins.py", "test_oracle_clamp.py", "test_oracle_cochran_chan.py",
              "test_oracle_reaction.py", "test_oracle_diagnostics.py",
              "test_oracle_positivity.py"]
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider",
                        *[os.path.join(TESTS, s) for s in suites]],
                       cwd=ROOT, capture_output=True, text=True, env=env, timeout=900)
    assert r.returncode == 0, (r.stdout[-3000:], r.stderr[-3000:])
    assert "runtime error" not in r.stderr, r.stderr[-3000:]
