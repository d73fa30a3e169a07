"""The pins must catch plausible mistakes in the oracle's pointwise stage.

Each case plants one mistake in a copy of the oracle's C source (the clamp of
z1 to [eps, 1 - eps] of the inert Strang source stage, Sec. 3), builds it on
the CPU and runs the clamp pins of ``test_oracle_clamp.py`` against it in a
separate process: every mutant must fail them, the unchanged copy must pass.
"""
import os
import subprocess
import sys

import pytest

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
TESTS = os.path.join(ROOT, "tests")

# (name, text in the oracle's source, replacement): each text occurs once.
# The full step clamps in clamp_z, the sampled-cell step on its own.
_FULL = "    long N = (long)P->nx * P->ny, k;\n    double lo = P->zeps, hi = 1.0 - P->zeps;"
_CELL = "            double lo = P->zeps, hi = 1.0 - P->zeps;\n            qo[5]"
MUTANTS = [
    ("no clamp", "    clamp_z(P, U);\n", "\n"),
    ("clamp to [0, 1]", _FULL, _FULL.replace("P->zeps, hi = 1.0 - P->zeps", "0.0, hi = 1.0")),
    ("fixed eps", _FULL, _FULL.replace("P->zeps, hi = 1.0 - P->zeps", "1e-6, hi = 1.0 - 1e-6")),
    ("wrong plane", "double *z = U + 5 * N;", "double *z = U + 4 * N;"),
    ("floor only", "z[k] = fmin(fmax(z[k], lo), hi);", "z[k] = fmax(z[k], lo);"),
    ("ceiling only", "z[k] = fmin(fmax(z[k], lo), hi);", "z[k] = fmin(z[k], hi);"),
    ("cells: no clamp", "            qo[5] = fmin(fmax(qo[5], lo), hi);\n", "\n"),
    ("cells: clamp to [0, 1]", _CELL,
     _CELL.replace("P->zeps, hi = 1.0 - P->zeps", "0.0, hi = 1.0")),
    ("cells: wrong plane", "qo[5] = fmin(fmax(qo[5], lo), hi);",
     "qo[4] = fmin(fmax(qo[4], lo), hi);"),
]


def _run_pins(lib):
    env = dict(os.environ, MESO_ORACLE_LIB=lib)
    code = ("import sys; sys.path[:0] = [%r, %r]; import test_oracle_clamp as t; t.run_all()"
            % (ROOT, TESTS))
    return subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True,
                          timeout=120)


def _variant(tmp_path, name, text):
    src = tmp_path / f"{name}.c"
    src.write_text(text)
    return oracle.build_variant(str(src), str(tmp_path / f"{name}.so"))


def test_unchanged_copy_passes(tmp_path):
    text = open(oracle.SOURCE).read()
    r = _run_pins(_variant(tmp_path, "control", text))
    assert r.returncode == 0, r.stderr[-2000:]


@pytest.mark.parametrize("name,old,new", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_mutant_fails_clamp_pins(tmp_path, name, old, new):
    text = open(oracle.SOURCE).read()
    assert text.count(old) == 1, f"mutation site of '{name}' not unique"
    r = _run_pins(_variant(tmp_path, name.replace(" ", "_").replace(",", ""),
                           text.replace(old, new)))
    assert r.returncode != 0, f"mutant '{name}' passes the clamp pins"
    assert "AssertionError" in r.stderr, r.stderr[-2000:]
