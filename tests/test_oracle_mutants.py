"""The pins are strong enough: every plausible mistake planted in a copy of
the oracle's source (a flipped sign, a transposed operand, a dropped term, a
wrong rounding or clamp, an off-by-one, a swapped index) is compiled on the
CPU and must make at least one pin fail. The committed oracle is untouched."""
import json
import os
import subprocess
import sys

import pytest

import oracle
import test_oracle_pins as pins

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)

# Runs every pin against one compiled oracle in a process of its own (a
# mutant may write out of bounds; a crash counts as caught) and prints the
# names of the pins that failed.
RUNNER = """
import json, sys
sys.path[:0] = [{root!r}, {here!r}]
import oracle, test_oracle_pins as pins
O = oracle.Oracle({lib!r})
failed = []
for pin in pins.PINS:
    try:
        pin(O)
    except Exception:
        failed.append(pin.__name__)
print(json.dumps(failed))
"""

SRC = open(os.path.join(os.path.dirname(oracle.__file__), "tdct_oracle.c")).read()

# (name, text in tdct_oracle.c, replacement)
MUTANTS = [
    ("T entry sign", "    {0, 0, -1, 0, 0, 1, 0, 0},", "    {0, 0, -1, 0, 0, -1, 0, 0},"),
    ("T entry dropped", "    {0, -1, 1, 0, 0, 1, -1, 0},", "    {0, -1, 1, 0, 0, 0, -1, 0},"),
    ("T rows swapped", "    {1, 0, 0, 0, 0, 0, 0, -1},\n    {1, 0, 0, -1, -1, 0, 0, 1},",
     "    {1, 0, 0, -1, -1, 0, 0, 1},\n    {1, 0, 0, 0, 0, 0, 0, -1},"),
    ("forward left operand transposed", "s += T[i][r] * X[8 * r + c];", "s += T[r][i] * X[8 * r + c];"),
    ("forward right operand transposed", "s += M[8 * i + c] * T[j][c];", "s += M[8 * i + c] * T[c][j];"),
    ("inverse left operand untransposed", "s += T[i][r] * W[8 * i + j];", "s += T[r][i] * W[8 * i + j];"),
    ("inverse right operand transposed", "s += M[8 * r + j] * T[j][c];", "s += M[8 * r + j] * T[c][j];"),
    ("1-D transpose ignored", "s += (transpose ? T[n][k] : T[k][n]) * x[n];", "s += T[k][n] * x[n];"),
    ("D^2 scale uses one index", "return 64 / (row_norm2(i) * row_norm2(j));",
     "return 64 / (row_norm2(i) * row_norm2(i));"),
    ("D^2 scale off by a factor", "return 64 / (row_norm2(i) * row_norm2(j));",
     "return 128 / (row_norm2(i) * row_norm2(j));"),
    ("no level shift", "X[8 * r + c] = (int64_t)p[r * stride + c] - 128;",
     "X[8 * r + c] = (int64_t)p[r * stride + c];"),
    ("level shift 127", "X[8 * r + c] = (int64_t)p[r * stride + c] - 128;",
     "X[8 * r + c] = (int64_t)p[r * stride + c] - 127;"),
    ("ties toward zero", "int64_t m = (2 * a + Q) / (2 * Q);", "int64_t m = (2 * a + Q - 1) / (2 * Q);"),
    ("truncating quotient", "int64_t m = (2 * a + Q) / (2 * Q);", "int64_t m = a / Q;"),
    ("negative side not mirrored", "return W < 0 ? -m : m;", "return W < 0 ? -m - (2 * a % (2 * Q) == Q) : m;"),
    ("zigzag orientation flipped", "        if (d % 2 == 1) {", "        if (d % 2 == 0) {"),
    ("zonal keep off by one", "q[k] = rank_of[k] < keep ? oracle_round_div(W, Q[k]) : 0;",
     "q[k] = rank_of[k] <= keep ? oracle_round_div(W, Q[k]) : 0;"),
    ("dequantise dropped", "for (int k = 0; k < 64; ++k) Wp[k] = (int64_t)qb[k] * (int64_t)Q[k];",
     "for (int k = 0; k < 64; ++k) Wp[k] = (int64_t)qb[k];"),
    ("reconstruction rounds with 31", "int64_t v = floor_div(S[8 * r + c] + 32, 64) + 128;",
     "int64_t v = floor_div(S[8 * r + c] + 31, 64) + 128;"),
    ("reconstruction truncates", "int64_t v = floor_div(S[8 * r + c] + 32, 64) + 128;",
     "int64_t v = (S[8 * r + c] + 32) / 64 + 128;"),
    ("reconstruction offset 127", "int64_t v = floor_div(S[8 * r + c] + 32, 64) + 128;",
     "int64_t v = floor_div(S[8 * r + c] + 32, 64) + 127;"),
    ("upper clamp 254", "if (v > 255) v = 255;", "if (v > 254) v = 254;"),
    ("lower clamp missing", "if (v < 0) v = 0;\n            if (v > 255)", "if (v < -1) v = 0;\n            if (v > 255)"),
    ("int8 saturation 126", "if (v > 127) v = 127;", "if (v > 126) v = 126;"),
    ("int8 stored in natural order", "int64_t v = q[order[r]];", "int64_t v = q[r];"),
    ("row stride ignored", "X[8 * r + c] = (int64_t)p[r * stride + c] - 128;",
     "X[8 * r + c] = (int64_t)p[r * w + c] - 128;"),
    ("block coordinates swapped", "int64_t by = b / nbx, bx = b % nbx;\n    const uint8_t* p",
     "int64_t bx = b / nbx, by = b % nbx;\n    const uint8_t* p"),
    ("inverse block placement swapped", "int64_t by = b / nbx, bx = b % nbx;\n        reconstruct_block",
     "int64_t bx = b / nbx, by = b % nbx;\n        reconstruct_block"),
]


@pytest.fixture(scope="module")
def mutant_dir(tmp_path_factory):
    return tmp_path_factory.mktemp("oracle_mutants")


def _failing_pins(lib):
    r = subprocess.run([sys.executable, "-c", RUNNER.format(root=ROOT, here=HERE, lib=lib)],
                       stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True, timeout=300)
    if r.returncode != 0:
        return ["process ended with status %d" % r.returncode]
    return json.loads(r.stdout.strip().splitlines()[-1])


@pytest.mark.parametrize("name,old,new", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_planted_mistake_is_caught(name, old, new, mutant_dir):
    assert SRC.count(old) == 1, "mutation site not unique: " + name
    d = mutant_dir / name.replace(" ", "_").replace("^", "")
    d.mkdir()
    src = d / "tdct_oracle.c"
    src.write_text(SRC.replace(old, new))
    lib = oracle.build(force=True, src=str(src), out=str(d / "liboracle.so"))
    assert _failing_pins(lib), "no pin catches: " + name


def test_unmutated_copy_passes_every_pin(mutant_dir):
    d = mutant_dir / "identity"
    d.mkdir()
    (d / "tdct_oracle.c").write_text(SRC)
    lib = oracle.build(force=True, src=str(d / "tdct_oracle.c"), out=str(d / "liboracle.so"))
    assert _failing_pins(lib) == []
