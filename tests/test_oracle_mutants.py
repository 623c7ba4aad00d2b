"""The pins must catch plausible mistakes in the oracle.

Each case below plants one mistake (a flipped tie, a wrong sign, a dropped
term, a swapped index, a wrong quad order ...) in a copy of the oracle's C
source, builds it with gcc into a temporary directory, points the oracle
module at it and runs a quick subset of the pins.  At least one pin must
fail for every mutant; the unmodified source must pass the same subset.
"""
import os
import subprocess

import pytest

import test_oracle_pins as pins

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "hough_oracle.c")

MUTANTS = [
    ("tie rule: corner on the line counted as below",
     "return Bc < v * scale - u * Mc;", "return Bc <= v * scale - u * Mc;"),
    ("sign of the slope column", "const int64_t Mc = 2 * ic - scale;",
     "const int64_t Mc = 2 * ic + scale;"),
    ("b extent 2S instead of 3S", "const int64_t Bc = -S * scale + 3 * S * jc;",
     "const int64_t Bc = -S * scale + 2 * S * jc;"),
    ("dropped scale on v", "return Bc < v * scale - u * Mc;", "return Bc < v - u * Mc;"),
    ("NE and NW bits swapped", "if (corner_below(S, l, i + 1, j + 1, u, v)) code |= 8;",
     "if (corner_below(S, l, i + 1, j + 1, u, v)) code |= 4;"),
    ("SE corner at the wrong row", "if (corner_below(S, l, i + 1, j, u, v))     code |= 1;",
     "if (corner_below(S, l, i + 1, j + 1, u, v)) code |= 1;"),
    ("vote rule drops the 1111 case", "return code != 0 && code != 15;", "return code != 0;"),
    ("threshold >= instead of >", "if (votes <= w->threshold)", "if (votes < w->threshold)"),
    ("quad order NE, SW, NW, SE", "static const int north[4] = {1, 1, 0, 0};",
     "static const int north[4] = {1, 0, 1, 0};"),
    ("children tested against the parent's candidates",
     "int rc = evaluate(w, l + 1, 2 * i + east[q], 2 * j + north[q], voters, votes,",
     "int rc = evaluate(w, l + 1, 2 * i + east[q], 2 * j + north[q], cand, n,"),
    ("pass 1 not swapped", "w.u = pass == 0 ? x : y;   /* pass 1", "w.u = x;   /* pass 1"),
    ("code tests count votes", "st[4] += n;", "st[4] += votes;"),
    ("circle centre off by half a cell",
     "const int64_t D = 3 * S * (2 * j + 1) + 2 * u * (2 * i + 1) - ((v + u + S) << (l + 1));",
     "const int64_t D = 3 * S * (2 * j) + 2 * u * (2 * i + 1) - ((v + u + S) << (l + 1));"),
    ("circle radius 9S^2 -> 8S^2",
     "const __int128 rhs = (__int128)2 * (9 * (__int128)S * S + 4 * (__int128)u * u);",
     "const __int128 rhs = (__int128)2 * (8 * (__int128)S * S + 4 * (__int128)u * u);"),
]
# "lhs <= rhs" versus "lhs < rhs" in the circle test is not a mutant: the two
# agree on every valid input (test_oracle_pins.test_circle_never_tangent).


def _quick_pins(orc):
    pins.test_corner_code_matches_exact_rationals(orc)
    pins.test_circle_matches_exact_rationals(orc)
    pins.test_code_alphabet_root_and_cross_rule(orc)
    for case in (0, 3, 4, 7):
        for variant in ("code", "circle"):
            pins.test_hierarchy_equals_brute_force(orc, case, variant)
    for c in (5, 7):
        pins.test_horizontal_line_closed_form(orc, c)
    pins.test_metamorphic_permutation_duplication_swap(orc)


def _build(src_text, tmp_path, name):
    c = tmp_path / f"{name}.c"
    so = tmp_path / f"lib{name}.so"
    c.write_text(src_text)
    subprocess.run(["gcc", "-O1", "-std=gnu11", "-shared", "-fPIC", "-o", str(so), str(c)],
                   check=True)
    return str(so)


def _run_with(lib_path, orc):
    saved_lib, saved_path = orc._lib, orc._LIB_PATH
    orc._lib, orc._LIB_PATH = None, lib_path
    try:
        _quick_pins(orc)
        return True
    except AssertionError:
        return False
    finally:
        orc._lib, orc._LIB_PATH = saved_lib, saved_path


def test_unmodified_oracle_passes_quick_pins(orc, tmp_path):
    src = open(SRC).read()
    assert _run_with(_build(src, tmp_path, "orig"), orc)


@pytest.mark.parametrize("k", range(len(MUTANTS)))
def test_mutant_is_caught(orc, tmp_path, k):
    what, old, new = MUTANTS[k]
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutation site not found: {what}"
    mutated = src.replace(old, new)
    assert mutated != src
    assert not _run_with(_build(mutated, tmp_path, f"mut{k}"), orc), f"pins missed: {what}"
