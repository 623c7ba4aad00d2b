"""Pins of the CPU oracle against what the paper and the mathematics fix.

* Corner test and 4-bit code (Sec. 2): exact rationals from the paper's
  F(x0, y0) = y0 - m*x0 - b, including corners lying exactly on a line
  (positive or zero means above).
* Code alphabet: with u >= 0 the parameter line never rises to the east, so
  only 0000, 0010, 0011, 0111 and 1111 occur, the root code is 0011 for
  every edge point (every line crosses level 0, Sec. 3), and a line crosses
  iff SW is below and NE is not.
* Whole detection: brute force over every region of every level
  (tests/brute.py) equals the hierarchical oracle -- cells, votes, members
  and per-level statistics -- for all thresholds 0..15, both passes, both
  variants, square and non-square tiny images and depth overrides.
* Hand closed form: a horizontal image line y = c (pass 0) in the two
  columns next to m = 0.
* The search of Sec. 3 written as a recursion over candidate sets (float64
  geometry, no oracle code) visits and detects the same cells in the same
  order, with the same total votes.
* Invariants and metamorphic relations: child voters within parent voters;
  a crossing line crosses 1..3 children (code variant); circle voters contain code voters;
  point permutation, duplication with T' = 2T + 1, and the x <-> y swap.
"""
import itertools
import os

import numpy as np
import pytest

import brute

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def tiny_image(seed, W, H, p):
    rng = np.random.default_rng(seed)
    return (rng.random((H, W)) < p).astype(np.uint8)


def points(img):
    ys, xs = np.nonzero(img)
    return xs.astype(np.int32), ys.astype(np.int32)


# --------------------------------------------------------------------------
# Sec. 2: the edge points a binary image contributes


def test_edge_points_row_major(orc):
    """Edge points are the nonzero pixels, ranked in row-major order (y, then
    x): a hand-made image, then random ones against a plain double loop."""
    img = np.array([[0, 3, 0, 0],
                    [1, 0, 0, 9],
                    [0, 0, 1, 0]], np.uint8)
    x, y = orc.edge_points(img)
    assert x.dtype == np.int32 and y.dtype == np.int32
    assert x.tolist() == [1, 0, 3, 2] and y.tolist() == [0, 1, 1, 2]
    for seed in range(3):
        im = tiny_image(seed, 13, 7, 0.3)
        want = [(c, r) for r in range(im.shape[0]) for c in range(im.shape[1]) if im[r, c]]
        x, y = orc.edge_points(im)
        assert list(zip(x.tolist(), y.tolist())) == want
    x, y = orc.edge_points(np.zeros((5, 6), np.uint8))
    assert len(x) == 0 and len(y) == 0


# --------------------------------------------------------------------------
# Sec. 2: the corner test and getcode()


def test_corner_code_matches_exact_rationals(orc):
    rng = np.random.default_rng(1)
    n_checked = 0
    for S in (1, 2, 4, 16, 64, 1024, 16384):
        for _ in range(300):
            l = int(rng.integers(0, 15))
            n = 1 << l
            i, j = int(rng.integers(0, n)), int(rng.integers(0, n))
            u, v = int(rng.integers(0, S)), int(rng.integers(0, S))
            assert orc.getcode(S, l, i, j, u, v) == brute.fraction_code(S, l, i, j, u, v)
            n_checked += 1
    assert n_checked == 2100


def test_corner_on_line_counts_as_above(orc):
    # the line b = v - u*m through a corner: F = 0 is "positive or zero" -> above
    S, l = 16, 4
    n = 1 << l
    ties = 0
    for i in range(n):
        for j in range(n):
            for u in range(S):
                # choose v so the SW corner (i, j) lies exactly on the line
                # b_c = v - u*m_c  =>  v = b_c + u*m_c, must be an integer in [0, S)
                m = -1 + 2 * i / n
                b = -S + 3 * S * j / n
                vf = b + u * m
                if vf != int(vf) or not (0 <= vf < S):
                    continue
                v = int(vf)
                code = orc.getcode(S, l, i, j, u, v)
                assert (code >> 1) & 1 == 0, (i, j, u, v, code)
                assert code == brute.fraction_code(S, l, i, j, u, v)
                ties += 1
    assert ties > 100


def test_circle_matches_exact_rationals(orc):
    rng = np.random.default_rng(2)
    for S in (1, 2, 16, 256, 16384):
        for _ in range(300):
            l = int(rng.integers(0, 15))
            n = 1 << l
            i, j = int(rng.integers(0, n)), int(rng.integers(0, n))
            u, v = int(rng.integers(0, S)), int(rng.integers(0, S))
            assert orc.circle_test(S, l, i, j, u, v) == brute.fraction_circle(S, l, i, j, u, v)


def test_circle_exhaustive_small_grid(orc):
    # every (region, line) pair of a small grid against exact rationals
    for S, l in ((8, 3), (16, 2), (4, 4)):
        n = 1 << l
        for i, j, u, v in itertools.product(range(n), range(n), range(S), range(S)):
            assert orc.circle_test(S, l, i, j, u, v) == brute.fraction_circle(S, l, i, j, u, v)


def test_circle_never_tangent():
    """No line is ever exactly at circumradius distance from a region centre.

    The scaled test compares D^2 with 2(9S^2 + 4u^2).  For S = 2^s and
    0 <= u < S the right side is never a perfect square (divide out powers
    of 4: u must stay even until 9 + u'^2 = 2k^2 with u' in {0, 1}, which
    has no solution), so "<=" and "<" give the same votes."""
    from math import isqrt
    for s in range(0, 15):
        S = 1 << s
        for u in range(S):
            r = 2 * (9 * S * S + 4 * u * u)
            assert isqrt(r) ** 2 != r


def test_code_alphabet_root_and_cross_rule(orc):
    rng = np.random.default_rng(3)
    seen = set()
    for S in (4, 16, 256, 4096):
        for _ in range(2000):
            l = int(rng.integers(0, 13))
            n = 1 << l
            i, j = int(rng.integers(0, n)), int(rng.integers(0, n))
            u, v = int(rng.integers(0, S)), int(rng.integers(0, S))
            c = orc.getcode(S, l, i, j, u, v)
            seen.add(c)
            ne, sw = (c >> 3) & 1, (c >> 1) & 1
            assert ((c not in (0, 15)) == (sw == 1 and ne == 0))
            assert orc.getcode(S, 0, 0, 0, u, v) == 0b0011
    assert seen <= {0b0000, 0b0010, 0b0011, 0b0111, 0b1111}
    assert {0b0000, 0b0011, 0b1111} <= seen


# --------------------------------------------------------------------------
# Sec. 3: the whole hierarchy against brute force


def _compare(res, cells, stats, passes):
    assert len(res.cells) == len(cells)
    for c, (p, i, j, vv, mem) in enumerate(cells):
        assert (int(res.cells["pass"][c]), int(res.cells["i"][c]), int(res.cells["j"][c])) == (p, i, j)
        assert int(res.cells["votes"][c]) == vv
        assert int(res.cells["key"][c]) == brute.key_of(i, j, res.dmax)
        np.testing.assert_array_equal(res.cell_members(c), mem)
    for p in (0, 1):
        if passes & (1 << p):
            np.testing.assert_array_equal(res.stats[p], stats[p])


CASES = [
    # (W, H, noise, dmax)
    (16, 16, 0.08, 0), (16, 16, 0.3, 0), (8, 8, 0.5, 0), (13, 7, 0.2, 0),
    (5, 16, 0.25, 0), (16, 3, 0.4, 0), (8, 8, 0.2, 5), (4, 4, 0.6, 6),
    (16, 16, 0.15, 2), (1, 1, 1.0, 0), (1, 9, 0.7, 0), (9, 1, 0.7, 0),
    (2, 2, 1.0, 0), (3, 3, 1.0, 3), (16, 16, 1.0, 0), (7, 12, 0.05, 0),
]


@pytest.mark.parametrize("variant", ["code", "circle"])
@pytest.mark.parametrize("case", range(len(CASES)))
def test_hierarchy_equals_brute_force(orc, case, variant):
    W, H, p, dmax = CASES[case]
    for seed in range(4):
        x, y = points(tiny_image(100 * case + seed, W, H, p))
        for T in range(16):
            cells, stats = brute.brute_detect(x, y, W, H, T, dmax, variant)
            res = orc.detect(x, y, W, H, T, dmax, variant)
            _compare(res, cells, stats, 3)


def test_depth_zero_root_is_the_cell(orc):
    x, y = points(tiny_image(5, 6, 6, 0.5))
    for T in (0, len(x) - 1, len(x)):
        res = orc.detect(x, y, 6, 6, T, -1)
        assert res.dmax == 0
        if len(x) > T:
            assert len(res.cells) == 2
            np.testing.assert_array_equal(res.cell_members(0), np.arange(len(x)))
        else:
            assert len(res.cells) == 0


def test_empty_input(orc):
    e = np.zeros(0, dtype=np.int32)
    res = orc.detect(e, e, 64, 64, 0)
    assert len(res.cells) == 0
    assert res.stats[0][0].tolist() == [1, 0, 0, 0, 0, 0]
    assert res.stats[0][1:].sum() == 0


def test_out_of_range_point_rejected(orc):
    with pytest.raises(orc.OracleError):
        orc.detect(np.array([4]), np.array([0]), 4, 4, 0)
    with pytest.raises(orc.OracleError):
        orc.detect(np.array([0]), np.array([-1]), 4, 4, 0)


# --------------------------------------------------------------------------
# hand closed form: a horizontal image line


@pytest.mark.parametrize("c", [5, 7, 8, 10])
def test_horizontal_line_closed_form(orc, c):
    """Pass 0, points (x, c) for x = 0..W-1, W = H = S = 16, depth 4.

    Every parameter line b = c - x*m passes through (0, c).  Column 7 spans
    m in [-1/8, 0]: a line crosses cell (7, j) iff its SW corner is below it
    (b_lo < c + x/8) and its NE corner is not (b_hi >= c); column 8 spans
    m in [0, 1/8]: it crosses (8, j) iff b_lo < c and b_hi >= c - x/8.
    Cell j spans b in [-16 + 3j, -13 + 3j].  For c on a grid line (c = 5 is
    the top of cell 6 and the bottom of cell 7) the x = 0 line misses (7, 7)
    because its SW corner lies on the line, and every line misses (8, 7)."""
    W = 16
    x = np.arange(W, dtype=np.int32)
    y = np.full(W, c, dtype=np.int32)
    for j in range(16):
        blo, bhi = -16 + 3 * j, -13 + 3 * j
        want7 = sum(1 for xx in range(W) if 8 * blo < 8 * c + xx and bhi >= c)
        want8 = sum(1 for xx in range(W) if blo < c and 8 * bhi >= 8 * c - xx)
        assert len(orc.region_voters(x, y, W, W, 0, 4, 7, j)) == want7
        assert len(orc.region_voters(x, y, W, W, 0, 4, 8, j)) == want8
    if c == 5:
        assert len(orc.region_voters(x, y, W, W, 0, 4, 7, 7)) == W - 1
        assert len(orc.region_voters(x, y, W, W, 0, 4, 8, 7)) == 0
        assert len(orc.region_voters(x, y, W, W, 0, 4, 7, 6)) == W
        assert len(orc.region_voters(x, y, W, W, 0, 4, 8, 6)) == W
    # the detection (T = W - 2) finds every cell with W or W-1 votes in these columns
    res = orc.detect(x, y, W, W, W - 2, 0, "code", 1)
    got = {(int(i), int(j)) for i, j in zip(res.cells["i"], res.cells["j"]) if i in (7, 8)}
    want = set()
    for j in range(16):
        for i in (7, 8):
            if len(orc.region_voters(x, y, W, W, 0, 4, i, j)) > W - 2:
                want.add((i, j))
    assert got == want and len(want) >= 2


# --------------------------------------------------------------------------
# the search as a recursion over candidate sets


@pytest.mark.parametrize("seed", range(6))
def test_recursive_search_same_cells(orc, seed):
    W, H = (16, 16) if seed % 2 == 0 else (11, 14)
    x, y = points(tiny_image(700 + seed, W, H, 0.12))
    for T in (0, 2, 4, 7):
        for p in (0, 1):
            out, total = brute.recursive_search(x, y, W, H, T, 0, p)
            res = orc.detect(x, y, W, H, T, 0, "code", 1 << p)
            assert len(out) == len(res.cells)
            for c, (i, j, vv, mem) in enumerate(out):
                assert (int(res.cells["i"][c]), int(res.cells["j"][c])) == (i, j)
                assert int(res.cells["votes"][c]) == vv
                np.testing.assert_array_equal(res.cell_members(c), mem)
            if len(x) > T:
                assert total == int(res.stats[p][:, 1].sum())


# --------------------------------------------------------------------------
# invariants


def test_child_voters_within_parent_and_one_to_three_children(orc):
    rng = np.random.default_rng(9)
    W = H = 64
    x, y = points(tiny_image(11, W, H, 0.05))
    for _ in range(200):
        l = int(rng.integers(0, 6))
        n = 1 << l
        i, j, p = int(rng.integers(0, n)), int(rng.integers(0, n)), int(rng.integers(0, 2))
        for variant in ("code", "circle"):
            par = set(orc.region_voters(x, y, W, H, p, l, i, j, variant).tolist())
            hits = {k: 0 for k in par}
            for e, nn in ((1, 1), (0, 1), (0, 0), (1, 0)):
                ch = set(orc.region_voters(x, y, W, H, p, l + 1, 2 * i + e, 2 * j + nn,
                                           variant).tolist())
                assert ch <= par
                for k in ch:
                    hits[k] += 1
            if variant == "code":
                assert all(1 <= h <= 3 for h in hits.values())
            else:
                # child discs lie inside the parent disc but do not cover it:
                # a line can graze the parent's circle and miss all four children
                assert all(0 <= h <= 4 for h in hits.values())


def test_circle_contains_code(orc):
    rng = np.random.default_rng(10)
    W = H = 128
    x, y = points(tiny_image(12, W, H, 0.02))
    for _ in range(100):
        l = int(rng.integers(0, 8))
        n = 1 << l
        i, j, p = int(rng.integers(0, n)), int(rng.integers(0, n)), int(rng.integers(0, 2))
        code = set(orc.region_voters(x, y, W, H, p, l, i, j, "code").tolist())
        circ = set(orc.region_voters(x, y, W, H, p, l, i, j, "circle").tolist())
        assert code <= circ
    rc = orc.detect(x, y, W, H, 6, 0, "code")
    rk = orc.detect(x, y, W, H, 6, 0, "circle")
    kc = set(zip(rc.cells["pass"].tolist(), rc.cells["i"].tolist(), rc.cells["j"].tolist()))
    kk = set(zip(rk.cells["pass"].tolist(), rk.cells["i"].tolist(), rk.cells["j"].tolist()))
    assert kc <= kk
    # Table 1's qualitative finding: the circle test casts more votes
    assert sum(int(s[:, 1].sum()) for s in rk.stats.values()) > \
        sum(int(s[:, 1].sum()) for s in rc.stats.values())


def test_metamorphic_permutation_duplication_swap(orc):
    import synth
    img = synth.full_span_image(4, 64, 64, 4, 0.01)
    x, y = points(img)
    T = 20
    base = orc.detect(x, y, 64, 64, T)
    # permutation of the edge points: same cells, members mapped
    perm = np.random.default_rng(0).permutation(len(x))
    px, py = x[perm], y[perm]
    res = orc.detect(px, py, 64, 64, T)
    np.testing.assert_array_equal(res.cells[["pass", "i", "j", "key", "votes"]],
                                  base.cells[["pass", "i", "j", "key", "votes"]])
    for c in range(len(base.cells)):
        np.testing.assert_array_equal(np.sort(perm[res.cell_members(c)]), base.cell_members(c))
    # every point twice and T' = 2T + 1: same cells, doubled votes
    dx, dy = np.concatenate([x, x]), np.concatenate([y, y])
    res = orc.detect(dx, dy, 64, 64, 2 * T + 1)
    np.testing.assert_array_equal(res.cells[["pass", "i", "j"]], base.cells[["pass", "i", "j"]])
    np.testing.assert_array_equal(res.cells["votes"], 2 * base.cells["votes"])
    # x <-> y with W <-> H swaps the passes
    W, H = 48, 64
    img2 = synth.full_span_image(5, W, H, 4, 0.01)
    x2, y2 = points(img2)
    a = orc.detect(x2, y2, W, H, 15)
    b = orc.detect(y2, x2, H, W, 15)
    for p in (0, 1):
        ca, cb = a.pass_cells(p), b.pass_cells(1 - p)
        np.testing.assert_array_equal(ca[["i", "j", "key", "votes"]], cb[["i", "j", "key", "votes"]])
        np.testing.assert_array_equal(a.stats[p], b.stats[1 - p])


def test_solution_removal_equals_dfs_with_removal(orc):
    """solution() with removal (Sec. 3) as a greedy walk in key order equals
    the depth-first search that zeroes the codes of plotted points."""
    for seed in range(8):
        W = H = 16
        x, y = points(tiny_image(900 + seed, W, H, 0.15))
        for T in (1, 3, 5):
            cells, keep, plotted = orc.solution(x, y, W, H, T, 0, 0)
            want_cells, want_plot = _dfs_with_removal(x, y, W, H, T)
            got = [(int(c["i"]), int(c["j"])) for c, k in zip(cells, keep) if k]
            assert got == want_cells
            np.testing.assert_array_equal(plotted, want_plot)


def _dfs_with_removal(x, y, W, H, T):
    S = brute.side_pow2(W, H)
    D = S.bit_length() - 1
    u, v = np.asarray(x, np.int64), np.asarray(y, np.int64)
    cr = {l: brute.crosses_code(u, v, S, l) for l in range(D + 1)}
    removed = np.zeros(len(x), dtype=bool)
    kept = []

    def visit(l, i, j, cand):
        live = cand & cr[l][i, j] & ~removed
        if live.sum() <= T:
            return
        if l == D:
            kept.append((i, j))
            removed[live] = True
            return
        for e, n in ((1, 1), (0, 1), (0, 0), (1, 0)):
            visit(l + 1, 2 * i + e, 2 * j + n, live)

    visit(0, 0, 0, np.ones(len(x), dtype=bool))
    return kept, removed


# --------------------------------------------------------------------------
# golden regression fixture (written by tests/golden/make_golden.py)


def test_golden_line256(orc):
    import json
    import synth
    with open(os.path.join(GOLDEN, "line256_seed0.json")) as f:
        g = json.load(f)
    w = synth.workload("line256", 0)
    x, y = orc.edge_points(w.image)
    assert len(x) == g["E"]
    res = orc.detect(x, y, w.width, w.height, w.threshold, w.max_depth)
    for p in (0, 1):
        assert res.stats[p].tolist() == g["stats"][str(p)]
    assert len(res.cells) == g["n_cells"]
    assert int(res.members.astype(np.int64).sum()) == g["members_sum"]


def test_solution_removal_closed_forms(orc):
    """One row of W collinear points (optionally each point twice): every
    point's parameter line passes through (m, b) = (0, row), and with T one
    below the number of points only cells crossed by every line are detected.
    The first of them in key order is kept and plots every point, so no later
    cell has a live voter: exactly one kept cell, every point plotted (Sec. 3,
    solution()).  Rows inside a cell and on a b grid line, both passes."""
    for W, H, row, dup in ((32, 32, 7, 1), (32, 32, 5, 1), (64, 16, 9, 1), (20, 40, 13, 2)):
        x = np.tile(np.arange(W), dup).astype(np.int32)
        y = np.full(W * dup, row, dtype=np.int32)
        n = W * dup
        cells, keep, plotted = orc.solution(x, y, W, H, n - 1, 0, 0)
        assert len(cells) >= 3 and (cells["votes"] == n).all(), (W, row)   # removal must skip cells 2..n
        assert keep.sum() == 1 and keep[0] and plotted.all(), (W, row)
        # the same row read as a column goes to pass 1
        cells, keep, plotted = orc.solution(y, x, H, W, n - 1, 0, 1)
        assert keep.sum() == 1 and keep[0] and plotted.all(), (W, row, "pass 1")
