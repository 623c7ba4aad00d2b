"""Brute-force reference for tiny inputs, written from the paper's geometry.

Independent of the oracle's scaled-integer formulation: corners and centres
are placed in the (m, b) plane as float64 numbers and the paper's own
expression F(x0, y0) = y0 - m*x0 - b (Sec. 2) is evaluated for each corner
against the parameter line b = v - u*m (slope -u, intercept v).  Every
operand is a dyadic rational with few significant bits for the sizes these
tests use (S <= 64, depth <= 6), so float64 evaluates F exactly; see
``assert_exact_sizes``.

Nothing here is hierarchical: every region of every level is tested
against every line.
"""
from __future__ import annotations

from fractions import Fraction

import numpy as np


def assert_exact_sizes(S: int, dmax: int) -> None:
    # b_c has at most log2(3S) + dmax + 1 bits, u*m_c at most log2(S) + dmax + 2;
    # squares in the circle test double that.  Keep everything far below 53.
    assert S <= 64 and dmax <= 6, "brute force is only exact for tiny sizes"


def corner_grid(S: int, level: int):
    n = 1 << level
    mc = -1.0 + 2.0 * np.arange(n + 1, dtype=np.float64) / n      # m of corner columns
    bc = -float(S) + 3.0 * S * np.arange(n + 1, dtype=np.float64) / n  # b of corner rows
    return mc, bc


def codes(u: np.ndarray, v: np.ndarray, S: int, level: int) -> np.ndarray:
    """4-bit codes, shape (2^l, 2^l, E), index [i, j, k]; NE is the leftmost bit."""
    mc, bc = corner_grid(S, level)
    u = u.astype(np.float64)
    v = v.astype(np.float64)
    # F(corner) = b_c - (-u) * m_c - v; the corner is below the line when F < 0
    F = bc[None, :, None] + mc[:, None, None] * u[None, None, :] - v[None, None, :]
    below = (F < 0).astype(np.int64)
    ne = below[1:, 1:]
    nw = below[:-1, 1:]
    sw = below[:-1, :-1]
    se = below[1:, :-1]
    return 8 * ne + 4 * nw + 2 * sw + se


def crosses_code(u, v, S, level) -> np.ndarray:
    c = codes(u, v, S, level)
    return (c != 0) & (c != 15)


def crosses_circle(u, v, S, level) -> np.ndarray:
    """Distance from region centre to the line <= circumradius, measured in
    units where a region is a unit square (its circumradius is sqrt(2)/2)."""
    n = 1 << level
    ic = np.arange(n, dtype=np.float64)
    mcen = -1.0 + (2.0 * ic + 1.0) / n
    bcen = -float(S) + 3.0 * S * (2.0 * ic + 1.0) / (2 * n)
    dm, db = 2.0 / n, 3.0 * S / n
    u = u.astype(np.float64)
    v = v.astype(np.float64)
    g = bcen[None, :, None] + mcen[:, None, None] * u[None, None, :] - v[None, None, :]
    # squared distance g^2 / (db^2 + u^2 dm^2) <= 1/2
    return 2.0 * g * g <= (db * db + (u * dm) ** 2)[None, None, :]


def crosses(u, v, S, level, variant):
    return crosses_code(u, v, S, level) if variant == "code" else crosses_circle(u, v, S, level)


def fraction_below(S: int, level: int, ic: int, jc: int, u: int, v: int) -> bool:
    """Exact rational version of the corner test (Sec. 2)."""
    n = 1 << level
    m = Fraction(-1) + Fraction(2 * ic, n)
    b = Fraction(-S) + Fraction(3 * S * jc, n)
    F = b + u * m - v          # y0 - m*x0 - b with the parameter line's slope -u
    return F < 0


def fraction_code(S, level, i, j, u, v) -> int:
    return (8 * fraction_below(S, level, i + 1, j + 1, u, v)
            + 4 * fraction_below(S, level, i, j + 1, u, v)
            + 2 * fraction_below(S, level, i, j, u, v)
            + fraction_below(S, level, i + 1, j, u, v))


def fraction_circle(S, level, i, j, u, v) -> bool:
    n = 1 << level
    mcen = Fraction(-1) + Fraction(2 * i + 1, n)
    bcen = Fraction(-S) + Fraction(3 * S * (2 * j + 1), 2 * n)
    g = bcen + u * mcen - v
    dm, db = Fraction(2, n), Fraction(3 * S, n)
    return 2 * g * g <= db * db + u * u * dm * dm


def side_pow2(W, H):
    S = 1
    while S < max(W, H):
        S *= 2
    return S


def brute_detect(x, y, W, H, T, dmax=0, variant="code", passes=3):
    """Closed form of the hierarchy: for every level, the direct votes of
    every region; a region is evaluated iff it is the root or its parent has
    more than T votes (child voters are a subset of parent voters, so every
    ancestor then has more than T too).  Returns (cells, stats) with cells a
    list of (pass, i, j, votes, members) in (pass, key) order and stats[pass]
    an (dmax+1, 6) int64 array: evaluated, votes, split, detected,
    code_tests, entries."""
    S = side_pow2(W, H)
    if dmax == 0:
        dmax = S.bit_length() - 1
    if dmax < 0:
        dmax = 0
    assert_exact_sizes(S, dmax)
    x = np.asarray(x, dtype=np.int64)
    y = np.asarray(y, dtype=np.int64)
    cells, stats = [], {}
    for p in (0, 1):
        if not passes & (1 << p):
            continue
        u, v = (x, y) if p == 0 else (y, x)
        st = np.zeros((dmax + 1, 6), dtype=np.int64)
        votes = []
        cross_levels = []
        for l in range(dmax + 1):
            cr = crosses(u, v, S, l, variant)
            cross_levels.append(cr)
            votes.append(cr.sum(axis=2))
        for l in range(dmax + 1):
            n = 1 << l
            for i in range(n):
                for j in range(n):
                    if l == 0:
                        ev, cand = True, x.size
                    else:
                        pv = votes[l - 1][i // 2, j // 2]
                        ev, cand = pv > T, pv
                    if not ev:
                        continue
                    vv = int(votes[l][i, j])
                    st[l, 0] += 1
                    st[l, 1] += vv
                    st[l, 4] += cand
                    if vv > T:
                        if l == dmax:
                            st[l, 3] += 1
                        else:
                            st[l, 2] += 1
                            st[l, 5] += vv
        stats[p] = st
        fin = votes[dmax]
        found = []
        for i in range(1 << dmax):
            for j in range(1 << dmax):
                if fin[i, j] > T and (dmax == 0 or votes[dmax - 1][i // 2, j // 2] > T):
                    found.append((key_of(i, j, dmax), i, j))
        for _, i, j in sorted(found):
            mem = np.nonzero(cross_levels[dmax][i, j])[0].astype(np.int32)
            cells.append((p, i, j, int(fin[i, j]), mem))
    return cells, stats


def key_of(i: int, j: int, depth: int) -> int:
    """Quad digits NE=0, NW=1, SW=2, SE=3 along the path, most significant first."""
    key = 0
    for lv in range(depth - 1, -1, -1):
        e, n = (i >> lv) & 1, (j >> lv) & 1
        digit = {(1, 1): 0, (0, 1): 1, (0, 0): 2, (1, 0): 3}[(e, n)]
        key = key * 4 + digit
    return key


def recursive_search(x, y, W, H, T, dmax=0, pass_=0):
    """The hierarchical search of Sec. 3 written as a recursion over sets,
    from the method's definition rather than from its printed listing: a
    region's voters are the lines of its candidate set (its parent's
    voters; every line at the root) whose 4-bit code is neither 0000 nor
    1111; a region with more than T voters recurses into its children in
    quad order NE, NW, SW, SE, or, at the finest level, is reported with its
    voters.  Sets are boolean masks over all lines; codes come from
    ``codes`` (float64 corner geometry), not from the oracle.  Returns the
    detected (i, j, votes, members) in visiting order and the total votes
    of all evaluated regions."""
    S = side_pow2(W, H)
    if dmax == 0:
        dmax = S.bit_length() - 1
    assert_exact_sizes(S, dmax)
    x = np.asarray(x, dtype=np.int64)
    y = np.asarray(y, dtype=np.int64)
    u, v = (x, y) if pass_ == 0 else (y, x)
    cross = {l: crosses_code(u, v, S, l) for l in range(dmax + 1)}
    found = []
    total = 0

    def visit(level, i, j, cand):
        nonlocal total
        voters = cand & cross[level][i, j]
        n = int(voters.sum())
        total += n
        if n <= T:
            return
        if level == dmax:
            found.append((i, j, n, np.nonzero(voters)[0].astype(np.int32)))
            return
        for e, nn in ((1, 1), (0, 1), (0, 0), (1, 0)):   # NE, NW, SW, SE
            visit(level + 1, 2 * i + e, 2 * j + nn, voters)

    visit(0, 0, 0, np.ones(x.size, dtype=bool))
    return found, total
