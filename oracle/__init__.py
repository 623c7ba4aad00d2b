"""CPU oracle for the hierarchical slope-intercept Hough vote.

TEST INFRASTRUCTURE ONLY.  The oracle is the plain, slow, obviously correct
reference the GPU library is checked against.  Only ``tests/``, the smoke
check and the benchmark's CPU-baseline leg may import it; the GPU library
never does, and the two share no code.

* :func:`edge_points` -- edge staging: the nonzero pixels of a binary image
  in row-major order (the image-space edge points of Sec. 1 / Sec. 3).
* :func:`detect` -- the depth-first hierarchical vote of Sec. 3 with the
  4-bit corner code of Sec. 2 (``variant='code'``) or the circumscribed
  circle test of the comparison method (``variant='circle'``), both passes
  (ALPHA as given, BETA with the axes swapped), implemented in plain C
  (``hough_oracle.c``) with exact integer arithmetic.
* :func:`detect_subtree` -- the same search restricted to one region and
  everything below it (a part of a large search, run or timed on its own).
* :func:`region_voters` -- the voters of one region found by testing every
  line against it directly, with no hierarchy.
* :func:`member_digest` -- the checksum ``detect(..., keep_members="digest")``
  folds a pass's voters into, computed from a voter list.
* :func:`solution` -- solution() of Sec. 3 with the removal of plotted edge
  points, as a greedy walk over the detected cells in depth-first order.
* :func:`sobel_partition` -- the edge front end of Sec. 3: Sobel's gradient
  operator on a gray image gives the edge points and, from the gradient
  direction, the set (ALPHA or BETA) each one belongs to.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass
from typing import Dict

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libhough_oracle.so")
_lib = None

STAT_NAMES = ("evaluated", "votes", "split", "detected", "code_tests", "entries")
VARIANTS = {"code": 0, "circle": 1}
MEMBERS = {False: 0, True: 1, "digest": 2}
DIGEST_A = 0x9E3779B97F4A7C15
DIGEST_B = 0x632BE59BD9B4E019

_i32p = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
_i64p = np.ctypeslib.ndpointer(dtype=np.int64, flags="C_CONTIGUOUS")
_u8p = np.ctypeslib.ndpointer(dtype=np.uint8, flags="C_CONTIGUOUS")


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        from . import build as _b
        _b.build()
    lib = C.CDLL(_LIB_PATH)
    lib.hough_oracle_detect.restype = C.c_void_p
    lib.hough_oracle_detect.argtypes = [C.c_void_p, C.c_void_p, C.c_int64, C.c_int32,
                                        C.c_int32, C.c_int32, C.c_int32, C.c_int32,
                                        C.c_uint32, C.c_int32]
    for name in ("hough_oracle_status", "hough_oracle_n_levels"):
        getattr(lib, name).restype = C.c_int32
        getattr(lib, name).argtypes = [C.c_void_p]
    for name in ("hough_oracle_S", "hough_oracle_n_cells", "hough_oracle_n_members"):
        getattr(lib, name).restype = C.c_int64
        getattr(lib, name).argtypes = [C.c_void_p]
    lib.hough_oracle_cells.restype = None
    lib.hough_oracle_cells.argtypes = [C.c_void_p, _i32p, _i32p, _i32p, _i64p, _i32p, _i64p]
    lib.hough_oracle_members.restype = None
    lib.hough_oracle_members.argtypes = [C.c_void_p, _i32p]
    lib.hough_oracle_stats.restype = None
    lib.hough_oracle_stats.argtypes = [C.c_void_p, C.c_int32, _i64p]
    lib.hough_oracle_free.restype = None
    lib.hough_oracle_free.argtypes = [C.c_void_p]
    lib.hough_oracle_member_digest.restype = C.c_uint64
    lib.hough_oracle_member_digest.argtypes = [C.c_void_p, C.c_int32]
    lib.hough_oracle_pass_members.restype = C.c_int64
    lib.hough_oracle_pass_members.argtypes = [C.c_void_p, C.c_int32]
    lib.hough_oracle_detect_subtree.restype = C.c_void_p
    lib.hough_oracle_detect_subtree.argtypes = [C.c_void_p, C.c_void_p, C.c_int64, C.c_int32, C.c_int32,
                                                C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_int32,
                                                C.c_int64, C.c_int64, C.c_int64, C.c_void_p, C.c_int64,
                                                C.c_int32]
    lib.hough_oracle_region_voters.restype = C.c_int64
    lib.hough_oracle_region_voters.argtypes = [C.c_void_p, C.c_void_p, C.c_int64, C.c_int32,
                                               C.c_int32, C.c_int32, C.c_int32, C.c_int64,
                                               C.c_int64, C.c_int32, C.c_void_p]
    lib.hough_oracle_getcode.restype = C.c_int32
    lib.hough_oracle_getcode.argtypes = [C.c_int64, C.c_int32, C.c_int64, C.c_int64,
                                         C.c_int64, C.c_int64]
    lib.hough_oracle_circle.restype = C.c_int32
    lib.hough_oracle_circle.argtypes = [C.c_int64, C.c_int32, C.c_int64, C.c_int64,
                                        C.c_int64, C.c_int64]
    lib.hough_oracle_solution.restype = C.c_int64
    lib.hough_oracle_solution.argtypes = [C.c_void_p, C.c_int32, C.c_int32, C.c_int64,
                                          _u8p, _u8p]
    _lib = lib
    return lib


class OracleError(RuntimeError):
    pass


def edge_points(image: np.ndarray):
    """Edge points of a binary image: nonzero pixels, row-major (y, then x).

    Returns ``(x, y)`` as int32 arrays; point id = position in this order."""
    img = np.asarray(image)
    if img.ndim != 2:
        raise ValueError("image must be 2-D (H, W)")
    ys, xs = np.nonzero(img)
    return xs.astype(np.int32), ys.astype(np.int32)


def sobel_partition(gray: np.ndarray, edge_threshold: int):
    """Sobel's gradient operator (Sec. 3: edge points are sorted into ALPHA
    and BETA while the operator is applied) on a gray image.

    Gx and Gy are the 3x3 Sobel sums, written out term by term:
    Gx = (p[y-1,x+1] + 2 p[y,x+1] + p[y+1,x+1]) - (p[y-1,x-1] + 2 p[y,x-1] + p[y+1,x-1]),
    Gy = (p[y+1,x-1] + 2 p[y+1,x] + p[y+1,x+1]) - (p[y-1,x-1] + 2 p[y-1,x] + p[y-1,x+1]).
    A pixel with a full 3x3 neighbourhood is an edge point iff
    Gx^2 + Gy^2 > edge_threshold^2 (exact integers); border pixels never are.
    The image line through an edge point runs across its gradient, so its
    slope is -Gx/Gy: the point is in ALPHA (|slope| <= 1, pass 0) iff
    |Gx| <= |Gy|, else in BETA (pass 1, axes swapped).

    Returns ``(x, y, beta)``: all edge points row-major (point id = position)
    and a bool array, True for BETA."""
    p = np.asarray(gray)
    if p.ndim != 2:
        raise ValueError("image must be 2-D (H, W)")
    H, W = p.shape
    xs, ys, beta = [], [], []
    if H >= 3 and W >= 3:
        q = p.astype(np.int64)
        n = q[:-2, 1:-1]
        s_ = q[2:, 1:-1]
        w = q[1:-1, :-2]
        e = q[1:-1, 2:]
        nw, ne, sw, se = q[:-2, :-2], q[:-2, 2:], q[2:, :-2], q[2:, 2:]
        gx = (ne + 2 * e + se) - (nw + 2 * w + sw)
        gy = (sw + 2 * s_ + se) - (nw + 2 * n + ne)
        edge = gx * gx + gy * gy > int(edge_threshold) * int(edge_threshold)
        yy, xx = np.nonzero(edge)
        return ((xx + 1).astype(np.int32), (yy + 1).astype(np.int32),
                (np.abs(gx[yy, xx]) > np.abs(gy[yy, xx])))
    return np.zeros(0, np.int32), np.zeros(0, np.int32), np.zeros(0, bool)


def side_pow2(W: int, H: int) -> int:
    """S = 2^ceil(log2(max(W, H)))."""
    S = 1
    while S < max(W, H):
        S *= 2
    return S


def default_depth(W: int, H: int) -> int:
    """ceil(log2 N) for an N x N image, with N = max(W, H)."""
    return int(side_pow2(W, H)).bit_length() - 1


@dataclass
class OracleResult:
    """Detected cells of all enabled passes in (pass, key) order.

    ``cells`` is a structured array with fields pass, i, j, key, votes,
    member_off; ``members`` holds each cell's voters (ascending ids) at
    ``member_off`` (empty when membership was not kept); ``stats[pass]`` is
    an int64 array of shape (Dmax + 1, 6) with columns ``STAT_NAMES``.
    ``member_digest[pass]`` is the pass's voter checksum (``keep_members=
    "digest"``, else 0) and ``pass_members[pass]`` its number of voters."""
    S: int
    dmax: int
    cells: np.ndarray
    members: np.ndarray
    stats: Dict[int, np.ndarray]
    member_digest: Dict[int, int] = None
    pass_members: Dict[int, int] = None

    def cell_members(self, c: int) -> np.ndarray:
        off = int(self.cells["member_off"][c])
        return self.members[off: off + int(self.cells["votes"][c])]

    def pass_cells(self, p: int) -> np.ndarray:
        return self.cells[self.cells["pass"] == p]

    def code_tests(self) -> int:
        return int(sum(int(s[:, 4].sum()) for s in self.stats.values()))


CELL_DTYPE = np.dtype([("pass", np.int32), ("i", np.int32), ("j", np.int32),
                       ("key", np.int64), ("votes", np.int32), ("member_off", np.int64)])


def _as_i32(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.int32))


def detect(x, y, W: int, H: int, threshold: int, max_depth: int = 0,
           variant: str = "code", passes: int = 3, keep_members=True) -> OracleResult:
    """Hierarchical vote (Sec. 3) of the edge points ``(x, y)`` of a W x H
    image.  ``max_depth=0`` selects ceil(log2(max(W, H))), ``-1`` depth 0.
    ``passes`` bit 0 = pass 0 (|m| <= 1 as given), bit 1 = pass 1 (x, y
    swapped).  ``keep_members``: True stores every cell's voters, False
    none, ``"digest"`` folds them into ``member_digest`` instead."""
    lib = _load()
    x, y = _as_i32(x), _as_i32(y)
    if x.shape != y.shape:
        raise ValueError("x and y must have the same length")
    E = int(x.size)
    h = lib.hough_oracle_detect(x.ctypes.data if E else None, y.ctypes.data if E else None,
                                E, int(W), int(H), int(threshold), int(max_depth),
                                VARIANTS[variant], int(passes), MEMBERS[keep_members])
    return _collect(lib, h, passes)


def detect_subtree(x, y, W: int, H: int, threshold: int, max_depth: int, pass_: int,
                   level: int, i: int, j: int, key: int, cand, variant: str = "code",
                   keep_members=False) -> OracleResult:
    """The search of :func:`detect` for one pass restricted to region
    ``(level, i, j)`` and the regions below it, the region evaluated against
    the lines ``cand`` (the voters of its parent; all lines for the root).
    ``key`` is the region's quad-digit key.  Statistics cover levels >=
    ``level``."""
    lib = _load()
    x, y = _as_i32(x), _as_i32(y)
    cand = _as_i32(cand)
    E = int(x.size)
    h = lib.hough_oracle_detect_subtree(x.ctypes.data if E else None, y.ctypes.data if E else None,
                                        E, int(W), int(H), int(threshold), int(max_depth),
                                        VARIANTS[variant], int(pass_), int(level), int(i), int(j),
                                        int(key), cand.ctypes.data if cand.size else None,
                                        int(cand.size), MEMBERS[keep_members])
    return _collect(lib, h, 1 << int(pass_))


def member_digest(ids) -> int:
    """The checksum of ``keep_members="digest"`` over one pass's voter list
    (cells in key order, voters ascending): sum over positions t of
    (t * A + B) * (id + 1) modulo 2^64."""
    ids = np.asarray(ids, dtype=np.uint64)
    t = np.arange(ids.size, dtype=np.uint64)
    with np.errstate(over="ignore"):
        return int(((t * np.uint64(DIGEST_A) + np.uint64(DIGEST_B)) * (ids + np.uint64(1))).sum(dtype=np.uint64))


def _collect(lib, h, passes) -> OracleResult:
    if not h:
        raise MemoryError("oracle out of memory")
    try:
        st = lib.hough_oracle_status(h)
        if st != 0:
            raise OracleError(f"oracle status {st}")
        nl = lib.hough_oracle_n_levels(h)
        n = lib.hough_oracle_n_cells(h)
        cols = {k: np.zeros(n, dtype=CELL_DTYPE[k]) for k in CELL_DTYPE.names}
        lib.hough_oracle_cells(h, cols["pass"], cols["i"], cols["j"], cols["key"],
                               cols["votes"], cols["member_off"])
        cells = np.zeros(n, dtype=CELL_DTYPE)
        for k in CELL_DTYPE.names:
            cells[k] = cols[k]
        nm = lib.hough_oracle_n_members(h)
        members = np.zeros(nm, dtype=np.int32)
        lib.hough_oracle_members(h, members)
        stats = {}
        for p in (0, 1):
            if passes & (1 << p):
                s = np.zeros(nl * 6, dtype=np.int64)
                lib.hough_oracle_stats(h, p, s)
                stats[p] = s.reshape(nl, 6)
        return OracleResult(int(lib.hough_oracle_S(h)), nl - 1, cells, members, stats,
                            {p: int(lib.hough_oracle_member_digest(h, p)) for p in (0, 1)},
                            {p: int(lib.hough_oracle_pass_members(h, p)) for p in (0, 1)})
    finally:
        lib.hough_oracle_free(h)


def region_voters(x, y, W: int, H: int, pass_: int, level: int, i: int, j: int,
                  variant: str = "code") -> np.ndarray:
    """Ids of the lines voting for region (level, i, j), by direct test."""
    lib = _load()
    x, y = _as_i32(x), _as_i32(y)
    out = np.zeros(max(1, x.size), dtype=np.int32)
    n = lib.hough_oracle_region_voters(x.ctypes.data, y.ctypes.data, x.size, int(W), int(H),
                                       int(pass_), int(level), int(i), int(j),
                                       VARIANTS[variant], out.ctypes.data)
    if n < 0:
        raise ValueError("bad region")
    return out[:n].copy()


def getcode(S: int, level: int, i: int, j: int, u: int, v: int) -> int:
    """4-bit code (NE, NW, SW, SE; NE leftmost) of line b = v - u*m for region (level, i, j)."""
    return int(_load().hough_oracle_getcode(S, level, i, j, u, v))


def circle_test(S: int, level: int, i: int, j: int, u: int, v: int) -> bool:
    """Circumscribed-circle vote of line b = v - u*m for region (level, i, j)."""
    return bool(_load().hough_oracle_circle(S, level, i, j, u, v))


def solution(x, y, W: int, H: int, threshold: int, max_depth: int = 0, pass_: int = 0,
             variant: str = "code"):
    """solution() with removal (Sec. 3) for one pass.

    Returns ``(cells, keep, plotted)``: the pass's detected cells before
    removal, a bool mask of the cells that survive removal, and a bool mask
    over edge points of the plotted (output) points."""
    lib = _load()
    x, y = _as_i32(x), _as_i32(y)
    E = int(x.size)
    h = lib.hough_oracle_detect(x.ctypes.data if E else None, y.ctypes.data if E else None,
                                E, int(W), int(H), int(threshold), int(max_depth),
                                VARIANTS[variant], 1 << pass_, 1)
    try:
        if lib.hough_oracle_status(h) != 0:
            raise OracleError("oracle status")
        n = lib.hough_oracle_n_cells(h)
        keep = np.zeros(max(1, n), dtype=np.uint8)
        plotted = np.zeros(max(1, E), dtype=np.uint8)
        lib.hough_oracle_solution(h, pass_, int(threshold), E, keep, plotted)
        cols = {k: np.zeros(n, dtype=CELL_DTYPE[k]) for k in CELL_DTYPE.names}
        lib.hough_oracle_cells(h, cols["pass"], cols["i"], cols["j"], cols["key"],
                               cols["votes"], cols["member_off"])
        cells = np.zeros(n, dtype=CELL_DTYPE)
        for k in CELL_DTYPE.names:
            cells[k] = cols[k]
        return cells, keep[:n].astype(bool), plotted[:E].astype(bool)
    finally:
        lib.hough_oracle_free(h)
