"""Write the full-size oracle fixtures for the two largest workloads.

Calls only ``oracle/`` and the seeded generator ``synth/``; run from the
repo root: ``python tests/golden/make_full_golden.py [seg4096|batch512|all]``
(about a minute of work per workload on 8 cores).  The fixtures hold, per
pass, the exact per-level statistics, the number of detected cells, a
sha256 over the cells' (i, j, key, votes) in key order, and the voter
checksum of ``oracle.member_digest`` over the pass's voter list (cells in
key order, voters ascending), so a GPU result can be compared in full
without storing gigabytes of voters.

* ``seg4096_seed0.json``: the 4096x4096 image (seed 0, T = 300, depth 12).
  The search is split into the subtrees of level ``SPLIT_LEVEL``, each run
  by ``oracle.detect_subtree`` with its parent's voters (``oracle.
  region_voters``) as candidates, in a process pool.  The statistics of the
  levels above come from ``region_voters`` of every region there.  That the
  subtrees of a level rebuild the whole search is itself pinned by
  ``tests/test_oracle_parts.py``.
* ``batch512_seed0.json``: every image of the 512-image batch (seed 0),
  each run whole by ``oracle.detect`` in a process pool.
"""
import hashlib
import json
import multiprocessing as mp
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle  # noqa: E402
import synth  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
SPLIT_LEVEL = 4
MASK64 = (1 << 64) - 1


def cells_sha256(i, j, key, votes) -> str:
    """sha256 over the little-endian int64 columns i, j, key, votes."""
    h = hashlib.sha256()
    for a in (i, j, key, votes):
        h.update(np.ascontiguousarray(np.asarray(a, dtype="<i8")).tobytes())
    return h.hexdigest()


def voter_sums(ids: np.ndarray):
    """(sum over t of (t A + B)(id + 1), sum of (id + 1)), both mod 2^64:
    the checksum of a voter list and what shifting its positions needs."""
    return oracle.member_digest(ids), int(np.asarray(ids, dtype=np.uint64).sum(dtype=np.uint64) + np.uint64(ids.size)) & MASK64


def key_of(i: int, j: int, level: int) -> int:
    """Quad-digit key (NE=0, NW=1, SW=2, SE=3 from level 1 down)."""
    k = 0
    for b in range(level - 1, -1, -1):
        e, n = (i >> b) & 1, (j >> b) & 1
        k = k * 4 + {(1, 1): 0, (0, 1): 1, (0, 0): 2, (1, 0): 3}[(e, n)]
    return k


_G = {}


def _init_seg(x, y, W, H, T, D, k):
    _G.update(x=x, y=y, W=W, H=H, T=T, D=D, k=k)


def _subtree(task):
    p, i, j, key, cand = task
    g = _G
    r = oracle.detect_subtree(g["x"], g["y"], g["W"], g["H"], g["T"], g["D"], p, g["k"], i, j, key,
                              cand, keep_members=True)
    c = r.cells
    ids = r.members
    s1, s0 = voter_sums(ids)
    return (p, key, r.stats[p], np.array(c["i"]), np.array(c["j"]), np.array(c["key"]), np.array(c["votes"]),
            int(ids.size), s1, s0)


def split_search(x, y, W, H, T, D, k=SPLIT_LEVEL, workers=8):
    """Per-pass summary ({"stats", "n_cells", "cells_sha256", "n_members",
    "member_digest"}) of the search over (x, y), computed as the subtrees of
    level k (k < D) in a process pool plus the levels above them."""
    assert 0 < k < D
    tasks = []
    top = {}
    E = len(x)
    for p in (0, 1):
        # levels 0 .. k-1 from the direct voters of every region there: a
        # region is evaluated iff its parent split (had more than T voters)
        st = np.zeros((D + 1, 6), dtype=np.int64)
        st[0] = [1, E, 0, 0, E, 0]
        if E > T:
            st[0][2], st[0][5] = 1, E
        level = {(0, 0): np.arange(E, dtype=np.int32)}
        for lev in range(1, k + 1):
            kids = {}
            for (i, j), v in sorted(level.items()):
                if len(v) <= T:
                    continue
                for e in (0, 1):
                    for n in (0, 1):
                        kids[(2 * i + e, 2 * j + n)] = v
            if lev == k:
                for (i, j), parent in sorted(kids.items()):
                    tasks.append((p, i, j, key_of(i, j, k), parent))
                break
            level = {c: oracle.region_voters(x, y, W, H, p, lev, c[0], c[1]) for c in kids}
            votes = [len(v) for v in level.values()]
            st[lev] = [len(level), sum(votes), sum(1 for n in votes if n > T), 0, 4 * st[lev - 1][5],
                       sum(n for n in votes if n > T)]
        top[p] = st
    with mp.Pool(workers, initializer=_init_seg, initargs=(x, y, W, H, T, D, k)) as pool:
        res = pool.map(_subtree, tasks, chunksize=1)
    out = {}
    for p in (0, 1):
        mine = sorted([r for r in res if r[0] == p], key=lambda r: r[1])
        st = top[p].copy()
        for r in mine:
            st[k:] += r[2][k:]
        cols = [np.concatenate([r[c] for r in mine]) if mine else np.zeros(0, np.int64) for c in (3, 4, 5, 6)]
        digest, t = 0, 0
        for r in mine:
            digest = (digest + r[8] + (t * oracle.DIGEST_A % (1 << 64)) * r[9]) & MASK64
            t += r[7]
        assert np.all(np.diff(cols[2]) > 0)
        out[str(p)] = {"stats": st.tolist(), "n_cells": int(len(cols[0])), "cells_sha256": cells_sha256(*cols),
                       "n_members": int(t), "member_digest": digest}
    return out


def summary(r, p):
    """The same per-pass summary from a whole ``oracle.detect`` result
    (``keep_members="digest"``)."""
    c = r.pass_cells(p)
    return {"stats": r.stats[p].tolist(), "n_cells": int(len(c)),
            "cells_sha256": cells_sha256(c["i"], c["j"], c["key"], c["votes"]),
            "n_members": int(r.pass_members[p]), "member_digest": int(r.member_digest[p])}


def seg4096(seed=0, workers=8):
    w = synth.workload("seg4096", seed)
    x, y = oracle.edge_points(w.image)
    W, H, T, D = w.width, w.height, w.threshold, w.max_depth
    t0 = time.time()
    passes = split_search(x, y, W, H, T, D, SPLIT_LEVEL, workers)
    print(f"seg4096: {time.time() - t0:.1f} s", flush=True)
    out = {"what": f"oracle output for seg4096 seed {seed} (4096x4096, 128 segments 2-3 px thick, 1% noise), "
                   f"T={T}, depth {D}, code variant, both passes; the search split at level {SPLIT_LEVEL}",
           "E": int(len(x)), "T": T, "depth": D, "stats_columns": list(oracle.STAT_NAMES), "passes": passes}
    path = os.path.join(HERE, f"seg4096_seed{seed}.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print(path, flush=True)


def _image(task):
    k, seed = task
    ws = _G.get("batch")
    if ws is None:
        ws = _G["batch"] = synth.batch_images(seed=seed, n=512)
    w = ws[k]
    x, y = oracle.edge_points(w.image)
    r = oracle.detect(x, y, w.width, w.height, w.threshold, w.max_depth, keep_members="digest")
    per = {str(p): summary(r, p) for p in (0, 1)}
    return k, {"W": w.width, "H": w.height, "T": w.threshold, "E": int(len(x)), "passes": per}


def batch512(seed=0, workers=8):
    t0 = time.time()
    with mp.Pool(workers) as pool:
        # largest images first, so the pool's tail is short
        ws = synth.batch_images(seed=seed, n=512)
        order = sorted(range(512), key=lambda k: -int(np.count_nonzero(ws[k].image)) * max(ws[k].width, ws[k].height))
        res = pool.map(_image, [(k, seed) for k in order], chunksize=1)
    print(f"batch512: {len(res)} images in {time.time() - t0:.1f} s", flush=True)
    images = [None] * 512
    for k, v in res:
        images[k] = v
    out = {"what": f"oracle output for every image of the 512-image batch, seed {seed} (sides log-uniform "
                   "128..2048, Poisson(24) segments, noise U[0.5%,3%], T=floor(side/10), depth ceil(log2 side)), "
                   "code variant, both passes",
           "stats_columns": list(oracle.STAT_NAMES), "images": images}
    path = os.path.join(HERE, f"batch512_seed{seed}.json")
    with open(path, "w") as f:
        json.dump(out, f, separators=(",", ":"))
    print(path, flush=True)


if __name__ == "__main__":
    which = sys.argv[1] if len(sys.argv) > 1 else "all"
    if which in ("seg4096", "all"):
        seg4096()
    if which in ("batch512", "all"):
        batch512()
