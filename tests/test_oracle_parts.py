"""The oracle's partial-search entry and its voter checksum.

* ``detect_subtree``: the regions of one level, each evaluated against the
  voters of its parent found by direct test (``region_voters``), together
  reproduce the whole search -- every cell (keys, votes, voters) and every
  statistic from that level down.  The union is taken over all regions of
  the level in key order, so a subtree that drops, adds or reorders work
  fails the comparison.
* ``keep_members="digest"``: the checksum equals the same sum computed from
  the stored voter list, and the cells and statistics are those of a run
  that stores the voters.
"""
import numpy as np
import pytest

import brute


def points(seed, W, H, p):
    rng = np.random.default_rng(seed)
    ys, xs = np.nonzero(rng.random((H, W)) < p)
    return xs.astype(np.int32), ys.astype(np.int32)


def regions_in_key_order(level):
    """(i, j, key) of every region of a level, sorted by key."""
    out = [(brute.key_of(i, j, level), i, j) for i in range(1 << level) for j in range(1 << level)]
    return [(i, j, k) for k, i, j in sorted(out)]


@pytest.mark.parametrize("seed,W,H,T,variant", [(1, 32, 32, 3, "code"), (2, 27, 19, 1, "code"),
                                                 (3, 32, 32, 4, "circle"), (4, 64, 40, 6, "code")])
def test_subtrees_of_a_level_rebuild_the_search(orc, seed, W, H, T, variant):
    x, y = points(seed, W, H, 0.08)
    full = orc.detect(x, y, W, H, T, 0, variant)
    D = full.dmax
    for p in (0, 1):
        want = full.pass_cells(p)
        for level in (1, 2):
            cells, members, st = [], [], np.zeros_like(full.stats[p])
            for i, j, key in regions_in_key_order(level):
                cand = orc.region_voters(x, y, W, H, p, level - 1, i // 2, j // 2, variant)
                if len(cand) <= T:   # the parent did not split: the search never comes here
                    continue
                r = orc.detect_subtree(x, y, W, H, T, 0, p, level, i, j, key, cand, variant, keep_members=True)
                assert r.dmax == D
                st += r.stats[p]
                for c in range(len(r.cells)):
                    cells.append(r.cells[c])
                    members.append(r.cell_members(c))
            got = np.array(cells, dtype=want.dtype) if cells else want[:0]
            for f in ("i", "j", "key", "votes"):
                np.testing.assert_array_equal(got[f], want[f])
            for c in range(len(want)):
                np.testing.assert_array_equal(members[c], full.cell_members(int(np.nonzero(
                    (full.cells["pass"] == p) & (full.cells["key"] == want["key"][c]))[0][0])))
            np.testing.assert_array_equal(st[level:], full.stats[p][level:])


def test_subtree_of_the_root_is_the_pass(orc):
    x, y = points(7, 48, 48, 0.06)
    full = orc.detect(x, y, 48, 48, 5, 0)
    for p in (0, 1):
        r = orc.detect_subtree(x, y, 48, 48, 5, 0, p, 0, 0, 0, 0, np.arange(len(x)), keep_members=True)
        np.testing.assert_array_equal(r.stats[p], full.stats[p])
        np.testing.assert_array_equal(r.cells["key"], full.pass_cells(p)["key"])
        np.testing.assert_array_equal(r.members, full.members[full.pass_cells(p)["member_off"][0]:][:len(r.members)])


def test_subtree_rejects_bad_regions(orc):
    x, y = points(8, 16, 16, 0.1)
    with pytest.raises(orc.OracleError):
        orc.detect_subtree(x, y, 16, 16, 2, 0, 0, 2, 4, 0, 0, np.arange(len(x)))
    with pytest.raises(orc.OracleError):
        orc.detect_subtree(x, y, 16, 16, 2, 0, 0, 1, 0, 0, 0, np.array([len(x)]))


@pytest.mark.parametrize("variant", ["code", "circle"])
def test_member_digest_matches_stored_voters(orc, variant):
    x, y = points(9, 64, 64, 0.05)
    full = orc.detect(x, y, 64, 64, 6, 0, variant)
    dig = orc.detect(x, y, 64, 64, 6, 0, variant, keep_members="digest")
    assert dig.members.size == 0 and (dig.cells["member_off"] == -1).all()
    for p in (0, 1):
        c = full.pass_cells(p)
        ids = np.concatenate([full.members[o:o + v] for o, v in zip(c["member_off"], c["votes"])])
        assert dig.pass_members[p] == ids.size == int(c["votes"].sum())
        assert dig.member_digest[p] == orc.member_digest(ids)
        np.testing.assert_array_equal(dig.stats[p], full.stats[p])
        for f in ("i", "j", "key", "votes"):
            np.testing.assert_array_equal(dig.pass_cells(p)[f], c[f])
    # the checksum sees order and values
    c = full.pass_cells(0)
    ids = np.concatenate([full.members[o:o + v] for o, v in zip(c["member_off"], c["votes"])])
    swapped = ids.copy()
    swapped[[0, 1]] = swapped[[1, 0]]
    assert orc.member_digest(swapped) != orc.member_digest(ids)
    bumped = ids.copy()
    bumped[-1] += 1
    assert orc.member_digest(bumped) != orc.member_digest(ids)
