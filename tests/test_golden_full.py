"""The full-size fixture writer (``tests/golden/make_full_golden.py``):
its split search (subtrees of one level in a process pool, the levels above
from direct voters, the voter checksums shifted and summed) gives the same
summary as one whole ``oracle.detect`` run, and the fixtures it wrote are
well formed."""
import json
import os

import numpy as np
import pytest

import make_full_golden as mfg

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.mark.parametrize("seed,W,H,T,k", [(3, 64, 64, 6, 2), (4, 96, 50, 8, 3), (5, 128, 128, 12, 1)])
def test_split_search_equals_whole_search(orc, seed, W, H, T, k):
    rng = np.random.default_rng(seed)
    ys, xs = np.nonzero(rng.random((H, W)) < 0.05)
    x, y = xs.astype(np.int32), ys.astype(np.int32)
    D = orc.default_depth(W, H)
    whole = orc.detect(x, y, W, H, T, D, keep_members="digest")
    split = mfg.split_search(x, y, W, H, T, D, k, workers=2)
    for p in (0, 1):
        assert split[str(p)] == mfg.summary(whole, p)


def test_voter_sums_shift():
    rng = np.random.default_rng(0)
    a = rng.integers(0, 1 << 20, 1000).astype(np.int32)
    b = rng.integers(0, 1 << 20, 700).astype(np.int32)
    s1a, _ = mfg.voter_sums(a)
    s1b, s0b = mfg.voter_sums(b)
    whole, _ = mfg.voter_sums(np.concatenate([a, b]))
    import oracle
    assert whole == (s1a + s1b + (a.size * oracle.DIGEST_A % (1 << 64)) * s0b) % (1 << 64)


@pytest.mark.parametrize("name", ["seg4096_seed0.json", "batch512_seed0.json"])
def test_full_fixtures_well_formed(name):
    path = os.path.join(HERE, "golden", name)
    if not os.path.exists(path):
        pytest.skip(f"{name} not written")
    g = json.load(open(path))
    passes = [g["passes"]] if "passes" in g else [im["passes"] for im in g["images"]]
    for pp in passes:
        for p in ("0", "1"):
            s = np.array(pp[p]["stats"], dtype=np.int64)
            assert s[-1][3] == pp[p]["n_cells"]
            # evaluated regions at l+1 are the children of the regions split at l
            np.testing.assert_array_equal(s[1:, 0], 4 * s[:-1, 2])
            np.testing.assert_array_equal(s[1:, 4], 4 * s[:-1, 5])
