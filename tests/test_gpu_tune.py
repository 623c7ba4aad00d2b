"""hough_hier_autotune: the launch shape is chosen by timing candidates on
the caller's call, written to the cache file, read back for the same
workload class, and the detection in the chosen shape equals the oracle."""
import json
import sys

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def hh():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1007_0547_amd as m
    return m


def test_autotune_cache_and_parity(hh, tmp_path, monkeypatch):
    import torch
    cache = tmp_path / "tune.json"
    monkeypatch.setenv("HH_TUNE_CACHE", str(cache))
    w = synth.workload("line256", 3)
    img = torch.from_numpy(w.image).cuda()
    inp = dict(image=img, width=w.width, height=w.height)
    say("case autotune line256")
    with hh.HoughHier(threshold=w.threshold, max_depth=w.max_depth) as ctx:
        first = ctx.autotune([inp])
        assert not first["from_cache"]
        assert first["task_steps"] in (1, 2, 4, 8, 16) and first["wg_per_cu"] in (0, 4)
        assert ctx.launch() == {k: first[k] for k in ("task_steps", "queue_batch", "wg_per_cu")}
        entries = json.loads(cache.read_text())
        assert len(entries) == 1
        (key, val), = entries.items()
        assert key.startswith("gfx950/") and val["task_steps"] == first["task_steps"] and val["ms"] > 0
        second = ctx.autotune([inp])
        assert second["from_cache"] and second["task_steps"] == first["task_steps"]
        r = ctx.detect(**inp)
        x, y = oracle.edge_points(w.image)
        ref = oracle.detect(x, y, w.width, w.height, w.threshold, w.max_depth)
        for p in (0, 1):
            got, want = r.cells(p), ref.pass_cells(p)
            for f in ("i", "j", "key", "votes"):
                np.testing.assert_array_equal(got[f], want[f])
            np.testing.assert_array_equal(r.stats_array(p), ref.stats[p])
        r.free()


def test_every_launch_shape_gives_the_same_result(hh):
    """Results do not depend on the launch shape: each task size, the work
    queue and a reduced grid against the oracle on one image."""
    import torch
    w = synth.workload("seg1024", 1)
    img = torch.from_numpy(w.image).cuda()
    x, y = oracle.edge_points(w.image)
    ref = oracle.detect(x, y, w.width, w.height, w.threshold, w.max_depth)
    with hh.HoughHier(threshold=w.threshold, max_depth=w.max_depth) as ctx:
        for shape in ((1, 0, 0), (3, 0, 0), (16, 0, 0), (64, 0, 0), (2, 256, 0), (4, 0, 1)):
            say(f"case seg1024 seed 1, launch shape {shape}")
            ctx.set_launch(*shape)
            r = ctx.detect(image=img, width=w.width, height=w.height)
            members = r.members()
            for p in (0, 1):
                got, want = r.cells(p), ref.pass_cells(p)
                for f in ("i", "j", "key", "votes"):
                    np.testing.assert_array_equal(got[f], want[f], err_msg=f"{shape} pass {p} {f}")
                np.testing.assert_array_equal(r.stats_array(p), ref.stats[p])
                for c in range(0, len(got), 97):
                    o, v, wo = int(got["member_off"][c]), int(got["votes"][c]), int(want["member_off"][c])
                    np.testing.assert_array_equal(members[o:o + v], ref.members[wo:wo + v])
            r.free()
