"""hough_hier_detect_noalloc through the C ABI: the entry point for callers
that cannot allocate device memory (its scratch is a fixed array in the
library).  Two calls in a row, the second on a smaller input, each compared
with hough_hier_detect on the same input: the same cells (i, j, key, votes,
pass) in the same order, the same voter ids per cell, the same per-level
statistics.  Output buffers are the caller's torch tensors."""
import sys

import numpy as np
import pytest

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


def compare(hh, ctx, w, cells_buf, ids_buf):
    import torch
    img = torch.from_numpy(w.image).cuda()
    out = ctx.detect_noalloc(image=img, width=w.width, height=w.height, threshold=w.threshold,
                             max_depth=w.max_depth, cells_out=cells_buf, members_out=ids_buf)
    torch.cuda.synchronize()
    r = ctx.detect(image=img, width=w.width, height=w.height, threshold=w.threshold, max_depth=w.max_depth)
    ref_members = r.members()
    nc = out["n_cells"][0] + out["n_cells"][1]
    got_cells = cells_buf[: nc * hh.CELL_DTYPE.itemsize].cpu().numpy().view(hh.CELL_DTYPE)
    got_ids = ids_buf[: out["n_members"]].cpu().numpy()
    at = 0
    for p in (0, 1):
        want = r.cells(p)
        assert out["n_cells"][p] == len(want)
        got = got_cells[at: at + len(want)]
        at += len(want)
        for f in ("pass", "i", "j", "key", "votes"):
            np.testing.assert_array_equal(got[f], want[f], err_msg=f"pass {p} field {f}")
        for c in range(len(want)):
            o, v, wo = int(got["member_off"][c]), int(got["votes"][c]), int(want["member_off"][c])
            np.testing.assert_array_equal(got_ids[o: o + v], ref_members[wo: wo + v], err_msg=f"pass {p} cell {c}")
        st = r.stats_array(p)
        np.testing.assert_array_equal(out["stats"][p][: len(st)], st)
        assert not out["stats"][p][len(st):].any()
    assert out["n_members"] == len(ref_members)
    r.free()
    return nc


def test_noalloc_matches_detect_twice(hh):
    import torch
    cells_buf = torch.zeros(64 << 20, dtype=torch.uint8, device="cuda")   # 2M cells
    ids_buf = torch.zeros(16 << 20, dtype=torch.int32, device="cuda")
    with hh.HoughHier(threshold=0) as ctx:
        big = synth.workload("line256", 0)
        say("case noalloc: line256 seed 0, then a smaller 96x80 image")
        n1 = compare(hh, ctx, big, cells_buf, ids_buf)
        small_img = synth.full_span_image(5, 96, 80, 4, 0.02)
        small = synth.Workload("small", small_img, 12, 0, {})
        n2 = compare(hh, ctx, small, cells_buf, ids_buf)
        assert n1 > n2 > 0


def test_noalloc_capacity_errors(hh):
    import torch
    w = synth.workload("line256", 1)
    img = torch.from_numpy(w.image).cuda()
    with hh.HoughHier(threshold=w.threshold, max_depth=w.max_depth) as ctx:
        tiny = torch.zeros(32 * 4, dtype=torch.uint8, device="cuda")   # 4 cells
        ids = torch.zeros(1 << 20, dtype=torch.int32, device="cuda")
        with pytest.raises(hh.HHError) as e:
            ctx.detect_noalloc(image=img, width=w.width, height=w.height, cells_out=tiny, members_out=ids)
        assert e.value.status == -3
        # the scratch cannot hold a 4096x4096 image's level lists
        w4 = synth.workload("seg4096", 0)
        big = torch.zeros(32 << 20, dtype=torch.uint8, device="cuda")
        with pytest.raises(hh.HHError) as e:
            ctx.detect_noalloc(image=torch.from_numpy(w4.image).cuda(), width=w4.width, height=w4.height,
                               threshold=w4.threshold, max_depth=w4.max_depth, cells_out=big, members_out=ids)
        assert e.value.status == -3
        # and the context still works afterwards
        cells = torch.zeros(64 << 20, dtype=torch.uint8, device="cuda")
        out = ctx.detect_noalloc(image=img, width=w.width, height=w.height, cells_out=cells, members_out=ids)
        assert out["n_cells"][0] > 0
