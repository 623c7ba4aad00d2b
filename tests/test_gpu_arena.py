"""A caller-owned arena (hh_config.arena): every device buffer of a
detection call is carved from a torch tensor's memory.  Results match the
oracle; an arena too small for the call fails with HH_ECAPACITY; a second
call while results of the first still live in the arena fails with HH_EBUSY;
a batch in the arena equals plain calls."""
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


def check(r, ref):
    members = r.members()
    for p in (0, 1):
        got, want = r.cells(p), ref.pass_cells(p)
        assert len(got) == len(want), (p, len(got), len(want))
        for f in ("i", "j", "key", "votes"):
            np.testing.assert_array_equal(got[f], want[f], err_msg=f"pass {p} {f}")
        np.testing.assert_array_equal(r.stats_array(p), ref.stats[p])
        for c in range(len(got)):
            a = members[got["member_off"][c]: got["member_off"][c] + got["votes"][c]]
            np.testing.assert_array_equal(a, ref.members[want["member_off"][c]: want["member_off"][c] + want["votes"][c]])


def test_seg1024_in_a_torch_arena(hh):
    import torch
    w = synth.workload("seg1024", 0)
    say("case seg1024 in a 2 GiB torch arena")
    arena = torch.empty(2 << 30, dtype=torch.uint8, device="cuda")
    img = torch.from_numpy(w.image).cuda()
    x, y = oracle.edge_points(w.image)
    ref = oracle.detect(x, y, w.width, w.height, w.threshold, w.max_depth)
    with hh.HoughHier(threshold=w.threshold, max_depth=w.max_depth, arena=arena) as ctx:
        for rep in range(2):
            r = ctx.detect(image=img, width=w.width, height=w.height)
            check(r, ref)
            if rep == 0:
                with pytest.raises(hh.HHError) as e:   # the first result still lives in the arena
                    ctx.detect(image=img, width=w.width, height=w.height)
                assert e.value.status == -5
            r.free()


def test_too_small_arena(hh):
    import torch
    w = synth.workload("seg1024", 0)
    say("case seg1024 in a 16 MiB arena")
    arena = torch.empty(16 << 20, dtype=torch.uint8, device="cuda")
    img = torch.from_numpy(w.image).cuda()
    with hh.HoughHier(threshold=w.threshold, max_depth=w.max_depth, arena=arena) as ctx:
        with pytest.raises(hh.HHError) as e:
            ctx.detect(image=img, width=w.width, height=w.height)
        assert e.value.status == -3
        # a small input still runs in it
        small = synth.full_span_image(1, 128, 128, 6, 0.01)
        x, y = oracle.edge_points(small)
        r = ctx.detect(image=small, width=128, height=128, threshold=20, max_depth=0)
        check(r, oracle.detect(x, y, 128, 128, 20, 0))
        r.free()


def test_batch_in_arena_equals_plain(hh):
    import torch
    ws = synth.batch_images(seed=3, n=12, side_hi=512)
    say("case 12-image batch in a 1 GiB arena")
    arena = torch.empty(1 << 30, dtype=torch.uint8, device="cuda")
    inputs = [dict(image=torch.from_numpy(w.image).cuda(), width=w.width, height=w.height, threshold=w.threshold)
              for w in ws]
    with hh.HoughHier(threshold=0, arena=arena) as ctx, hh.HoughHier(threshold=0) as plain:
        rs = ctx.detect_batch(inputs)
        for inp, r in zip(inputs, rs):
            q = plain.detect(**inp)
            for p in (0, 1):
                np.testing.assert_array_equal(r.cells(p), q.cells(p))
                np.testing.assert_array_equal(r.stats_array(p), q.stats_array(p))
            np.testing.assert_array_equal(r.members(), q.members())
            q.free()
        for r in rs:
            r.free()
