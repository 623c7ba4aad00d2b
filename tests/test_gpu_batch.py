"""GPU parity of the batched call (hough_hier_detect_batch): every image of a
batch against the CPU oracle, and against the single-image call, including
the device-side views (cells, voter ids, voter entries) of each result."""
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


class _DevView:
    """A device byte range as a torch tensor (no copy)."""

    def __init__(self, ptr, nbytes):
        self.__cuda_array_interface__ = {"shape": (int(nbytes),), "typestr": "|u1",
                                         "data": (int(ptr), False), "version": 2}


def dev_array(ptr, count, dtype):
    import torch
    dtype = np.dtype(dtype)
    if count == 0:
        return np.zeros(0, dtype)
    t = torch.as_tensor(_DevView(ptr, count * dtype.itemsize), device="cuda")
    return t.cpu().numpy().view(dtype).copy()


def host_view(r):
    return {p: (r.cells(p), r.stats_array(p)) for p in (0, 1)} | {"members": r.members()}


def check_against_oracle(got, ref, passes=3):
    for p in (0, 1):
        cells, stats = got[p]
        if not passes & (1 << p):
            assert len(cells) == 0
            continue
        want = ref.pass_cells(p)
        assert len(cells) == len(want), (p, len(cells), len(want))
        for f in ("i", "j", "key", "votes"):
            np.testing.assert_array_equal(cells[f], want[f], err_msg=f"pass {p} field {f}")
        np.testing.assert_array_equal(stats, ref.stats[p], err_msg=f"pass {p} stats")
        gm = got["members"]
        for c in range(len(cells)):
            a = gm[cells["member_off"][c]: cells["member_off"][c] + cells["votes"][c]]
            o = want["member_off"][c]
            if not np.array_equal(a, ref.members[o: o + want["votes"][c]]):
                raise AssertionError(f"pass {p} cell {c} members differ")


def check_device_views(hh, r):
    """Device cells index the device voter ids and entries of the same result."""
    ids_ptr, slots = r.device_members()
    ids = dev_array(ids_ptr, slots, np.int32)
    ent_ptr, n_ent, eb = r.member_points()
    assert n_ent == slots
    ent = dev_array(ent_ptr, n_ent, np.uint32 if eb == 4 else np.uint64)
    host_m = r.members()
    for p in (0, 1):
        ptr, n = r.device_cells(p)
        dc = dev_array(ptr, n, hh.CELL_DTYPE)
        hc = r.cells(p)
        for f in ("i", "j", "key", "votes", "pass"):
            np.testing.assert_array_equal(dc[f], hc[f])
        for c in range(n):
            o, v = int(dc["member_off"][c]), int(dc["votes"][c])
            assert 0 <= o and o + v <= slots
            want = host_m[hc["member_off"][c]: hc["member_off"][c] + v]
            np.testing.assert_array_equal(ids[o: o + v], want)
            if eb == 8:
                np.testing.assert_array_equal((ent[o: o + v] >> np.uint64(32)).astype(np.int32), want)


def test_batch_mixed_images_vs_oracle(hh):
    ws = synth.batch_images(seed=11, n=24, side_lo=64, side_hi=512)
    say(f"case batch of {len(ws)} images 64..512, host images")
    with hh.HoughHier(threshold=0) as ctx:
        rs = ctx.detect_batch([dict(image=w.image, width=w.width, height=w.height,
                                    threshold=w.threshold, max_depth=w.max_depth) for w in ws])
        for k, (w, r) in enumerate(zip(ws, rs)):
            x, y = oracle.edge_points(w.image)
            ref = oracle.detect(x, y, w.width, w.height, w.threshold, w.max_depth)
            assert r.info["n_points"] == len(x)
            check_against_oracle(host_view(r), ref)
            if k % 6 == 0:
                check_device_views(hh, r)
        for r in rs:
            r.free()


def test_batch_equals_single_calls(hh):
    import torch
    ws = synth.batch_images(seed=12, n=10, side_lo=32, side_hi=300)
    # degenerate members of a batch: an empty image, a depth-0 input, a
    # threshold above every vote, an image deeper than its side
    ws[1].image[:] = 0
    ws[3].max_depth = -1
    ws[5].threshold = 10 ** 6
    ws[7].max_depth = 11
    say("case batch == single calls (device images, degenerate members)")
    dev = [torch.from_numpy(w.image).cuda() for w in ws]
    with hh.HoughHier(threshold=0) as ctx:
        rs = ctx.detect_batch([dict(image=d, width=w.width, height=w.height, threshold=w.threshold,
                                    max_depth=w.max_depth) for d, w in zip(dev, ws)])
        for k, (d, w) in enumerate(zip(dev, ws)):
            one = ctx.detect(image=d, width=w.width, height=w.height, threshold=w.threshold,
                             max_depth=w.max_depth)
            a, b = host_view(rs[k]), host_view(one)
            for p in (0, 1):
                np.testing.assert_array_equal(a[p][0], b[p][0], err_msg=f"image {k} pass {p} cells")
                np.testing.assert_array_equal(a[p][1], b[p][1], err_msg=f"image {k} pass {p} stats")
            np.testing.assert_array_equal(a["members"], b["members"], err_msg=f"image {k} members")
            check_device_views(hh, rs[k])
            one.free()
        # results are independent handles: freeing some leaves the rest intact
        for r in rs[::2]:
            r.free()
        x, y = oracle.edge_points(ws[9].image)
        check_against_oracle(host_view(rs[9]), oracle.detect(x, y, ws[9].width, ws[9].height,
                                                             ws[9].threshold, ws[9].max_depth))
        for r in rs[1::2]:
            r.free()


@pytest.mark.parametrize("variant", ["code", "circle"])
def test_batch_point_lists(hh, variant):
    import torch
    rng = np.random.default_rng(21)
    cases = []
    for k in range(9):
        W, H = int(rng.integers(1, 400)), int(rng.integers(1, 400))
        n = int(rng.integers(0, 3000)) if k != 4 else 0
        x = rng.integers(0, W, n).astype(np.int32)
        y = rng.integers(0, H, n).astype(np.int32)
        T = int(rng.integers(0, 40))
        cases.append((W, H, x, y, T))
    say(f"case batch of point lists ({variant}), host and device lists mixed")
    inputs = []
    for k, (W, H, x, y, T) in enumerate(cases):
        if k % 2:
            inputs.append(dict(x=torch.from_numpy(x).cuda(), y=torch.from_numpy(y).cuda(), width=W,
                               height=H, threshold=T))
        else:
            inputs.append(dict(x=x, y=y, width=W, height=H, threshold=T))
    with hh.HoughHier(threshold=0, variant=variant) as ctx:
        rs = ctx.detect_batch(inputs)
        for k, ((W, H, x, y, T), r) in enumerate(zip(cases, rs)):
            ref = oracle.detect(x, y, W, H, T, 0, variant)
            check_against_oracle(host_view(r), ref)
            check_device_views(hh, r)
            r.free()


def test_batch_one_pass_and_membership_off(hh):
    ws = synth.batch_images(seed=13, n=6, side_lo=64, side_hi=256)
    say("case batch, pass 1 only, membership off")
    with hh.HoughHier(threshold=0, passes=2, membership=False) as ctx:
        rs = ctx.detect_batch([dict(image=w.image, width=w.width, height=w.height,
                                    threshold=w.threshold) for w in ws])
        for w, r in zip(ws, rs):
            x, y = oracle.edge_points(w.image)
            ref = oracle.detect(x, y, w.width, w.height, w.threshold, 0, "code", 2, False)
            assert len(r.cells(0)) == 0
            c = r.cells(1)
            want = ref.pass_cells(1)
            for f in ("i", "j", "key", "votes"):
                np.testing.assert_array_equal(c[f], want[f])
            assert np.all(c["member_off"] == -1)
            np.testing.assert_array_equal(r.stats_array(1), ref.stats[1])
            r.free()


def test_batch_invalid(hh):
    say("case batch argument errors")
    with hh.HoughHier(threshold=1) as ctx:
        img = np.zeros((8, 8), np.uint8)
        with pytest.raises(hh.HHError) as e:
            ctx.detect_batch([dict(image=img, width=8, height=8),
                              dict(x=np.zeros(1, np.int32), y=np.zeros(1, np.int32), width=8, height=8)])
        assert e.value.status == -1
        with pytest.raises(hh.HHError) as e:
            ctx.detect_batch([dict(image=img, width=8, height=8)] * 1025)
        assert e.value.status == -3
        with pytest.raises(hh.HHError) as e:
            ctx.detect_batch([dict(x=np.array([3], np.int32), y=np.array([9], np.int32), width=8,
                                   height=8)])
        assert e.value.status == -1
        r = ctx.detect_batch([dict(image=img, width=8, height=8)])[0]
        assert r.info["n_points"] == 0
        r.free()


@pytest.mark.parametrize("membership", [True, False])
def test_levels_outgrowing_the_arena(hh, membership):
    """A context whose arena starts far too small: the call resumes at each
    level that does not fit (and reruns a root setup that does not), with
    results identical to the oracle; a second call starts at the grown
    sizes."""
    ws = synth.batch_images(seed=14, n=8, side_lo=64, side_hi=384)
    say(f"case tiny arena, batch of 8 and single calls, membership {membership}")
    with hh.HoughHier(threshold=0, arena_hint=4096, membership=membership) as ctx:
        for rep in range(2):
            rs = ctx.detect_batch([dict(image=w.image, width=w.width, height=w.height,
                                        threshold=w.threshold) for w in ws])
            for w, r in zip(ws, rs):
                x, y = oracle.edge_points(w.image)
                ref = oracle.detect(x, y, w.width, w.height, w.threshold, 0, "code", 3, membership)
                if membership:
                    check_against_oracle(host_view(r), ref)
                else:
                    for p in (0, 1):
                        c = r.cells(p)
                        want = ref.pass_cells(p)
                        for f in ("i", "j", "key", "votes"):
                            np.testing.assert_array_equal(c[f], want[f])
                        np.testing.assert_array_equal(r.stats_array(p), ref.stats[p])
                r.free()
    with hh.HoughHier(threshold=40, max_depth=8, arena_hint=4096) as ctx:
        w = synth.workload("line256", 2)
        r = ctx.detect(image=w.image, width=w.width, height=w.height)
        x, y = oracle.edge_points(w.image)
        check_against_oracle(host_view(r), oracle.detect(x, y, w.width, w.height, 40, 8))
        r.free()


@pytest.mark.parametrize("steps", [2, 16, 64])
def test_long_tasks_without_room(hh, steps):
    """Long tasks in a context whose arena starts tiny: each level's lists get
    little more room than they need, so the last tasks of a level have no
    room for all their entries and run checked, chunk after chunk, through
    tasks of several chunks; results equal the oracle's for every task
    size."""
    w = synth.workload("line256", 2)
    x, y = oracle.edge_points(w.image)
    ref = oracle.detect(x, y, w.width, w.height, 40, 8)
    say(f"case line256 seed 2, tiny arena, {steps} steps per task")
    with hh.HoughHier(threshold=40, max_depth=8, arena_hint=4096) as ctx:
        ctx.set_launch(steps, 0, 0)
        for rep in range(2):
            r = ctx.detect(image=w.image, width=w.width, height=w.height)
            check_against_oracle(host_view(r), ref)
            r.free()


def test_batch_in_groups_under_a_memory_limit(hh):
    """An arena limit far below what the whole batch needs: the call runs in
    groups of images (the limit is learnt for the next call), every result
    equals the oracle, and one image that alone exceeds the limit fails
    cleanly."""
    ws = synth.batch_images(seed=15, n=16, side_lo=64, side_hi=512)
    say("case batch in groups, 400 MiB arena limit")
    with hh.HoughHier(threshold=0, arena_hint=1 << 16, arena_limit_mib=400) as ctx:
        for rep in range(2):
            rs = ctx.detect_batch([dict(image=w.image, width=w.width, height=w.height,
                                        threshold=w.threshold) for w in ws])
            t = rs[0].timing()
            say(f"  rep {rep}: groups {t['groups']}, resumes {t['resumes']}")
            assert t["groups"] > 1
            for k, (w, r) in enumerate(zip(ws, rs)):
                x, y = oracle.edge_points(w.image)
                check_against_oracle(host_view(r), oracle.detect(x, y, w.width, w.height, w.threshold, 0))
                if k % 5 == 0:
                    check_device_views(hh, r)
            for r in rs:
                r.free()
    with hh.HoughHier(threshold=40, max_depth=8, arena_limit_mib=1) as ctx:
        w = synth.workload("line256", 4)
        with pytest.raises(hh.HHError) as e:
            ctx.detect(image=w.image, width=w.width, height=w.height)
        assert e.value.status == -3
        # the context stays usable
        small = np.zeros((16, 16), np.uint8)
        small[3, :] = 1
        ctx.detect(image=small, width=16, height=16, threshold=2).free()


def test_batch512_full_size_sampled(hh):
    """The 512-image batch at full size in the launch configuration the
    benchmark times: six sampled images (the smallest, the largest and four
    drawn by seed) against the oracle, and for every image the properties
    that hold at any size (edge count, root statistics, sorted keys, votes
    above the threshold, per-level consistency of the statistics)."""
    import torch
    ws = synth.batch_images(seed=0, n=512)
    px = np.array([w.width * w.height for w in ws])
    rng = np.random.default_rng(99)
    pick = sorted(set([int(np.argmin(px)), int(np.argmax(px))] + rng.choice(512, 4, replace=False).tolist()))
    say(f"case batch of 512 at full size, sampled images {pick}")
    imgs = [torch.from_numpy(w.image).cuda() for w in ws]
    with hh.HoughHier(threshold=0) as ctx:
        rs = ctx.detect_batch([dict(image=d, width=w.width, height=w.height, threshold=w.threshold)
                               for d, w in zip(imgs, ws)])
        say(f"  groups {rs[0].timing()['groups']}")
        for k, (w, r) in enumerate(zip(ws, rs)):
            E = int(np.count_nonzero(w.image))
            assert r.info["n_points"] == E
            for p in (0, 1):
                st = r.stats(p)
                assert st["evaluated"][0] == 1 and st["votes"][0] == E
                c = r.cells(p)
                assert np.all(np.diff(c["key"]) > 0)
                assert np.all(c["votes"] > w.threshold)
                assert len(c) == st["detected"][-1]
                # a level's evaluated regions are four per region split above it
                np.testing.assert_array_equal(st["evaluated"][1:], 4 * st["split"][:-1])
        for k in pick:
            w = ws[k]
            x, y = oracle.edge_points(w.image)
            say(f"  oracle image {k} ({w.width}x{w.height}, {len(x)} points)")
            check_against_oracle(host_view(rs[k]), oracle.detect(x, y, w.width, w.height, w.threshold, 0))
        for r in rs:
            r.free()
