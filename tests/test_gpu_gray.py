"""GPU parity of the Sobel front end (gray images, kind 2): the edge points,
their ALPHA/BETA sets and the hierarchical vote of each set against the
oracle (Sobel partition, then the vote of pass 0 on ALPHA and pass 1 on
BETA), bit-exact, with point ids as ranks among all edge points."""
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


def gray_image(seed, W, H, n_seg=12):
    """Bright segments on a darker, noisy background."""
    rng = np.random.default_rng(seed)
    lines = synth.segment_image(rng, W, H, n_seg, 0.2 * min(W, H), 0.9 * min(W, H), 0.0)
    g = rng.integers(0, 40, (H, W)) + lines.astype(np.int64) * 170
    return g.astype(np.uint8)


def reference(g, et, T, dmax=0, variant="code", passes=3):
    H, W = g.shape
    x, y, beta = oracle.sobel_partition(g, et)
    out = {"E": len(x)}
    for p, sel in ((0, ~beta), (1, beta)):
        if not passes & (1 << p):
            continue
        ids = np.nonzero(sel)[0]
        r = oracle.detect(x[ids], y[ids], W, H, T, dmax, variant, 1 << p)
        cells = r.pass_cells(p)
        mem = [ids[r.members[o: o + v]] for o, v in zip(cells["member_off"], cells["votes"])]
        out[p] = (cells, r.stats[p], mem)
    return out


def check(r, ref, passes=3):
    assert r.info["n_points"] == ref["E"]
    members = r.members()
    for p in (0, 1):
        cells = r.cells(p)
        if not passes & (1 << p):
            assert len(cells) == 0
            continue
        want, stats, mem = ref[p]
        assert len(cells) == len(want), (p, len(cells), len(want))
        for f in ("i", "j", "key", "votes"):
            np.testing.assert_array_equal(cells[f], want[f], err_msg=f"pass {p} {f}")
        np.testing.assert_array_equal(r.stats_array(p), stats, err_msg=f"pass {p} stats")
        for c in range(len(cells)):
            got = members[cells["member_off"][c]: cells["member_off"][c] + cells["votes"][c]]
            np.testing.assert_array_equal(got, mem[c], err_msg=f"pass {p} cell {c}")


@pytest.mark.parametrize("case", [(0, 64, 48, 120, 8), (1, 200, 150, 200, 20), (2, 511, 300, 150, 30),
                                  (3, 257, 333, 250, 25)])
@pytest.mark.parametrize("variant", ["code", "circle"])
def test_gray_vs_oracle(hh, case, variant):
    seed, W, H, et, T = case
    say(f"case gray seed {seed} {W}x{H} edge {et} T {T} {variant}")
    g = gray_image(seed, W, H)
    ref = reference(g, et, T, 0, variant)
    with hh.HoughHier(threshold=T, variant=variant) as ctx:
        r = ctx.detect(gray=g, edge_threshold=et, width=W, height=H)
        check(r, ref)
        r.free()


def test_gray_input_forms_batch_and_serving(hh):
    import torch
    say("case gray: host / device / strided device, one pass, batch, served")
    g = gray_image(7, 300, 220)
    ref = reference(g, 180, 24)
    dev = torch.from_numpy(g).cuda()
    padded = torch.zeros((220, 300 + 20), dtype=torch.uint8, device="cuda")
    padded[:, :300] = dev
    torch.cuda.synchronize()
    with hh.HoughHier(threshold=24) as ctx:
        for img in (g, dev, padded[:, :300]):
            r = ctx.detect(gray=img, edge_threshold=180, width=300, height=220)
            check(r, ref)
            r.free()
        imgs = [gray_image(20 + k, 90 + 37 * k, 160 - 11 * k) for k in range(6)]
        rs = ctx.detect_batch([dict(gray=im, edge_threshold=150, width=im.shape[1], height=im.shape[0])
                               for im in imgs])
        for im, r in zip(imgs, rs):
            check(r, reference(im, 150, 24))
            r.free()
        ctx.serve_start(lanes=2, max_batch=4)
        ts = [ctx.submit(gray=im, edge_threshold=150, width=im.shape[1], height=im.shape[0]) for im in imgs]
        for im, t in zip(imgs, ts):
            r = ctx.poll(t)
            check(r, reference(im, 150, 24))
            r.free()
    with hh.HoughHier(threshold=24, passes=2) as ctx:
        r = ctx.detect(gray=g, edge_threshold=180, width=300, height=220)
        check(r, reference(g, 180, 24, passes=2), passes=2)
        r.free()


def test_gray_edge_cases(hh):
    say("case gray edge cases: no edges, tiny images, depth 0, bad threshold")
    with hh.HoughHier(threshold=1) as ctx:
        for shape in ((2, 2), (1, 9), (3, 3), (40, 40)):
            g = np.full(shape, 77, np.uint8)
            r = ctx.detect(gray=g, edge_threshold=0, width=shape[1], height=shape[0])
            assert r.info["n_points"] == 0 and len(r.cells(0)) == 0 and len(r.cells(1)) == 0
            r.free()
        g = gray_image(3, 33, 31)
        r = ctx.detect(gray=g, edge_threshold=0, width=33, height=31)   # every gradient above 0
        check(r, reference(g, 0, 1))
        r.free()
        with pytest.raises(hh.HHError) as e:
            ctx.detect(gray=g, edge_threshold=0, width=33, height=31, max_depth=-1)
        assert e.value.status == -1
        with pytest.raises(hh.HHError) as e:
            ctx.detect(gray=g, edge_threshold=-5, width=33, height=31)
        assert e.value.status == -1
