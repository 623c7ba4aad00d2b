"""GPU parity of solution() with point removal (hough_hier_solution) against
the oracle's walk over the detected cells in key order (itself pinned against
the depth-first search with removal): keep flags per cell, plotted flags per
point id and their counts, bit-exact, for every input kind, the LDS and the
device-memory bitmap, cells longer than a window, batched and served results."""
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


def expect(x, y, W, H, T, dmax=0, variant="code", passes=3):
    """Oracle keep and plotted flags per pass (pass -> (keep, plotted))."""
    out = {}
    for p in (0, 1):
        if passes & (1 << p):
            cells, keep, plotted = oracle.solution(x, y, W, H, T, dmax, p, variant)
            out[p] = (keep, plotted)
    return out


def check(r, want, E, what=""):
    for p in (0, 1):
        s = r.solution(p)
        if p not in want:
            assert s["kept"] == 0 and len(s["keep"]) == 0 and len(s["plotted"]) == 0
            continue
        keep, plotted = want[p]
        assert len(s["keep"]) == len(r.cells(p)) == len(keep), (what, p)
        np.testing.assert_array_equal(s["keep"], keep, err_msg=f"{what} pass {p} keep")
        np.testing.assert_array_equal(s["plotted"], plotted, err_msg=f"{what} pass {p} plotted")
        assert len(s["plotted"]) == E
        assert s["kept"] == int(keep.sum()) and s["plotted_points"] == int(plotted.sum()), (what, p)


def points(img):
    return oracle.edge_points(img)


def check_image(r, want, x, y, what=""):
    """The output image: 255 at the points plotted by any pass, else 0."""
    H, W = r.info["height"], r.info["width"]
    ref = np.zeros((H, W), np.uint8)
    for p, (_, plotted) in want.items():
        ref[np.asarray(y)[plotted], np.asarray(x)[plotted]] = 255
    np.testing.assert_array_equal(r.solution_image(), ref, err_msg=f"{what} image")


CASES = [
    # name, image maker, T, dmax, variant
    ("line256", lambda: synth.workload("line256", 0).image, 40, 0, "code"),
    ("fs64 T0", lambda: synth.full_span_image(0, 64, 64, 6, 0.05), 0, 0, "code"),
    ("fs64 T1", lambda: synth.full_span_image(1, 64, 64, 6, 0.05), 1, 0, "code"),
    ("fs64 T3", lambda: synth.full_span_image(2, 64, 64, 6, 0.05), 3, 0, "code"),
    ("fs100x80 circle", lambda: synth.full_span_image(5, 100, 80, 5, 0.03), 10, 0, "circle"),
    ("fs200x150 depth 5", lambda: synth.full_span_image(6, 200, 150, 8, 0.02), 12, 5, "code"),
]


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_solution_images(hh, case):
    name, make, T, dmax, variant = case
    say(f"case solution {name} T {T} depth {dmax} {variant}")
    img = make()
    H, W = img.shape
    x, y = points(img)
    want = expect(x, y, W, H, T, dmax, variant)
    with hh.HoughHier(threshold=T, max_depth=dmax, variant=variant) as ctx:
        r = ctx.detect(image=img, width=W, height=H)
        ms = ctx.solution([r])
        assert ms > 0
        check(r, want, len(x), name)
        check_image(r, want, x, y, name)
        assert ctx.solution([r]) == 0.0   # solved results are skipped
        r.free()


def test_solution_point_lists(hh):
    """8-byte entries (ids carried), duplicate points (separate lines), and a
    row of 16000 points whose cells are longer than a window."""
    rng = np.random.default_rng(1)
    xd = np.repeat(rng.integers(0, 50, 200), 2).astype(np.int32)
    yd = np.repeat(rng.integers(0, 40, 200), 2).astype(np.int32)
    xs = np.concatenate([np.arange(16000), rng.integers(0, 16384, 400)]).astype(np.int32)
    ys = np.concatenate([np.full(16000, 5), rng.integers(0, 8, 400)]).astype(np.int32)
    for name, x, y, W, H, T in (("duplicates", xd, yd, 50, 40, 6), ("long cells", xs, ys, 16384, 8, 300)):
        say(f"case solution points {name}: E {len(x)} T {T}")
        want = expect(x, y, W, H, T)
        with hh.HoughHier(threshold=T) as ctx:
            r = ctx.detect(x, y, width=W, height=H)
            ctx.solution(r)
            check(r, want, len(x), name)
            check_image(r, want, x, y, name)
            r.free()


def test_solution_device_bitmap(hh):
    """More points than the LDS bitmap holds: the walk keeps the plotted set
    in device memory."""
    rng = np.random.default_rng(11)
    img = synth.segment_image(rng, 1024, 1024, 40, 300, 1000, 0.0)
    img = (img | (rng.random((1024, 1024)) < 0.33)).astype(np.uint8)
    x, y = points(img)
    assert len(x) > 40 * 1024 * 8
    say(f"case solution device bitmap: E {len(x)} T 1200 pass 0")
    want = expect(x, y, 1024, 1024, 1200, passes=1)
    with hh.HoughHier(threshold=1200, passes=1) as ctx:
        r = ctx.detect(image=img, width=1024, height=1024)
        ctx.solution(r)
        check(r, want, len(x), "device bitmap")
        r.free()


def test_solution_gray(hh):
    """Gray input: each pass walks its own point set (ALPHA or BETA), ids
    are ranks among all edge points."""
    rng = np.random.default_rng(3)
    W, H = 300, 220
    lines = synth.segment_image(rng, W, H, 12, 0.2 * H, 0.9 * W, 0.0)
    g = (rng.integers(0, 40, (H, W)) + lines.astype(np.int64) * 170).astype(np.uint8)
    x, y, beta = oracle.sobel_partition(g, 180)
    say(f"case solution gray: E {len(x)} alpha {int((~beta).sum())} beta {int(beta.sum())}")
    want = {}
    for p, sel in ((0, ~beta), (1, beta)):
        ids = np.nonzero(sel)[0]
        _, keep, plot_sub = oracle.solution(x[ids], y[ids], W, H, 15, 0, p)
        plotted = np.zeros(len(x), bool)
        plotted[ids[plot_sub]] = True
        want[p] = (keep, plotted)
    with hh.HoughHier(threshold=15) as ctx:
        r = ctx.detect(gray=g, edge_threshold=180, width=W, height=H)
        ctx.solution(r)
        check(r, want, len(x), "gray")
        check_image(r, want, x, y, "gray")
        import torch
        out = torch.full((H, W + 8), 7, dtype=torch.uint8, device="cuda")   # strided device rows
        r.solution_image(out[:, :W])
        torch.cuda.synchronize()
        ref = r.solution_image()
        np.testing.assert_array_equal(out[:, :W].cpu().numpy(), ref)
        assert (out[:, W:] == 7).all()
        r.free()


def test_solution_batch_served_and_mixed(hh):
    """One call over a batch's results, over served results (each on the
    lane that made it) and over results of two contexts at once."""
    imgs = [synth.full_span_image(30 + k, 60 + 23 * k, 140 - 9 * k, 5, 0.03) for k in range(6)]
    wants = []
    for im in imgs:
        x, y = points(im)
        wants.append((expect(x, y, im.shape[1], im.shape[0], 9), len(x)))
    say("case solution batch / served / mixed: 6 images")
    with hh.HoughHier(threshold=9) as ctx, hh.HoughHier(threshold=9) as srv:
        rs = ctx.detect_batch([dict(image=im, width=im.shape[1], height=im.shape[0]) for im in imgs])
        hh.solution(rs)
        for k, r in enumerate(rs):
            check(r, *wants[k], what=f"batch {k}")
            r.free()
        srv.serve_start(lanes=2, max_batch=3)
        ts = [srv.submit(image=im, width=im.shape[1], height=im.shape[0]) for im in imgs]
        served = [srv.poll(t) for t in ts]
        plain = [ctx.detect(image=im, width=im.shape[1], height=im.shape[0]) for im in imgs[:3]]
        hh.solution(served[:3] + plain + served[3:])
        for k, r in enumerate(served):
            check(r, *wants[k], what=f"served {k}")
            x, y = points(imgs[k])
            check_image(r, wants[k][0], x, y, f"served {k}")
            r.free()
        for k, r in enumerate(plain):
            check(r, *wants[k], what=f"plain {k}")
            r.free()


def test_solution_edge_cases(hh):
    say("case solution edge cases: no cells, depth 0, no membership, not solved")
    img = synth.full_span_image(2, 40, 40, 3, 0.0)
    x, y = points(img)
    with hh.HoughHier(threshold=10 ** 6) as ctx:   # nothing above T
        r = ctx.detect(image=img, width=40, height=40)
        with pytest.raises(hh.HHError) as e:
            r.solution(0)
        assert e.value.status == -1
        ctx.solution([r])
        for p in (0, 1):
            s = r.solution(p)
            assert s["kept"] == 0 and s["plotted_points"] == 0 and len(s["plotted"]) == len(x)
        r.free()
    with hh.HoughHier(threshold=0) as ctx:   # no edge points at all
        r = ctx.detect(image=np.zeros((16, 24), np.uint8), width=24, height=16)
        ctx.solution(r)
        for p in (0, 1):
            s = r.solution(p)
            assert s["kept"] == 0 and s["plotted_points"] == 0 and len(s["keep"]) == 0 and len(s["plotted"]) == 0
        assert (r.solution_image() == 0).all() and r.solution_image().shape == (16, 24)
        r.free()
    # a 1x1 image: depth 0, the root is the finest region and every point votes
    xs = np.zeros(7, np.int32)
    with hh.HoughHier(threshold=3) as ctx:
        r = ctx.detect(xs, xs, width=1, height=1)
        ctx.solution(r)
        check(r, expect(xs, xs, 1, 1, 3), 7, "depth 0")
        assert r.solution_image().tolist() == [[255]]
        r.free()
    with hh.HoughHier(threshold=5, membership=False) as ctx:
        r = ctx.detect(image=img, width=40, height=40)
        with pytest.raises(hh.HHError) as e:
            ctx.solution([r])
        assert e.value.status == -1
        r.free()
    with hh.HoughHier(threshold=5, passes=2) as ctx:   # one pass enabled
        r = ctx.detect(image=img, width=40, height=40)
        ctx.solution(r)
        check(r, expect(x, y, 40, 40, 5, passes=2), len(x), "pass 1 only")
        r.free()


def test_solution_seg1024_full_size(hh):
    """The benchmark image (1024x1024, T = 120, depth 10, both passes) in the
    configuration the benchmark times: every keep and plotted flag."""
    w = synth.workload("seg1024", 0)
    x, y = points(w.image)
    say(f"case solution seg1024 full size: E {len(x)}")
    want = expect(x, y, w.width, w.height, w.threshold, w.max_depth)
    with hh.HoughHier(threshold=w.threshold, max_depth=w.max_depth) as ctx:
        r = ctx.detect(image=w.image, width=w.width, height=w.height)
        ctx.solution(r)
        check(r, want, len(x), "seg1024")
        r.free()
