"""HH_FLAG_GRAPH: a context with a caller arena captures a call's level
launches into a HIP graph and replays it for calls with the same sizes and
addresses.  Every replay is checked against an eager call (a context
without the flag) on the same input, with eager work and synchronisation
between the replays; new image contents in the same buffer replay the same
graph and give the new image's result; a different size captures anew."""
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


def view(r):
    return [(r.cells(p), r.stats_array(p)) for p in (0, 1)], r.members()


def same(a, b, what):
    for p in (0, 1):
        np.testing.assert_array_equal(a[0][p][0], b[0][p][0], err_msg=f"{what} pass {p} cells")
        np.testing.assert_array_equal(a[0][p][1], b[0][p][1], err_msg=f"{what} pass {p} stats")
    np.testing.assert_array_equal(a[1], b[1], err_msg=f"{what} members")


def test_graph_replays_match_eager(hh):
    import torch
    arena = torch.empty(256 << 20, dtype=torch.uint8, device="cuda")
    w0, w1 = synth.workload("line256", 0), synth.workload("line256", 5)
    buf = torch.from_numpy(w0.image).cuda()
    side = torch.cuda.Stream()   # a graph is captured on a stream of its own, not the null stream
    say("case graph replays: line256 seeds 0 and 5 in one device buffer")
    with hh.HoughHier(threshold=40, max_depth=8, arena=arena, graph=True, stream=side) as g, \
            hh.HoughHier(threshold=40, max_depth=8) as eager:
        replays = 0
        for k in range(6):
            w = w0 if k % 3 != 2 else w1
            buf.copy_(torch.from_numpy(w.image))
            torch.cuda.synchronize()
            r = g.detect(image=buf, width=256, height=256)
            replays += r.timing()["graph_replayed"]
            e = eager.detect(image=buf, width=256, height=256)
            same(view(r), view(e), f"call {k}")
            r.free()
            e.free()
            # eager work of the program between replays
            other = eager.detect(image=synth.workload("line256", 9).image, width=256, height=256)
            other.free()
            torch.cuda.synchronize()
        assert replays == 5
        # another size: captured anew
        w2 = synth.full_span_image(2, 200, 150, 6, 0.01)
        d2 = torch.from_numpy(w2).cuda()
        torch.cuda.synchronize()
        r = g.detect(image=d2, width=200, height=150)
        assert r.timing()["graph_replayed"] == 0
        e = eager.detect(image=d2, width=200, height=150)
        same(view(r), view(e), "new size")
        r.free()
        e.free()
