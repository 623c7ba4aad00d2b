"""GPU tests of serving (hough_hier_serve_start / submit / poll): a request's
result is the same alone (a plain call) and in the mix (continuous batches
on several lanes), failures stay with their request, and the queue bounds
hold."""
import sys
import time

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


def view(r):
    return [(r.cells(p), r.stats_array(p)) for p in (0, 1)], r.members()


def assert_same(a, b, what):
    for p in (0, 1):
        np.testing.assert_array_equal(a[0][p][0], b[0][p][0], err_msg=f"{what} pass {p} cells")
        np.testing.assert_array_equal(a[0][p][1], b[0][p][1], err_msg=f"{what} pass {p} stats")
    np.testing.assert_array_equal(a[1], b[1], err_msg=f"{what} members")


def test_served_equals_alone(hh):
    trace = synth.serving_trace(seed=3, rate_hz=400.0, duration_s=1.0, side_lo=64, side_hi=640,
                                mean_segments=12.0, max_requests=40)
    say(f"case serving: {len(trace)} requests, 3 lanes, batches of up to 6")
    with hh.HoughHier(threshold=0) as srv, hh.HoughHier(threshold=0) as plain:
        srv.serve_start(lanes=3, max_batch=6, max_batch_pixels=1 << 20)
        t0 = time.perf_counter()
        tickets = []
        for at, w in trace:   # submit on the trace's clock
            while time.perf_counter() - t0 < at:
                time.sleep(0.0005)
            tickets.append(srv.submit(image=w.image, width=w.width, height=w.height, threshold=w.threshold))
        results = [srv.poll(t) for t in tickets]
        for k, ((at, w), r) in enumerate(zip(trace, results)):
            tm = r.timing()
            assert tm["service_ms"] > 0 and tm["queue_ms"] >= 0
            one = plain.detect(image=w.image, width=w.width, height=w.height, threshold=w.threshold)
            assert_same(view(r), view(one), f"request {k}")
            # every request against the oracle: cells, statistics and voters
            x, y = oracle.edge_points(w.image)
            ref = oracle.detect(x, y, w.width, w.height, w.threshold, 0)
            members = r.members()
            for p in (0, 1):
                got, want = r.cells(p), ref.pass_cells(p)
                for f in ("i", "j", "key", "votes"):
                    np.testing.assert_array_equal(got[f], want[f], err_msg=f"request {k} pass {p} {f}")
                np.testing.assert_array_equal(r.stats_array(p), ref.stats[p])
                for c in range(len(got)):
                    o, v, wo = int(got["member_off"][c]), int(got["votes"][c]), int(want["member_off"][c])
                    np.testing.assert_array_equal(members[o:o + v], ref.members[wo:wo + v],
                                                  err_msg=f"request {k} pass {p} cell {c}")
            one.free()
            r.free()


def test_served_result_errors_carry_their_text(hh):
    """An error on a served result (made by a serving lane) reports its
    message through the result."""
    w = synth.workload("line256", 2)
    with hh.HoughHier(threshold=w.threshold, max_depth=w.max_depth) as srv:
        srv.serve_start(lanes=2, max_batch=4)
        r = srv.poll(srv.submit(image=w.image, width=w.width, height=w.height))
        with pytest.raises(hh.HHError) as e:
            r.solution(0)   # hough_hier_solution has not run on it
        assert e.value.status == -1 and "hough_hier_solution" in str(e.value)
        r.free()


def test_served_failure_stays_with_its_request(hh):
    import torch
    say("case serving: one bad request among good ones")
    rng = np.random.default_rng(4)
    good = []
    for _ in range(5):
        x = rng.integers(0, 50, 400).astype(np.int32)
        y = rng.integers(0, 60, 400).astype(np.int32)
        good.append((x, y))
    bad_x = torch.tensor([1, 2, 99], dtype=torch.int32, device="cuda")   # 99 >= width
    bad_y = torch.tensor([0, 1, 2], dtype=torch.int32, device="cuda")
    torch.cuda.synchronize()
    with hh.HoughHier(threshold=3) as srv, hh.HoughHier(threshold=3) as plain:
        srv.serve_start(lanes=1, max_batch=16)
        tickets = [srv.submit(x, y, width=50, height=60) for x, y in good[:2]]
        tb = srv.submit(bad_x, bad_y, width=50, height=60)
        tickets += [srv.submit(x, y, width=50, height=60) for x, y in good[2:]]
        with pytest.raises(hh.HHError) as e:
            srv.poll(tb)
        assert e.value.status == -1
        for (x, y), t in zip(good, tickets):
            r = srv.poll(t)
            one = plain.detect(x, y, width=50, height=60)
            assert_same(view(r), view(one), "good request")
            r.free()
            one.free()


def test_queue_bounds_and_tickets(hh):
    say("case serving: queue capacity, unknown tickets, pending polls")
    img = np.zeros((300, 300), np.uint8)
    img[100, :] = 1
    img[:, 40] = 1
    with hh.HoughHier(threshold=5) as srv:
        with pytest.raises(hh.HHError):
            srv.submit(image=img, width=300, height=300)   # not serving yet
        srv.serve_start(lanes=1, max_batch=4, queue_capacity=3)
        with pytest.raises(hh.HHError):
            srv.serve_start()
        ts = [srv.submit(image=img, width=300, height=300) for _ in range(3)]
        with pytest.raises(hh.HHError) as e:
            srv.submit(image=img, width=300, height=300)
        assert e.value.status == -5
        with pytest.raises(hh.HHError) as e:
            srv.poll(10 ** 9, 0)
        assert e.value.status == -1
        first = srv.poll(ts[0], 0)   # may still be pending
        rs = [first if first is not None else srv.poll(ts[0])] + [srv.poll(t) for t in ts[1:]]
        for r in rs[1:]:
            np.testing.assert_array_equal(r.cells(0), rs[0].cells(0))
        with pytest.raises(hh.HHError):
            srv.poll(ts[0], 0)   # a ticket is consumed by the poll that returns it
        n0 = len(rs[0].cells(0))
        for r in rs:
            r.free()
        # plain calls still work on a serving context
        r = srv.detect(image=img, width=300, height=300)
        assert len(r.cells(0)) == n0
        r.free()
        # unclaimed tickets are released with the context
        srv.submit(image=img, width=300, height=300)


def test_slab_holds_batches_and_held_results(hh):
    """Every batch runs inside the serving slab; results keep their batch's
    slab space until freed; a request that finds no room while results are
    held runs outside the slab, with the same result as a plain call."""
    trace = synth.serving_trace(seed=5, rate_hz=1000.0, duration_s=1.0, side_lo=256, side_hi=512,
                                mean_segments=10.0, max_requests=18)
    ws = [w for _, w in trace]
    say(f"case serving slab: {len(ws)} requests, 256 MiB slab, 2 lanes")
    with hh.HoughHier(threshold=0, hbm_budget_bytes=256 << 20) as srv, hh.HoughHier(threshold=0) as plain:
        srv.serve_start(lanes=2, max_batch=4)
        st = srv.serve_stats()
        assert st["slab_bytes"] == 256 << 20 and st["slab_used"] == 0
        assert st["internal_reruns"] == 0 and st["internal_failures"] == 0 and st["first_internal_error"] == ""
        # requests freed as they complete: all inside the slab
        for w in ws[:8]:
            r = srv.poll(srv.submit(image=w.image, width=w.width, height=w.height, threshold=w.threshold))
            one = plain.detect(image=w.image, width=w.width, height=w.height, threshold=w.threshold)
            assert_same(view(r), view(one), "freed request")
            r.free()
            one.free()
        st = srv.serve_stats()
        assert st["outside_batches"] == 0 and st["slab_batches"] >= 1 and st["slab_used"] == 0, st
        # results held by the client: their space stays taken, and requests
        # that no longer fit still complete
        held = []
        for k, w in enumerate(ws[8:]):
            r = srv.poll(srv.submit(image=w.image, width=w.width, height=w.height, threshold=w.threshold))
            held.append((w, r))
        st = srv.serve_stats()
        say(f"  stats with {len(held)} results held: {st}")
        assert st["slab_used"] > 0
        for w, r in held:
            one = plain.detect(image=w.image, width=w.width, height=w.height, threshold=w.threshold)
            assert_same(view(r), view(one), "held request")
            one.free()
        for _, r in held:
            r.free()
        st = srv.serve_stats()
        assert st["slab_used"] == 0
        # a batch whose internal check fails runs once more; it never fails twice here
        assert st["internal_failures"] == 0, st
