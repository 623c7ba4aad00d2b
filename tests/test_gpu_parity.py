"""GPU parity: the HIP path through the C ABI against the CPU oracle.

Everything is integer, so the bar is bit-exact: the same detected cells
(pass, i, j, key), the same votes, the same voters (ascending ids) and the
same per-level statistics.
"""
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


def gpu_detect(hh, x=None, y=None, *, W, H, T, dmax=0, variant="code", passes=3,
               membership=True, wide=False, image=None):
    with hh.HoughHier(threshold=T, max_depth=dmax, passes=passes, variant=variant,
                      membership=membership, wide_compare=wide) as ctx:
        r = ctx.detect(x, y, image=image, width=W, height=H)
        out = {"info": dict(r.info)}
        for p in (0, 1):
            out[p] = (r.cells(p), r.stats_array(p))
        out["members"] = r.members() if membership else None
        r.free()
    return out


def assert_matches(got, ref, passes=3, membership=True):
    for p in (0, 1):
        cells, stats = got[p]
        if not passes & (1 << p):
            assert len(cells) == 0 and len(stats) == 0
            continue
        want = ref.pass_cells(p)
        assert len(cells) == len(want), (p, len(cells), len(want))
        for f in ("i", "j", "key", "votes"):
            np.testing.assert_array_equal(cells[f], want[f], err_msg=f"pass {p} field {f}")
        assert np.all(cells["pass"] == p)
        np.testing.assert_array_equal(stats, ref.stats[p], err_msg=f"pass {p} stats")
        if membership:
            gm = got["members"]
            # compact host members: offsets are the running sum of votes
            for c in range(len(cells)):
                a = gm[cells["member_off"][c]: cells["member_off"][c] + cells["votes"][c]]
                o = want["member_off"][c]
                b = ref.members[o: o + want["votes"][c]]
                if not np.array_equal(a, b):
                    raise AssertionError(f"pass {p} cell {c} ({cells['i'][c]},{cells['j'][c]}) members differ")
        else:
            assert np.all(cells["member_off"] == -1)


def ref_detect(x, y, W, H, T, dmax=0, variant="code", passes=3, membership=True):
    return oracle.detect(x, y, W, H, T, dmax, variant, passes, membership)


def test_smoke_line256(hh):
    w = synth.workload("line256", 0)
    say("case line256 seed 0 code")
    x, y = oracle.edge_points(w.image)
    got = gpu_detect(hh, x, y, W=w.width, H=w.height, T=w.threshold, dmax=w.max_depth)
    assert_matches(got, ref_detect(x, y, w.width, w.height, w.threshold, w.max_depth))


@pytest.mark.parametrize("seed", range(1, 10))
def test_line256_seeds(hh, seed):
    w = synth.workload("line256", seed)
    say(f"case line256 seed {seed} code (image input)")
    x, y = oracle.edge_points(w.image)
    got = gpu_detect(hh, image=w.image, W=w.width, H=w.height, T=w.threshold, dmax=w.max_depth)
    assert got["info"]["n_points"] == len(x)
    assert_matches(got, ref_detect(x, y, w.width, w.height, w.threshold, w.max_depth))


@pytest.mark.parametrize("seed", range(4))
def test_line256_circle(hh, seed):
    w = synth.workload("line256", seed)
    say(f"case line256 seed {seed} circle")
    x, y = oracle.edge_points(w.image)
    got = gpu_detect(hh, x, y, W=w.width, H=w.height, T=w.threshold, dmax=w.max_depth,
                     variant="circle")
    assert_matches(got, ref_detect(x, y, w.width, w.height, w.threshold, w.max_depth, "circle"))


@pytest.mark.parametrize("seed,variant,wide", [(0, "code", False), (1, "code", False),
                                               (2, "code", True), (0, "circle", False)])
def test_seg1024(hh, seed, variant, wide):
    w = synth.workload("seg1024", seed)
    say(f"case seg1024 seed {seed} {variant} wide={wide}")
    x, y = oracle.edge_points(w.image)
    got = gpu_detect(hh, image=w.image, W=w.width, H=w.height, T=w.threshold, dmax=w.max_depth,
                     variant=variant, wide=wide)
    assert got["info"]["compare_bits"] == (64 if (wide or variant == "circle") else 32)
    assert_matches(got, ref_detect(x, y, w.width, w.height, w.threshold, w.max_depth, variant))


def test_input_forms_agree(hh):
    import torch
    w = synth.workload("line256", 3)
    say("case input forms: host/device image, host/device points")
    x, y = oracle.edge_points(w.image)
    ref = ref_detect(x, y, w.width, w.height, w.threshold, w.max_depth)
    dev_img = torch.from_numpy(w.image).cuda()
    dx = torch.from_numpy(x).cuda()
    dy = torch.from_numpy(y).cuda()
    # an image with a row stride larger than its width
    padded = torch.zeros((w.height, w.width + 24), dtype=torch.uint8, device="cuda")
    padded[:, : w.width] = dev_img
    for kw in (dict(image=w.image), dict(image=dev_img), dict(image=padded[:, : w.width]),
               dict(x=x, y=y), dict(x=dx, y=dy)):
        got = gpu_detect(hh, **kw, W=w.width, H=w.height, T=w.threshold, dmax=w.max_depth)
        assert_matches(got, ref)


def tiny(seed, W, H, p):
    rng = np.random.default_rng(seed)
    img = (rng.random((H, W)) < p).astype(np.uint8)
    return oracle.edge_points(img)


EDGE_CASES = [
    # (name, W, H, noise, T, dmax, passes)
    ("empty", 64, 64, 0.0, 0, 0, 3),
    ("one pixel image", 1, 1, 1.0, 0, 0, 3),
    ("1xN", 1, 200, 0.5, 3, 0, 3),
    ("Nx1", 300, 1, 0.5, 3, 0, 3),
    ("T=0 dense", 32, 32, 0.3, 0, 0, 3),
    ("T=E", 32, 32, 0.1, -1, 0, 3),
    ("depth 0", 40, 40, 0.2, 5, -1, 3),
    ("depth deeper than side", 64, 64, 0.05, 4, 9, 3),
    ("depth shallower", 128, 96, 0.05, 10, 3, 3),
    ("pass 0 only", 100, 80, 0.04, 6, 0, 1),
    ("pass 1 only", 100, 80, 0.04, 6, 0, 2),
    ("non-square ragged", 77, 201, 0.03, 7, 0, 3),
    ("tile-spanning", 512, 300, 0.02, 30, 0, 3),
]


@pytest.mark.parametrize("case", range(len(EDGE_CASES)))
@pytest.mark.parametrize("variant", ["code", "circle"])
def test_edge_cases(hh, case, variant):
    name, W, H, p, T, dmax, passes = EDGE_CASES[case]
    say(f"case edge {name} {variant}")
    x, y = tiny(1000 + case, W, H, p)
    if T < 0:
        T = len(x)
    ref = ref_detect(x, y, W, H, T, dmax, variant, passes)
    got = gpu_detect(hh, x, y, W=W, H=H, T=T, dmax=dmax, variant=variant, passes=passes)
    assert_matches(got, ref, passes)


def test_duplicates_and_membership_off(hh):
    say("case duplicates, membership off")
    x, y = tiny(5, 64, 64, 0.05)
    dx, dy = np.concatenate([x, x, x[:10]]), np.concatenate([y, y, y[:10]])
    ref = ref_detect(dx, dy, 64, 64, 9)
    assert_matches(gpu_detect(hh, dx, dy, W=64, H=64, T=9), ref)
    assert_matches(gpu_detect(hh, dx, dy, W=64, H=64, T=9, membership=False), ref, membership=False)


def test_invalid_inputs(hh):
    import torch
    say("case invalid inputs")
    with hh.HoughHier(threshold=1) as ctx:
        with pytest.raises(hh.HHError) as e:
            ctx.detect(np.array([5], np.int32), np.array([0], np.int32), width=5, height=5)
        assert e.value.status == -1
        bad = torch.tensor([0, 1, 7], dtype=torch.int32, device="cuda")
        ok = torch.tensor([0, 1, 2], dtype=torch.int32, device="cuda")
        with pytest.raises(hh.HHError) as e:
            ctx.detect(bad, ok, width=5, height=5)
        assert e.value.status == -1
        with pytest.raises(hh.HHError):
            ctx.detect(np.zeros(1, np.int32), np.zeros(1, np.int32), width=20000, height=5)
        with pytest.raises(hh.HHError):
            # S * 2^depth = 2^14 * 2^15 exceeds 2^28
            ctx.detect(np.zeros(1, np.int32), np.zeros(1, np.int32), width=16384, height=8,
                       max_depth=15)
        # the context still works after errors
        x, y = tiny(9, 32, 32, 0.2)
        r = ctx.detect(x, y, width=32, height=32)
        ref = ref_detect(x, y, 32, 32, 1)
        assert len(r.cells(0)) == len(ref.pass_cells(0))
        r.free()


def test_repeatable_and_context_reuse(hh):
    say("case repeat on one context")
    w = synth.workload("line256", 7)
    with hh.HoughHier(threshold=w.threshold, max_depth=w.max_depth) as ctx:
        outs = []
        for _ in range(3):
            r = ctx.detect(image=w.image, width=w.width, height=w.height)
            outs.append((r.cells(0), r.cells(1), r.members()))
        for o in outs[1:]:
            for a, b in zip(o, outs[0]):
                np.testing.assert_array_equal(a, b)


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
    return torch.as_tensor(_DevView(ptr, count * dtype.itemsize), device="cuda").cpu().numpy().view(dtype).copy()


def test_seg4096_full_size_sampled(hh):
    """The 4096x4096 workload at full size (the oracle takes minutes on it):
    sampled detected cells against the direct test of every line (a detected
    finest cell's voters are exactly the lines crossing it), sampled other
    finest cells hold at most T crossing lines, and the statistics keep
    their invariants.  Voters are compared as the packed points the kernels
    store, read from the device for the sampled cells only."""
    import torch
    w = synth.workload("seg4096", 0)
    say("case seg4096 full size, sampled cells")
    x, y = oracle.edge_points(w.image)
    packed = (x.astype(np.uint32) | (y.astype(np.uint32) << 16))
    img = torch.from_numpy(w.image).cuda()
    rng = np.random.default_rng(7)
    with hh.HoughHier(threshold=w.threshold, max_depth=w.max_depth) as ctx:
        r = ctx.detect(image=img, width=w.width, height=w.height)
        assert r.info["n_points"] == len(x)
        ent_ptr, n_ent, eb = r.member_points()
        assert eb == 4
        D = r.info["depth"]
        for p in (0, 1):
            dptr, n = r.device_cells(p)
            cells = dev_array(dptr, n, hh.CELL_DTYPE)
            st = r.stats(p)
            assert n == st["detected"][-1] and n > 0
            assert np.all(np.diff(cells["key"]) > 0) and np.all(cells["votes"] > w.threshold)
            np.testing.assert_array_equal(st["evaluated"][1:], 4 * st["split"][:-1])
            for c in rng.choice(n, size=min(40, n), replace=False):
                i, j, v, o = (int(cells[f][c]) for f in ("i", "j", "votes", "member_off"))
                want = oracle.region_voters(x, y, w.width, w.height, p, D, i, j)
                assert v == len(want), (p, i, j, v, len(want))
                got = dev_array(ent_ptr + 4 * o, v, np.uint32)
                np.testing.assert_array_equal(got, packed[want])
            detected = set(zip(cells["i"].tolist(), cells["j"].tolist()))
            n_side = 1 << D
            tried = 0
            while tried < 60:
                i, j = int(rng.integers(0, n_side)), int(rng.integers(0, n_side))
                if (i, j) in detected:
                    continue
                tried += 1
                assert len(oracle.region_voters(x, y, w.width, w.height, p, D, i, j)) <= w.threshold
        r.free()
