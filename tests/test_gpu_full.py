"""Full-size GPU parity on the two largest workloads against the oracle's
fixtures (``tests/golden/*_seed0.json``, written by
``tests/golden/make_full_golden.py`` from ``oracle/`` alone).

Per pass, everything is compared: the exact per-level statistics, the number
of detected cells, a sha256 over every cell's (i, j, key, votes) in key
order, the number of voters and the checksum over every voter id in order
(computed on the device).  Both run in the launch configuration the
benchmark times (default context, voters kept on the device)."""
import json
import os
import sys

import numpy as np
import pytest

import digests
import synth

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


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


def compare(res, want_passes, where):
    ids_ptr, _ = res.device_members()
    for p in (0, 1):
        got = digests.pass_summary(res, p, ids_ptr)
        diff = digests.first_difference(got, want_passes[str(p)])
        assert diff is None, f"{where} pass {p}: {diff}"


def test_seg4096_full_parity(hh):
    import torch
    g = json.load(open(os.path.join(GOLDEN, "seg4096_seed0.json")))
    w = synth.workload("seg4096", 0)
    say(f"case seg4096 seed 0 full parity (E={g['E']})")
    img = torch.from_numpy(w.image).cuda()
    with hh.HoughHier(threshold=w.threshold, max_depth=w.max_depth) as ctx:
        r = ctx.detect(image=img, width=w.width, height=w.height)
        assert r.info["n_points"] == g["E"]
        compare(r, g["passes"], "seg4096")
        r.free()


def test_batch512_full_parity(hh):
    import torch
    g = json.load(open(os.path.join(GOLDEN, "batch512_seed0.json")))
    ws = synth.batch_images(seed=0, n=512)
    say("case batch of 512, every image against the oracle fixture")
    imgs = [torch.from_numpy(w.image).cuda() for w in ws]
    with hh.HoughHier(threshold=0) as ctx:
        rs = ctx.detect_batch([dict(image=d, width=w.width, height=w.height, threshold=w.threshold)
                               for d, w in zip(imgs, ws)])
        say(f"  groups {rs[0].timing()['groups']}")
        for k, (w, r, want) in enumerate(zip(ws, rs, g["images"])):
            assert (w.width, w.height, w.threshold) == (want["W"], want["H"], want["T"])
            assert r.info["n_points"] == want["E"], f"image {k}"
            compare(r, want["passes"], f"image {k} ({w.width}x{w.height})")
        for r in rs:
            r.free()
