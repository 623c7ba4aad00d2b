"""The device-side voter checksum (tests/digests.py) against the oracle's
definition, on the CPU: torch int64 arithmetic wraps modulo 2^64 as the
definition requires, and a list cut into pieces sums to the whole."""
import numpy as np
import torch

import digests
import oracle


def test_voter_digest_matches_oracle_definition():
    rng = np.random.default_rng(1)
    for n in (0, 1, 7, 1000, 70000):
        ids = rng.integers(0, (1 << 31) - 1, n).astype(np.int32)
        assert digests.voter_digest(torch.from_numpy(ids)) == oracle.member_digest(ids)


def test_voter_digest_chunks_and_offsets(monkeypatch):
    monkeypatch.setattr(digests, "CHUNK", 1000)
    rng = np.random.default_rng(2)
    ids = rng.integers(0, 1 << 24, 5555).astype(np.int32)
    whole = oracle.member_digest(ids)
    assert digests.voter_digest(torch.from_numpy(ids)) == whole
    a = digests.voter_digest(torch.from_numpy(ids[:2000]))
    b = digests.voter_digest(torch.from_numpy(ids[2000:]), start=2000)
    assert (a + b) % (1 << 64) == whole


def test_first_difference_names_the_level():
    s = {"stats": [[1, 2, 3, 4, 5, 6], [7, 8, 9, 10, 11, 12]], "n_cells": 1, "cells_sha256": "x",
         "n_members": 3, "member_digest": 5}
    t = {**s, "stats": [[1, 2, 3, 4, 5, 6], [7, 8, 9, 10, 11, 13]]}
    assert digests.first_difference(s, s) is None
    assert digests.first_difference(t, s).startswith("stats level 1")
    assert digests.first_difference({**s, "member_digest": 6}, s).startswith("member_digest")
