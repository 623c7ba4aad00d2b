"""Checksums of GPU results in the form of the full-size fixtures
(``tests/golden/make_full_golden.py``): a sha256 over a pass's cells and the
voter checksum ``oracle.member_digest`` defines (sum over positions t of
(t A + B) (id + 1) modulo 2^64), the latter computed with torch on the
device so gigabytes of voters never leave it."""
import numpy as np

from make_full_golden import cells_sha256  # noqa: F401  (same definition as the fixtures)

DIGEST_A = 0x9E3779B97F4A7C15
DIGEST_B = 0x632BE59BD9B4E019
MASK64 = (1 << 64) - 1
CHUNK = 1 << 26


def _signed(v: int) -> int:
    return v - (1 << 64) if v >= (1 << 63) else v


def voter_digest(ids, start: int = 0) -> int:
    """Checksum of the voter list ``ids`` (a 1-D int32 torch tensor on any
    device) whose first entry sits at position ``start`` of the pass's list.
    int64 products and sums wrap modulo 2^64, which is the arithmetic the
    checksum is defined in."""
    import torch
    a = torch.tensor(_signed(DIGEST_A), dtype=torch.int64, device=ids.device)
    b = torch.tensor(_signed(DIGEST_B), dtype=torch.int64, device=ids.device)
    total = 0
    n = int(ids.numel())
    for s in range(0, n, CHUNK):
        part = ids[s: s + CHUNK].to(torch.int64) + 1
        t = torch.arange(start + s, start + s + part.numel(), dtype=torch.int64, device=ids.device)
        total = (total + int((t * a + b).mul_(part).sum().item())) & MASK64
    return total


class DevView:
    """A device byte range as a torch tensor (no copy)."""

    def __init__(self, ptr, nbytes):
        self.__cuda_array_interface__ = {"shape": (int(nbytes),), "typestr": "|u1",
                                         "data": (int(ptr), False), "version": 2}


def device_ids(ptr: int, first: int, count: int):
    """int32 voter ids [first, first + count) of a device id buffer."""
    import torch
    if count == 0:
        return torch.zeros(0, dtype=torch.int32, device="cuda")
    return torch.as_tensor(DevView(ptr + 4 * first, 4 * count), device="cuda").view(torch.int32)


def pass_summary(res, p, ids_ptr=None):
    """Summary of pass p of a GPU result in the fixtures' form, from its
    device cells and device voter ids (cells of a pass hold consecutive
    voter ranges, checked here)."""
    cells = res.cells(p)
    st = res.stats_array(p)
    out = {"stats": st.tolist(), "n_cells": int(len(cells)),
           "cells_sha256": cells_sha256(cells["i"], cells["j"], cells["key"], cells["votes"]),
           "n_members": int(cells["votes"].astype(np.int64).sum())}
    if ids_ptr is not None and len(cells):
        dptr, n = res.device_cells(p)
        import torch
        dc = torch.as_tensor(DevView(dptr, n * cells.dtype.itemsize), device="cuda").cpu().numpy()
        dcells = dc.view(cells.dtype)
        off = dcells["member_off"].astype(np.int64)
        v = dcells["votes"].astype(np.int64)
        assert np.all(off[1:] == off[:-1] + v[:-1]), "voters of a pass are not consecutive"
        out["member_digest"] = voter_digest(device_ids(ids_ptr, int(off[0]), int(v.sum())))
    elif ids_ptr is not None:
        out["member_digest"] = 0
    return out


def first_difference(got, want):
    """Where two pass summaries first differ (a stats level first)."""
    gs, ws = np.array(got["stats"]), np.array(want["stats"])
    if gs.shape != ws.shape:
        return f"stats shape {gs.shape} vs {ws.shape}"
    for lev in range(len(ws)):
        if not np.array_equal(gs[lev], ws[lev]):
            return f"stats level {lev}: {gs[lev].tolist()} vs {ws[lev].tolist()}"
    for k in ("n_cells", "cells_sha256", "n_members", "member_digest"):
        if k in got and got[k] != want[k]:
            return f"{k}: {got[k]} vs {want[k]}"
    return None
