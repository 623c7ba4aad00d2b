"""Seeded synthetic binary edge images for the hierarchical Hough vote.

The paper evaluates on three 256x256 gray images that are not published
(Sec. 4.1, Figs. 3-5); no public dataset is named.  These generators stand
in for them with images of the same kind: a few straight edges (1-2 px
thick) over salt noise, at the sizes of the workloads the vote is measured
on.  Both the CPU oracle and the HIP path consume the images (or the point
lists derived from them) produced here, so the two always see identical
inputs.

This module only draws pixels.  It holds none of the method's arithmetic:
no parameter-space mapping, no corner codes, no votes.  An image is a
``uint8`` array of shape ``(H, W)``; nonzero pixels are edge points, with
``x`` the column and ``y`` the row.

Recipes (all from ``numpy.random.default_rng(seed)``):

* ``full_span_image``: lines that run from one border to the opposite one
  along their major axis (so each has exactly ``W`` or ``H`` pixels), angle
  uniform in [0, pi), offset uniform over the range that keeps the whole
  line inside the image, then Bernoulli(p) salt noise.
* ``segment_image``: segments with centre uniform in the image, angle
  uniform in [0, pi), length uniform in a range, thickness drawn from a set
  (default 1 or 2; a segment t pixels thick is t copies shifted by
  0 .. t-1 on the minor axis), clipped to the image, plus Bernoulli(p) salt
  noise.
* Segments are rasterised by stepping the major axis one pixel at a time
  and rounding the minor coordinate to nearest (DDA).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List

import numpy as np

__all__ = [
    "Workload", "full_span_image", "segment_image", "workload",
    "batch_images", "serving_trace", "WORKLOADS",
]


def _round(a):
    return np.floor(np.asarray(a, dtype=np.float64) + 0.5).astype(np.int64)


def _plot(img: np.ndarray, xs: np.ndarray, ys: np.ndarray) -> None:
    H, W = img.shape
    keep = (xs >= 0) & (xs < W) & (ys >= 0) & (ys < H)
    img[ys[keep], xs[keep]] = 1


def _draw_segment(img: np.ndarray, x0: float, y0: float, x1: float, y1: float,
                  thick: int) -> None:
    """Rasterise a segment by DDA along its major axis; a segment ``thick``
    pixels thick is drawn with copies shifted by 0 .. thick-1 on the minor
    axis."""
    dx, dy = x1 - x0, y1 - y0
    if abs(dx) >= abs(dy):
        a, b = int(_round(min(x0, x1))), int(_round(max(x0, x1)))
        xs = np.arange(a, b + 1, dtype=np.int64)
        slope = dy / dx if dx != 0 else 0.0
        ys = _round(y0 + slope * (xs - x0))
        for k in range(thick):
            _plot(img, xs, ys + k)
    else:
        a, b = int(_round(min(y0, y1))), int(_round(max(y0, y1)))
        ys = np.arange(a, b + 1, dtype=np.int64)
        slope = dx / dy
        xs = _round(x0 + slope * (ys - y0))
        for k in range(thick):
            _plot(img, xs + k, ys)


def _salt(rng: np.random.Generator, img: np.ndarray, p: float) -> None:
    if p > 0:
        img[rng.random(img.shape) < p] = 1


def full_span_image(seed: int, W: int = 256, H: int = 256, n_lines: int = 8,
                    noise: float = 0.01) -> np.ndarray:
    """``n_lines`` border-to-border 1-px lines plus salt noise."""
    rng = np.random.default_rng(seed)
    img = np.zeros((H, W), dtype=np.uint8)
    for _ in range(n_lines):
        th = rng.uniform(0.0, math.pi)
        c, s = math.cos(th), math.sin(th)
        if abs(c) >= abs(s):              # major axis x: y = off + k*x
            k = s / c
            lo = max(0.0, -k * (W - 1))
            hi = min(H - 1.0, (H - 1.0) - k * (W - 1))
            off = rng.uniform(lo, hi) if hi > lo else lo
            xs = np.arange(W, dtype=np.int64)
            ys = np.clip(_round(off + k * xs), 0, H - 1)
        else:                             # major axis y: x = off + k*y
            k = c / s
            lo = max(0.0, -k * (H - 1))
            hi = min(W - 1.0, (W - 1.0) - k * (H - 1))
            off = rng.uniform(lo, hi) if hi > lo else lo
            ys = np.arange(H, dtype=np.int64)
            xs = np.clip(_round(off + k * ys), 0, W - 1)
        _plot(img, xs, ys)
    _salt(rng, img, noise)
    return img


def segment_image(rng: np.random.Generator, W: int, H: int, n_seg: int,
                  len_lo: float, len_hi: float, noise: float,
                  thick_choices=(1, 2)) -> np.ndarray:
    """Random clipped segments (centre, angle, length, thickness) plus noise."""
    img = np.zeros((H, W), dtype=np.uint8)
    for _ in range(n_seg):
        cx, cy = rng.uniform(0, W - 1), rng.uniform(0, H - 1)
        th = rng.uniform(0.0, math.pi)
        ln = rng.uniform(len_lo, len_hi)
        thick = int(rng.choice(thick_choices))
        hx, hy = 0.5 * ln * math.cos(th), 0.5 * ln * math.sin(th)
        _draw_segment(img, cx - hx, cy - hy, cx + hx, cy + hy, thick)
    _salt(rng, img, noise)
    return img


@dataclass
class Workload:
    """One single-image workload: the image plus its vote parameters."""
    name: str
    image: np.ndarray
    threshold: int
    max_depth: int = 0          # 0 = ceil(log2(max(W, H)))
    meta: dict = field(default_factory=dict)

    @property
    def width(self) -> int:
        return int(self.image.shape[1])

    @property
    def height(self) -> int:
        return int(self.image.shape[0])


def _side_threshold(W: int, H: int) -> int:
    # votes > 0.1*side for integer votes is votes > floor(side/10)
    return max(W, H) // 10


def workload(name: str, seed: int = 0) -> Workload:
    """The single-image workloads, by name.

    * ``line256``: 256x256, 8 full-span lines, 1% noise, T=40, depth 8.
    * ``seg1024``: 1024x1024, 32 segments of length U[200,1000], 2% noise,
      T=120, depth 10.
    * ``seg4096``: 4096x4096, 128 segments of length U[500,4000], 2-3 px
      thick (the thickness is the one parameter the workload leaves open;
      2-3 px brings seed 0 to the ~700k edge points it names), 1% noise,
      T=300, depth 12.
    """
    if name == "line256":
        img = full_span_image(seed, 256, 256, 8, 0.01)
        return Workload(name, img, 40, 8, {"seed": seed})
    rng = np.random.default_rng(seed)
    if name == "seg1024":
        img = segment_image(rng, 1024, 1024, 32, 200.0, 1000.0, 0.02)
        return Workload(name, img, 120, 10, {"seed": seed})
    if name == "seg4096":
        img = segment_image(rng, 4096, 4096, 128, 500.0, 4000.0, 0.01, thick_choices=(2, 3))
        return Workload(name, img, 300, 12, {"seed": seed})
    raise KeyError(name)


WORKLOADS = ("line256", "seg1024", "seg4096")


def _log_uniform_int(rng, lo: int, hi: int) -> int:
    return int(round(math.exp(rng.uniform(math.log(lo), math.log(hi)))))


def batch_images(seed: int = 0, n: int = 512, side_lo: int = 128,
                 side_hi: int = 2048, mean_segments: float = 24.0,
                 noise_lo: float = 0.005, noise_hi: float = 0.03) -> List[Workload]:
    """Mixed-size batch: W and H log-uniform in [side_lo, side_hi], Poisson
    segment counts, segment length U[0.2, 1.0]*min(W, H), per-image noise
    U[noise_lo, noise_hi], T = floor(max(W, H)/10), default depth."""
    rng = np.random.default_rng(seed)
    out = []
    for k in range(n):
        W = _log_uniform_int(rng, side_lo, side_hi)
        H = _log_uniform_int(rng, side_lo, side_hi)
        K = int(rng.poisson(mean_segments))
        p = float(rng.uniform(noise_lo, noise_hi))
        m = min(W, H)
        img = segment_image(rng, W, H, K, 0.2 * m, 1.0 * m, p)
        out.append(Workload(f"batch{k}", img, _side_threshold(W, H), 0,
                            {"seed": seed, "index": k, "segments": K, "noise": p}))
    return out


def serving_trace(seed: int, rate_hz: float, duration_s: float,
                  side_lo: int = 256, side_hi: int = 4096,
                  mean_segments: float = 48.0, noise: float = 0.01,
                  max_requests: int | None = None):
    """Poisson arrivals at ``rate_hz`` over ``duration_s`` seconds.

    Returns a list of ``(arrival_s, Workload)``; images are drawn in
    arrival order from one generator, so a trace is fixed by its seed."""
    rng = np.random.default_rng(seed)
    t, out = 0.0, []
    while True:
        t += float(rng.exponential(1.0 / rate_hz))
        if t >= duration_s or (max_requests is not None and len(out) >= max_requests):
            break
        W = _log_uniform_int(rng, side_lo, side_hi)
        H = _log_uniform_int(rng, side_lo, side_hi)
        K = int(rng.poisson(mean_segments))
        m = min(W, H)
        img = segment_image(rng, W, H, K, 0.2 * m, 1.0 * m, noise)
        out.append((t, Workload(f"req{len(out)}", img, _side_threshold(W, H), 0,
                                {"seed": seed, "segments": K})))
    return out
