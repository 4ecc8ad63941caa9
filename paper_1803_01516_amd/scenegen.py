"""Seeded synthetic rectified stereo pairs with exact depth-number ground truth.

This module is the one input generator shared by the tests, the benchmark and
the oracle checks.  It holds none of the method's arithmetic (no cost volume,
no graph, no flow): it only renders images whose true cross points are known.

Geometry follows the gaze-line model (Sec. 3, Sec. 4.1 of the paper): the
surface is a depth number S(x, y) per gaze line; the cross point of site x at
depth S joins left pixel xl = x - S + (m-1) and right pixel xr = x + S - (m-1)
on the same row, so pixel disparity xl - xr = 2(m-1-S) (one depth step is two
pixels; Sec. 4.1).  The paper's model seeks continuous surfaces (neighbouring
depth numbers differ by at most one; Sec. 3), so the generated ground truth is
made 1-Lipschitz over 4-neighbours, which turns depth jumps at plane
boundaries into ramps along rays and leaves half-occluded pixels.

Recipe (stand-in for the Middlebury pair the paper uses, which is not shipped):
  1. P planes; Voronoi regions of P uniform seed points (ties to the lower
     index); plane depth round(c + a(x-x_p) + b(y-y_p)) clamped to [0, m-1];
     fronto-parallel planes have a = b = 0 and integer c.
  2. Lower 1-Lipschitz envelope (L1 metric), then S >= max(m-1-x, x+m-w) so
     every true cross point lies inside both images.
  3. Per row, cross points that share a left or right pixel form one class;
     each class gets one texel U{0..255}; unmatched pixels get their own;
     textureless rectangles give every class they touch one constant texel.
  4. Independent Gaussian noise per pixel, rounded and clamped to [0, 255].
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


@dataclass(frozen=True)
class SceneSpec:
    w: int
    h: int
    m: int
    planes: tuple[int, int]       # inclusive range for the plane count
    slanted: bool
    sigma: float
    cap: int
    lam: int = 1
    inhibit: int = 1023
    textureless: float = 0.0      # fraction of sites covered by flat regions
    name: str = ""
    channels: int = 1             # 3: colour images [h][w][3] (texels are RGB triples)


# Workloads (shapes, value distributions and structure of the paper's
# Tsukuba experiment, scaled as listed).
TINY = SceneSpec(64, 48, 8, (3, 3), False, 2.0, 20, name="tiny-64x48x8")
MID = SceneSpec(384, 288, 16, (6, 10), True, 3.0, 30, name="mid-384x288x16")
LARGE = SceneSpec(450, 375, 64, (12, 12), True, 2.0, 30, textureless=0.10,
                  name="large-450x375x64")
# Colour pairs for the paper's own data term (Sec. 4.3: RGB sum of absolute
# differences, untruncated, penalty 14, inhibit 1023).
MID_RGB = SceneSpec(384, 288, 16, (6, 10), True, 3.0, 765, lam=14, channels=3,
                    name="mid-rgb-384x288x16")
BATCH_SHAPES = ((320, 240, 16), (384, 288, 16), (450, 375, 64), (640, 480, 64))
SERVE_SHAPES = ((384, 288, 16), (640, 480, 64), (1280, 720, 128))


def spec_like(base: SceneSpec, w: int, h: int, m: int, **kw) -> SceneSpec:
    d = dict(base.__dict__)
    d.update(w=w, h=h, m=m, name=f"{w}x{h}x{m}")
    d.update(kw)
    return SceneSpec(**d)


@dataclass
class Pair:
    left: np.ndarray      # uint8 [h][w]
    right: np.ndarray     # uint8 [h][w]
    gt: np.ndarray        # int32 [h][w], true depth number per site
    spec: SceneSpec
    seed: tuple = field(default_factory=tuple)


def _lipschitz_envelope(S: np.ndarray) -> np.ndarray:
    """Largest function <= S with |f(u)-f(v)| <= |dx|+|dy| (separable L1)."""
    f = S.astype(np.int64)
    for axis in (1, 0):
        n = f.shape[axis]
        idx = np.arange(n).reshape((1, n) if axis == 1 else (n, 1))
        fwd = np.minimum.accumulate(f - idx, axis=axis) + idx
        rev_f = np.flip(f, axis=axis)
        bwd = np.flip(np.minimum.accumulate(rev_f - idx, axis=axis) + idx, axis=axis)
        f = np.minimum(fwd, bwd)
    return f


def _regions(rng, w, h, frac):
    """Axis-aligned rectangles until at least `frac` of the sites are covered."""
    rects = []
    if frac <= 0:
        return rects
    cover = np.zeros((h, w), dtype=bool)
    while cover.mean() < frac:
        rw = int(rng.integers(max(2, w // 12), max(3, w // 5)))
        rh = int(rng.integers(max(2, h // 12), max(3, h // 5)))
        x0 = int(rng.integers(0, max(1, w - rw)))
        y0 = int(rng.integers(0, max(1, h - rh)))
        val = int(rng.integers(0, 256))
        rects.append((x0, y0, rw, rh, val))
        cover[y0:y0 + rh, x0:x0 + rw] = True
    return rects


def depth_surface(spec: SceneSpec, rng: np.random.Generator) -> np.ndarray:
    w, h, m = spec.w, spec.h, spec.m
    lo, hi = spec.planes
    P = int(rng.integers(lo, hi + 1))
    px = rng.uniform(0, w, P)
    py = rng.uniform(0, h, P)
    if spec.slanted:
        a = rng.uniform(-0.25, 0.25, P)
        b = rng.uniform(-0.25, 0.25, P)
        c = rng.uniform(0, m - 1, P)
    else:
        a = np.zeros(P)
        b = np.zeros(P)
        c = rng.integers(0, m, P).astype(np.float64)
    ys, xs = np.mgrid[0:h, 0:w]
    d2 = (xs[None] - px[:, None, None]) ** 2 + (ys[None] - py[:, None, None]) ** 2
    region = np.argmin(d2, axis=0)                  # ties -> lower index
    raw = np.floor(c[region] + a[region] * (xs - px[region])
                   + b[region] * (ys - py[region]) + 0.5)
    raw = np.clip(raw, 0, m - 1).astype(np.int64)
    S = _lipschitz_envelope(raw)
    x = np.arange(w)[None, :]
    S = np.maximum(S, np.maximum(m - 1 - x, x + m - w))
    S = np.clip(S, 0, m - 1)
    return S.astype(np.int32)


def render(S: np.ndarray, spec: SceneSpec, rng: np.random.Generator):
    """Noise-free left/right images whose true cross points are exactly S."""
    h, w = S.shape
    m = spec.m
    x = np.arange(w)[None, :]
    xl = x - S + (m - 1)
    xr = x + S - (m - 1)
    assert xl.min() >= 0 and xl.max() < w and xr.min() >= 0 and xr.max() < w
    ch = () if spec.channels == 1 else (spec.channels,)
    T = rng.integers(0, 256, size=(h, 2 * w) + ch)
    rects = _regions(rng, w, h, spec.textureless)
    # Consecutive sites share a pixel iff their depths differ by one, so the
    # classes along a row are runs that break wherever the depth is flat.
    same = np.zeros((h, w), dtype=bool)
    same[:, 1:] = np.diff(S, axis=1) != 0
    first = np.where(~same, np.broadcast_to(x, (h, w)), 0)
    first = np.maximum.accumulate(first, axis=1)          # first site of the class
    cls_xl = np.take_along_axis(xl, first, axis=1)        # its left pixel
    idx = cls_xl if not ch else cls_xl[..., None]
    tex = np.take_along_axis(T, idx, axis=1)              # class texel
    if rects:
        cid = np.cumsum(~same, axis=1) - 1 + (np.arange(h) * w)[:, None]
        over = np.full(h * w, -1, dtype=np.int64)
        site_over = np.full((h, w), -1, dtype=np.int64)
        for (x0, y0, rw, rh, val) in rects:
            site_over[y0:y0 + rh, x0:x0 + rw] = val
        np.maximum.at(over, cid.ravel(), site_over.ravel())
        o = over[cid]
        if ch:
            o = o[..., None]                              # a grey texel in every channel
        tex = np.where(o >= 0, o, tex)
    left = T[:, :w].copy()
    right = T[:, w:].copy()
    rows = np.broadcast_to(np.arange(h)[:, None], (h, w))
    left[rows, xl] = tex
    right[rows, xr] = tex
    return left, right


def make_pair(spec: SceneSpec, seed) -> Pair:
    """Deterministic: the same (spec, seed) always gives the same bytes."""
    rng = np.random.default_rng(seed)
    S = depth_surface(spec, rng)
    left, right = render(S, spec, rng)
    if spec.sigma > 0:
        left = left + rng.normal(0.0, spec.sigma, left.shape)
        right = right + rng.normal(0.0, spec.sigma, right.shape)
    left = np.clip(np.rint(left), 0, 255).astype(np.uint8)
    right = np.clip(np.rint(right), 0, 255).astype(np.uint8)
    seed_t = tuple(seed) if isinstance(seed, (list, tuple)) else (seed,)
    return Pair(left, right, S, spec, seed_t)


def eq2_error(gt: np.ndarray, labels: np.ndarray):
    """Error of eq. (2): sum of |true - estimated| depth numbers, and the
    share of exact sites in percent, floored as the paper's tables print it."""
    d = np.abs(gt.astype(np.int64) - labels.astype(np.int64))
    err = int(d.sum())
    pct = int((100 * int((d == 0).sum())) // max(1, d.size))
    return err, pct
