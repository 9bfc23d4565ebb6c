"""Seeded synthetic inputs for the selective-segmentation solver.

The paper measures on its own real images (Fig. 1(a) and Problems 1-3 of
Sec. 5), which are not available; these generators stand in for them with
piecewise-constant objects on a dark background, noise and (for the large
images) blur and illumination bias.  This module holds none of the method's
arithmetic: it only draws images, marker points and the generator's own
target mask.  Both the GPU library and the CPU oracle consume its output.

Every generator uses ``numpy.random.Generator(PCG64(seed))``; images are
produced in float64 and rounded once to float32.  Markers are (row, col)
pixel coordinates of cell centres (cell (i, j) has centre (i + 0.5, j + 0.5)).
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np
from scipy import ndimage


@dataclass
class Instance:
    image: np.ndarray      # float32 (n, m) in [0, 1]
    markers: np.ndarray    # float64 (k, 2) pixel coordinates (row, col)
    target: np.ndarray     # bool (n, m): the object the markers select
    seed: int
    name: str


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def _disc(n, m, cy, cx, r):
    yy = np.arange(n)[:, None] + 0.5
    xx = np.arange(m)[None, :] + 0.5
    return (yy - cy) ** 2 + (xx - cx) ** 2 <= r * r


def _rect(n, m, y0, x0, hh, ww):
    yy = np.arange(n)[:, None] + 0.5
    xx = np.arange(m)[None, :] + 0.5
    return (yy >= y0) & (yy <= y0 + hh) & (xx >= x0) & (xx <= x0 + ww)


def _pick_markers(rng, mask, k, min_dist, max_dist=None):
    """k distinct cell centres of ``mask`` between ``min_dist`` and ``max_dist``
    px inside its boundary, spread out by farthest-point sampling (a user who
    clicks around the object, a few pixels inside its edge)."""
    depth = ndimage.distance_transform_edt(mask)
    band = depth >= min_dist
    if max_dist is not None:
        band &= depth <= max_dist
    if band.sum() < k:
        band = depth >= min(min_dist, depth.max())
    if band.sum() < k:
        band = mask
    idx = np.flatnonzero(band.ravel())
    m = mask.shape[1]
    pts = np.stack([idx // m + 0.5, idx % m + 0.5], axis=1)
    chosen = [int(rng.integers(len(pts)))]
    dist = np.full(len(pts), np.inf)
    while len(chosen) < min(k, len(pts)):
        dist = np.minimum(dist, ((pts - pts[chosen[-1]]) ** 2).sum(1))
        chosen.append(int(np.argmax(dist)))
    return pts[chosen].astype(np.float64)


def _box(n, lo, hi):
    """Index range [a, b) that holds every cell centre i + 0.5 in [lo, hi],
    widened by 2 cells (the overlap test dilates by one) and clipped."""
    return max(int(math.floor(lo - 0.5)) - 2, 0), min(int(math.ceil(hi - 0.5)) + 3, n)


def _shapes(rng, n, m, count, scale, margin=2, min_count=None, tries=1000):
    """Non-overlapping discs / rectangles (rejection after 1-px dilation).
    Each candidate is evaluated on its bounding box only (the same inclusion
    test at the same cell centres as on the whole grid); shapes are returned
    as full-size masks."""
    occupied = np.zeros((n, m), bool)
    boxes = []
    attempts = 0
    while len(boxes) < count and attempts < tries * count:
        attempts += 1
        if rng.random() < 0.5:
            r = rng.uniform(8, 24) * scale
            cy = rng.uniform(margin + r, n - margin - r) if n - 2 * (margin + r) > 0 else None
            cx = rng.uniform(margin + r, m - margin - r) if m - 2 * (margin + r) > 0 else None
            if cy is None or cx is None:
                continue
            i0, i1 = _box(n, cy - r, cy + r)
            j0, j1 = _box(m, cx - r, cx + r)
            yy = np.arange(i0, i1)[:, None] + 0.5
            xx = np.arange(j0, j1)[None, :] + 0.5
            mask = (yy - cy) ** 2 + (xx - cx) ** 2 <= r * r
        else:
            hh = rng.uniform(12, 40) * scale
            ww = rng.uniform(12, 40) * scale
            if n - 2 * margin - hh <= 0 or m - 2 * margin - ww <= 0:
                continue
            y0 = rng.uniform(margin, n - margin - hh)
            x0 = rng.uniform(margin, m - margin - ww)
            i0, i1 = _box(n, y0, y0 + hh)
            j0, j1 = _box(m, x0, x0 + ww)
            yy = np.arange(i0, i1)[:, None] + 0.5
            xx = np.arange(j0, j1)[None, :] + 0.5
            mask = (yy >= y0) & (yy <= y0 + hh) & (xx >= x0) & (xx <= x0 + ww)
        if mask.sum() == 0:
            continue
        if (ndimage.binary_dilation(mask) & occupied[i0:i1, j0:j1]).any():
            continue
        occupied[i0:i1, j0:j1] |= mask
        boxes.append((i0, i1, j0, j1, mask))
    if min_count is not None and len(boxes) < min_count:
        raise RuntimeError("shape placement failed")
    shapes = []
    for i0, i1, j0, j1, mask in boxes:
        full = np.zeros((n, m), bool)
        full[i0:i1, j0:j1] = mask
        shapes.append(full)
    return shapes


def shapes_instance(seed, n=128, m=128, count=3, scale=1.0, noise=0.05, markers=4,
                    name="shapes", min_count=None):
    """Discs / rectangles with intensities U[0.2, 1] on 0, Gaussian noise."""
    rng = _rng(seed)
    shapes = _shapes(rng, n, m, count, scale, min_count=min_count)
    img = np.zeros((n, m))
    for s in shapes:
        img[s] = rng.uniform(0.2, 1.0)
    img = np.clip(img + rng.normal(0.0, noise, (n, m)), 0.0, 1.0)
    target = shapes[0]
    mk = _pick_markers(rng, target, markers, 2.0, 2.0 + 2.0 * scale)
    return Instance(img.astype(np.float32), mk, target, seed, name)


def config1(seed: int) -> Instance:
    """128x128, 3 shapes, noise 0.05, 4 markers in shape 0."""
    return shapes_instance(seed, 128, 128, 3, 1.0, 0.05, 4, "c1_128", min_count=3)


def _ellipse(n, m, cy, cx, a, b, th):
    yy = np.arange(n)[:, None] + 0.5 - cy
    xx = np.arange(m)[None, :] + 0.5 - cx
    u = xx * math.cos(th) + yy * math.sin(th)
    v = -xx * math.sin(th) + yy * math.cos(th)
    return (u / a) ** 2 + (v / b) ** 2 <= 1.0


def config2(seed: int, n: int = 1024) -> Instance:
    """12 ellipses (axes 20-200 px), polynomial bias 0.1, noise 0.08, 6 markers."""
    rng = _rng(seed)
    s = n / 1024.0
    img = np.zeros((n, n))
    label = -np.ones((n, n), np.int32)
    for e in range(12):
        a = rng.uniform(20, 200) * s / 2.0
        b = rng.uniform(20, 200) * s / 2.0
        th = rng.uniform(0.0, math.pi)
        cy, cx = rng.uniform(0, n), rng.uniform(0, n)
        mask = _ellipse(n, n, cy, cx, a, b, th)
        img[mask] = rng.uniform(0.0, 1.0)
        label[mask] = e
    coef = rng.normal(0.0, 1.0, 6)
    y = np.linspace(-1, 1, n)[:, None]
    x = np.linspace(-1, 1, n)[None, :]
    p = coef[0] + coef[1] * x + coef[2] * y + coef[3] * x * x + coef[4] * x * y + coef[5] * y * y
    img = img + 0.1 * p / np.abs(p).max()
    img = np.clip(img + rng.normal(0.0, 0.08, (n, n)), 0.0, 1.0)
    areas = np.bincount(label[label >= 0].ravel(), minlength=12)
    tgt = int(np.argmax(areas))
    target = label == tgt
    mk = _pick_markers(rng, target, 6, 3.0, 3.0 + 4.0 * s)
    return Instance(img.astype(np.float32), mk, target, seed, "c2_1024")


def config3_sizes(seed: int = 3000, count: int = 64):
    """Image sides for the uneven batch: 32 * round(exp(U[ln256, ln2048]) / 32)."""
    out = []
    for k in range(count):
        rng = _rng(seed + k)
        n = 32 * int(round(math.exp(rng.uniform(math.log(256), math.log(2048))) / 32))
        m = 32 * int(round(math.exp(rng.uniform(math.log(256), math.log(2048))) / 32))
        out.append((n, m))
    return out


def config3(k: int, base_seed: int = 3000) -> Instance:
    n, m = config3_sizes(base_seed, k + 1)[k]
    inst = shapes_instance(10_000 + base_seed + k, n, m, 3, min(n, m) / 128.0, 0.05, 4,
                           f"c3_{n}x{m}", min_count=1)
    return inst


def _polygon_mask(n, m, cy, cx, verts):
    """Cell-centre inclusion in a star-shaped polygon (even-odd rule)."""
    ys, xs = verts[:, 0], verts[:, 1]
    y0, y1 = max(int(ys.min()) - 1, 0), min(int(ys.max()) + 2, n)
    x0, x1 = max(int(xs.min()) - 1, 0), min(int(xs.max()) + 2, m)
    mask = np.zeros((n, m), bool)
    if y0 >= y1 or x0 >= x1:
        return mask
    yy = np.arange(y0, y1)[:, None] + 0.5
    xx = np.arange(x0, x1)[None, :] + 0.5
    inside = np.zeros((y1 - y0, x1 - x0), bool)
    k = len(verts)
    for t in range(k):
        ay, ax = verts[t]
        by, bx = verts[(t + 1) % k]
        cond = (ay > yy) != (by > yy)
        with np.errstate(divide="ignore", invalid="ignore"):
            xint = ax + (yy - ay) * (bx - ax) / (by - ay)
        inside ^= cond & (xx < xint)
    mask[y0:y1, x0:x1] = inside
    return mask


def config4(seed: int, n: int = 8192, count: int = 200) -> Instance:
    """200 star polygons (5-12 vertices, 30-1500 px), blur 1.5, noise 0.05, 8 markers."""
    rng = _rng(seed)
    s = n / 8192.0
    img = np.zeros((n, n), np.float64)
    label = -np.ones((n, n), np.int32)
    for p in range(count):
        nv = int(rng.integers(5, 13))
        ang = np.sort(rng.uniform(0.0, 2 * math.pi, nv))
        R = math.exp(rng.uniform(math.log(30), math.log(1500))) / 2.0 * s
        rad = R * rng.uniform(0.5, 1.0, nv)
        cy, cx = rng.uniform(0, n), rng.uniform(0, n)
        verts = np.stack([cy + rad * np.sin(ang), cx + rad * np.cos(ang)], axis=1)
        mask = _polygon_mask(n, n, cy, cx, verts)
        img[mask] = rng.uniform(0.0, 1.0)
        label[mask] = p
    img = ndimage.gaussian_filter(img, 1.5, mode="reflect", truncate=4.0)
    img = np.clip(img + rng.normal(0.0, 0.05, (n, n)), 0.0, 1.0)
    areas = np.bincount(label[label >= 0].ravel(), minlength=count)
    tgt = int(np.flatnonzero(areas >= 400 * s * s)[0]) if (areas >= 400 * s * s).any() else int(np.argmax(areas))
    target = label == tgt
    mk = _pick_markers(rng, target, 8, 3.0, 3.0 + 8.0 * s)
    return Instance(img.astype(np.float32), mk, target, seed, f"c4_{n}")


def config5(seed: int, n: int = 512) -> Instance:
    """4-20 shapes (C1 rules scaled x4), noise U[0.02, 0.1], 3-8 markers."""
    rng = _rng(seed)
    count = int(rng.integers(4, 21))
    noise = float(rng.uniform(0.02, 0.1))
    k = int(rng.integers(3, 9))
    return shapes_instance(seed * 7 + 1, n, n, count, 4.0 * n / 512.0, noise, k, f"c5_{n}", min_count=4)


def config5_arrays(seed_n):
    """(image, markers, seed) of config5(seed, n) for a worker process."""
    seed, n = seed_n
    inst = config5(seed, n)
    return inst.image, inst.markers, seed


def tiny_instance(seed: int, n: int = 16, m: int = 16, markers: int = 3) -> Instance:
    """One object on a tiny grid (oracle self-consistency tests)."""
    rng = _rng(seed)
    r = rng.uniform(0.22, 0.3) * min(n, m)
    cy = rng.uniform(0.4, 0.6) * n
    cx = rng.uniform(0.4, 0.6) * m
    tgt = _disc(n, m, cy, cx, r)
    img = np.where(tgt, rng.uniform(0.6, 1.0), 0.0)
    img = np.clip(img + rng.normal(0.0, 0.02, (n, m)), 0.0, 1.0)
    mk = _pick_markers(rng, tgt, markers, 1.0, 2.0)
    return Instance(img.astype(np.float32), mk, tgt, seed, f"tiny_{n}x{m}")


def levels_for(n: int, m: int, min_side: int = 4) -> int:
    """Largest level count with n, m divisible by 2^(L-1) and min side >= min_side."""
    L = 1
    while (n % (1 << L) == 0 and m % (1 << L) == 0 and min(n, m) >> L >= min_side):
        L += 1
    return L
