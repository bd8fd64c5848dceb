"""Brute-force references for tiny inputs, written independently of `oracle/`.

No tiles lists, no sort kernels: every pixel gathers the Gaussians whose tile
rectangle contains the pixel's tile, orders them by (float32 depth, index) with
Python's `sorted`, and composites them front to back (Appendix A, Eq.
`alpha_compositing`).  Plain Python loops; only for a few thousand pixels.
"""
from __future__ import annotations

import math

import numpy as np

TILE = 16


def rect(mx, my, r, width, height):
    TX = -(-width // TILE)
    TY = -(-height // TILE)
    xi, yi = math.floor(mx), math.floor(my)
    cl = lambda v, hi: max(0, min(hi, v))  # noqa: E731
    return (cl((xi - r) // TILE, TX), cl((xi + r) // TILE + 1, TX),
            cl((yi - r) // TILE, TY), cl((yi + r) // TILE + 1, TY))


def pairs(pr, width, height):
    """(key, value) pairs in emission order and sorted order, Python only."""
    TX = -(-width // TILE)
    emitted = []
    for i in range(pr.n):
        r = int(pr.radius[i])
        if r <= 0:
            continue
        x0, x1, y0, y1 = rect(pr.mean2d[0, i], pr.mean2d[1, i], r, width, height)
        dbits = int(np.float32(pr.depth[i]).view(np.uint32))
        for ty in range(y0, y1):
            for tx in range(x0, x1):
                emitted.append(((ty * TX + tx) << 32 | dbits, i))
    ordered = sorted(enumerate(emitted), key=lambda e: (e[1][0], e[0]))
    return emitted, [e[1] for e in ordered]


def render(pr, width, height, bg=(0.0, 0.0, 0.0), colour=True):
    """Per-pixel brute-force compositing.  Returns (img [3][H][W], T [H][W],
    w [n], a [n]) where w, a are the importance accumulators."""
    img = np.zeros((3, height, width))
    Tf = np.zeros((height, width))
    w = np.zeros(pr.n)
    a = np.zeros(pr.n, dtype=np.int64)
    rects = {}
    for i in range(pr.n):
        r = int(pr.radius[i])
        if r > 0:
            rects[i] = rect(pr.mean2d[0, i], pr.mean2d[1, i], r, width, height)
    for v in range(height):
        for u in range(width):
            tx, ty = u // TILE, v // TILE
            cand = [i for i, (x0, x1, y0, y1) in rects.items() if x0 <= tx < x1 and y0 <= ty < y1]
            cand.sort(key=lambda i: (float(np.float32(pr.depth[i])), i))
            T = 1.0
            C = [0.0, 0.0, 0.0]
            for i in cand:
                dx = pr.mean2d[0, i] - (u + 0.5)
                dy = pr.mean2d[1, i] - (v + 0.5)
                ca, cb, cc = pr.conic[0, i], pr.conic[1, i], pr.conic[2, i]
                power = -0.5 * (ca * dx * dx + cc * dy * dy) - cb * dx * dy
                if power > 0:
                    continue
                alpha = min(0.99, pr.opacity[i] * math.exp(power))
                if alpha < 1.0 / 255.0:
                    continue
                Tn = T * (1.0 - alpha)
                if Tn < 1e-4:
                    break
                for c in range(3):
                    C[c] += pr.rgb[c, i] * alpha * T
                w[i] += alpha * T
                a[i] += 1
                T = Tn
            for c in range(3):
                img[c, v, u] = C[c] + T * bg[c]
            Tf[v, u] = T
    return img, Tf, w, a
