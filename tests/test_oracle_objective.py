"""Pins of the reference objective (Eqs. 4-5): SSIM closed forms and a
brute-force window, the photometric gradient against finite differences,
and the scale regulariser by hand (no GPU)."""
from __future__ import annotations

import math

import numpy as np
import torch


def test_ssim_of_identical_images_is_one(oracle):
    rng = np.random.default_rng(0)
    x = rng.random((3, 20, 23))
    m = oracle.ssim_map(x, x).numpy()
    np.testing.assert_allclose(m, 1.0, atol=1e-12)


def test_ssim_constant_images_closed_form(oracle):
    """Away from the zero-padded border: mu = a, b and zero variances, so
    SSIM = (2ab + C1) / (a^2 + b^2 + C1)."""
    a, b = 0.3, 0.7
    x = np.full((3, 30, 30), a)
    y = np.full((3, 30, 30), b)
    m = oracle.ssim_map(x, y).numpy()
    expect = (2 * a * b + 0.01 ** 2) / (a * a + b * b + 0.01 ** 2)
    np.testing.assert_allclose(m[:, 5:25, 5:25], expect, rtol=1e-12)


def test_ssim_matches_bruteforce_window(oracle):
    rng = np.random.default_rng(1)
    x = rng.random((3, 17, 19))
    y = rng.random((3, 17, 19))
    m = oracle.ssim_map(x, y).numpy()
    g = oracle.ssim_window()
    w2 = np.outer(g, g)
    for (c, v, u) in [(0, 0, 0), (1, 8, 9), (2, 16, 18), (0, 3, 14)]:
        S = dict(mx=0.0, my=0.0, xx=0.0, yy=0.0, xy=0.0)
        for dv in range(-5, 6):
            for du in range(-5, 6):
                vv, uu = v + dv, u + du
                if 0 <= vv < 17 and 0 <= uu < 19:
                    k = w2[dv + 5, du + 5]
                    X, Y = x[c, vv, uu], y[c, vv, uu]
                    S["mx"] += k * X
                    S["my"] += k * Y
                    S["xx"] += k * X * X
                    S["yy"] += k * Y * Y
                    S["xy"] += k * X * Y
        sxx, syy, sxy = S["xx"] - S["mx"] ** 2, S["yy"] - S["my"] ** 2, S["xy"] - S["mx"] * S["my"]
        ref = ((2 * S["mx"] * S["my"] + 1e-4) * (2 * sxy + 9e-4)) / \
              ((S["mx"] ** 2 + S["my"] ** 2 + 1e-4) * (sxx + syy + 9e-4))
        assert m[c, v, u] == __import__("pytest").approx(ref, rel=1e-12)


def test_window_is_normalised_gaussian(oracle):
    g = oracle.ssim_window()
    assert g.shape == (11,) and abs(g.sum() - 1) < 1e-15
    assert g[5] / g[6] == __import__("pytest").approx(math.exp(1 / (2 * 1.5 ** 2)), rel=1e-12)


def test_photo_loss_gradient_finite_differences(oracle):
    rng = np.random.default_rng(2)
    x = rng.random((3, 14, 16))
    y = rng.random((3, 14, 16))
    L, g = oracle.photo_loss(x, y, 0.2)
    assert L == __import__("pytest").approx(0.8 * np.abs(x - y).mean() + 0.2 * (1 - oracle.ssim_map(x, y).mean().item()))
    for (c, v, u) in [(0, 0, 0), (1, 7, 8), (2, 13, 15), (1, 2, 11)]:
        h = 1e-6
        xp, xm = x.copy(), x.copy()
        xp[c, v, u] += h
        xm[c, v, u] -= h
        fd = (oracle.photo_loss(xp, y)[0] - oracle.photo_loss(xm, y)[0]) / (2 * h)
        assert abs(fd - g[c, v, u]) <= 1e-8 + 1e-6 * abs(g[c, v, u])


def test_scale_reg_by_hand(oracle):
    ls = np.log(np.array([[1.0, 0.5, 2.0], [0.2, 0.5, 3.0], [0.3, 0.9, 0.1]]))   # [3][N=3]
    vis = np.array([True, True, False])
    L, g = oracle.scale_reg(ls, vis, beta=10.0)
    assert L == __import__("pytest").approx(10.0 * (0.2 + 0.5) / 2)
    # gradient w.r.t. the log of the smallest axis: beta * s / |V|
    expect = np.zeros((3, 3))
    expect[1, 0] = 10 * 0.2 / 2
    expect[0, 1] = 10 * 0.5 / 2           # tie between axes 0 and 1: the first wins
    np.testing.assert_allclose(g, expect, rtol=1e-12)
    assert oracle.scale_reg(ls, np.zeros(3, dtype=bool))[0] == 0.0
