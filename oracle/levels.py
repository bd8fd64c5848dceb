"""CPU reference (test infrastructure only) of the level structure behind the
distance-based LOD gate and of the spawn gate's rank veto.

Only tests, the smoke check and the CPU-baseline timing use this package; the
product path never imports it, and it shares no code with the HIP library.

Follows Sec. 3.3 ("Distance-based LOD gate": labels from multi-resolution
voxelisation, the clone/split inheritance rule, the coarse-to-fine ceiling
L_max(t)) and Sec. 3.2 "Spawn gate" with the veto equation of Appendix E
("Spawn gate features and veto").  The paper leaves the voxelisation, the
shape of the schedule and the spawn-time scorer to its code; the readings
taken here are stated at each function.
"""
from __future__ import annotations

import math

import numpy as np

MAX_LEVELS = 22          # 21 bits per axis of the finest cell coordinate
CELL_BITS = 21


# --------------------------------------------------------------------------
# Multi-resolution voxelisation (Sec. 3.3, first sentences of the LOD gate)
# --------------------------------------------------------------------------
def finest_cells(mean, origin, delta0: float, n_levels: int) -> np.ndarray:
    """Integer coordinates [3][N] of each point's cell at the finest level
    K-1, whose edge is delta0 / 2^(K-1).

    The decision of which cell a point falls in is taken in float32, as the
    GPU takes it: c = floor((mu - origin) * s) with s = 2^(K-1) / delta0, a
    float32 subtraction, then a float32 product, each rounded once; clamped to
    [0, 2^21 - 1]."""
    assert 1 <= n_levels <= MAX_LEVELS
    m = np.asarray(mean, dtype=np.float32)
    o = np.asarray(origin, dtype=np.float32).reshape(3, 1)
    s = np.float32(2 ** (n_levels - 1)) / np.float32(delta0)
    with np.errstate(over="ignore", invalid="ignore"):
        q = np.floor((m - o) * s)
    q = np.nan_to_num(q, nan=0.0, posinf=float(2 ** CELL_BITS - 1), neginf=0.0)
    return np.clip(q, 0, 2 ** CELL_BITS - 1).astype(np.int64)


def morton3(cells: np.ndarray) -> np.ndarray:
    """Z-order code of integer cell coordinates [3][N]: bit b of x, y and z go
    to bits 3b, 3b+1 and 3b+2.  Written bit by bit."""
    cells = np.asarray(cells, dtype=np.int64)
    code = np.zeros(cells.shape[1], dtype=np.int64)
    for b in range(CELL_BITS):
        for axis in range(3):
            code |= ((cells[axis] >> b) & 1) << (3 * b + axis)
    return code


def voxel_levels(mean, origin, delta0: float, n_levels: int) -> np.ndarray:
    """LOD label l_i in {0, ..., K-1} of every Gaussian.

    Reading of "multi-resolution voxelisation" (the paper cites octree-style
    anchors, one per occupied voxel of each level): level l partitions space
    into cubes of edge delta0 / 2^l anchored at `origin`, and each occupied
    level-l cube is represented by one of its Gaussians - the first in the
    order (Z-order code of the point's finest cell, index).  l_i is the
    coarsest level at which Gaussian i represents its cube; a Gaussian that
    represents no cube (it shares its finest cell with an earlier one) gets
    K-1.  So {i : l_i <= l} holds exactly one Gaussian per occupied level-l
    cube: keeping l_i <= L renders the scene at voxel resolution delta0/2^L.

    A level-l cube is the finest cell coordinate shifted right by K-1-l bits,
    so the cubes of consecutive levels nest exactly."""
    K = int(n_levels)
    cells = finest_cells(mean, origin, delta0, K)
    n = cells.shape[1]
    code = morton3(cells)
    idx = np.arange(n, dtype=np.int64)
    label = np.full(n, K - 1, dtype=np.int64)
    for lvl in range(K - 1, -1, -1):
        sh = K - 1 - lvl
        key = ((cells[0] >> sh) << (2 * CELL_BITS)) | ((cells[1] >> sh) << CELL_BITS) | (cells[2] >> sh)
        # representative of each cube: smallest (code, index) among its points
        order = np.lexsort((idx, code, key))
        first = np.ones(n, dtype=bool)
        first[1:] = key[order][1:] != key[order][:-1]
        reps = order[first]
        label[reps] = lvl
    return label.astype(np.uint8)


# --------------------------------------------------------------------------
# Coarse-to-fine ceiling L_max(t) (Sec. 3.3, after Eq. 2)
# --------------------------------------------------------------------------
def level_ceiling(t: int, t0: int, t1: int, n_levels: int) -> int:
    """L_max(t): the levels unlock coarse to fine at geometrically spaced
    iterations.  Reading: level k unlocks at u_k = t0 * (t1 / t0)^(k / (K-1)),
    so u_0 = t0, u_{K-1} = t1 and u_{k+1} / u_k is constant; L_max(t) is the
    largest k with u_k <= t (0 before t0, K-1 from t1 on)."""
    K = int(n_levels)
    if K <= 1 or t <= t0:
        return 0
    if t >= t1:
        return K - 1
    best = 0
    for k in range(K):
        u = t0 * (t1 / t0) ** (k / (K - 1))
        if u <= t:
            best = k
    return best


# --------------------------------------------------------------------------
# Spawn gate (Sec. 3.2 "Spawn gate"; Appendix E, the veto equation)
# --------------------------------------------------------------------------
def veto_count(n: int, rho: float) -> int:
    """|V_t| = ceil(rho |C_t|), with rho * |C_t| evaluated in double."""
    return min(n, max(0, int(math.ceil(float(rho) * n))))


def rank_veto(p, rho: float) -> np.ndarray:
    """Keep mask of one candidate set C_t: the ceil(rho |C_t|) candidates of
    lowest predicted survival p are vetoed (the subset of that size with the
    smallest sum of p); ties are broken by candidate index, the lower index
    vetoed first.  Returns True for the instantiated candidates C'_t."""
    p = np.asarray(p, dtype=np.float64)
    n = p.shape[0]
    order = np.lexsort((np.arange(n), p))
    keep = np.ones(n, dtype=bool)
    keep[order[:veto_count(n, rho)]] = False
    return keep


def stub_survival(opacity_logit, parents) -> np.ndarray:
    """Stand-in for the offline survival predictor (out of scope: it is fit on
    lineage logs of real scenes): the parent's opacity, one of the spawn-time
    features the paper lists.  The veto depends only on the ordering of the
    scores."""
    z = np.asarray(opacity_logit, dtype=np.float32)[np.asarray(parents, dtype=np.int64)]
    return (1.0 / (1.0 + np.exp(-z.astype(np.float64)))).astype(np.float32)


def child_level(parent_level, split: bool, n_levels: int):
    """Inheritance rule: a clone keeps its parent's level, a split is one level
    finer (reading: clamped at the finest level K-1)."""
    lv = np.asarray(parent_level, dtype=np.int64) + (1 if split else 0)
    return np.minimum(lv, n_levels - 1).astype(np.uint8)


def spawn_gate(lod, clone_parent, split_parent, p_clone, p_split, rho: float, n_levels: int):
    """One gated densification event.  Clones and splits are separate
    candidate sets; each is vetoed by rank.  Returns (child_parent, child_lod,
    child_split) of the instantiated candidates: the surviving clones in
    candidate order, then the surviving splits in candidate order."""
    lod = np.asarray(lod, dtype=np.int64)
    cp = np.asarray(clone_parent, dtype=np.int64)
    sp = np.asarray(split_parent, dtype=np.int64)
    kc = rank_veto(p_clone, rho)
    ks = rank_veto(p_split, rho)
    parent = np.concatenate([cp[kc], sp[ks]]).astype(np.int32)
    level = np.concatenate([child_level(lod[cp[kc]], False, n_levels),
                            child_level(lod[sp[ks]], True, n_levels)]).astype(np.uint8)
    split = np.concatenate([np.zeros(int(kc.sum()), dtype=np.uint8), np.ones(int(ks.sum()), dtype=np.uint8)])
    return parent, level, split


def reference_distance(cam_centres, mean) -> float:
    """d0 (reading): median over the training cameras of the distance from the
    camera centre to the mean of the Gaussian centres."""
    c = np.asarray(mean, dtype=np.float64).mean(axis=1)
    d = np.linalg.norm(np.asarray(cam_centres, dtype=np.float64) - c[None, :], axis=1)
    return float(np.median(d))
