"""Pins of the CPU reference's LOD levels, L_max(t) schedule and spawn-gate
veto (Sec. 3.3 LOD gate; Sec. 3.2 spawn gate and the veto equation of
Appendix E), against hand-derived values, brute force over the definitions
and exact invariants.  No GPU.

Each pin is a function of the reference module, so that
`test_oracle_mutations.py` can run it against copies with planted mistakes.
"""
from __future__ import annotations

import itertools
import os

import numpy as np

from oracle import levels as LV

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _fixture(name):
    out = {}
    for line in open(os.path.join(GOLDEN, name)):
        line = line.split("#", 1)[0].strip()
        if "=" in line:
            k, v = (s.strip() for s in line.split("=", 1))
            out[k] = v
    return out


def _lattice_points(rng, n, n_levels, delta0, origin, span_cells):
    """Points at the centres of random finest cells (exact in float32 and
    float64: delta0 is a power of two)."""
    fine = delta0 / 2 ** (n_levels - 1)
    cells = rng.integers(0, span_cells, size=(3, n))
    return (np.asarray(origin, dtype=np.float64)[:, None] + (cells + 0.5) * fine).astype(np.float32)


# ---------------------------------------------------------------- voxel labels
def pin_hand_example(L):
    f = _fixture("voxel_levels.txt")
    mean = np.array([[float(v) for v in f[a].split()] for a in ("x", "y", "z")], dtype=np.float32)
    origin = [float(v) for v in f["origin"].split()]
    got = L.voxel_levels(mean, origin, float(f["delta0"]), int(f["n_levels"]))
    want = np.array([int(v) for v in f["levels"].split()])
    assert np.array_equal(got.astype(np.int64), want), (got, want)


def pin_one_per_occupied_cube(L):
    """For every level l < K-1, {i : l_i <= l} holds exactly one Gaussian per
    occupied level-l cube, the cubes computed independently in float64 by
    division by the edge.  (At the finest level the label K-1 also goes to
    the points that represent no cube.)"""
    rng = np.random.default_rng(3)
    for K, delta0, span in ((4, 8.0, 8), (6, 32.0, 40), (8, 1.0, 300)):
        origin = (-3.0, 5.0, 0.25)
        mean = _lattice_points(rng, 3000, K, delta0, origin, span)
        lab = L.voxel_levels(mean, origin, delta0, K).astype(np.int64)
        assert lab.min() >= 0 and lab.max() <= K - 1
        for lvl in range(K - 1):
            edge = delta0 / 2 ** lvl
            cube = np.floor((mean.astype(np.float64) - np.asarray(origin)[:, None]) / edge).astype(np.int64)
            occupied = {tuple(c) for c in cube.T}
            chosen = [tuple(c) for c in cube[:, lab <= lvl].T]
            assert len(chosen) == len(set(chosen)) == len(occupied), (K, lvl, len(chosen), len(occupied))


def _interleave_by_strings(cell):
    """Z-order code of one cell by interleaving binary strings (an
    independent construction)."""
    bx, by, bz = (format(int(c), "021b") for c in cell)
    s = "".join(z + y + x for x, y, z in zip(bx, by, bz))  # most significant first
    return int(s, 2)


def pin_brute_force_pairwise(L):
    """Tiny inputs: l_i = the smallest level at which no other point of i's
    cube precedes i in (Z-order code, index), by pairwise comparison."""
    rng = np.random.default_rng(7)
    K, delta0, origin = 4, 4.0, (0.0, 0.0, 0.0)
    for trial in range(4):
        n = 48
        mean = _lattice_points(rng, n, K, delta0, origin, 6 if trial % 2 else 3)
        fine = delta0 / 2 ** (K - 1)
        cells = np.floor(mean.astype(np.float64) / fine).astype(np.int64)
        code = [_interleave_by_strings(cells[:, i]) for i in range(n)]
        want = []
        for i in range(n):
            lab = K - 1
            for lvl in range(K):
                sh = K - 1 - lvl
                ci = tuple(cells[:, i] >> sh)
                beaten = any(tuple(cells[:, j] >> sh) == ci and (code[j], j) < (code[i], i)
                             for j in range(n) if j != i)
                if not beaten:
                    lab = lvl
                    break
            want.append(lab)
        got = L.voxel_levels(mean, origin, delta0, K).astype(np.int64)
        assert np.array_equal(got, np.array(want)), trial


def pin_cell_decision_in_float32(L):
    """The cell of a point is floor((mu - o) * s) taken in float32: a point a
    float32 rounding below a cell boundary lands in the lower cell, one at the
    boundary in the upper."""
    K, delta0 = 2, 2.0                       # finest edge 1
    below = np.float32(np.nextafter(np.float32(1.0), np.float32(0.0)))
    mean = np.array([[below, 1.0], [0.0, 0.0], [0.0, 0.0]], dtype=np.float32)
    cells = L.finest_cells(mean, (0.0, 0.0, 0.0), delta0, K)
    assert cells[0].tolist() == [0, 1]
    # both points share the level-0 cube; the one in cell 0 comes first in
    # Z-order, so it holds level 0 and the other level 1
    assert L.voxel_levels(mean, (0.0, 0.0, 0.0), delta0, K).tolist() == [0, 1]
    # 1 - 2^-25 is 0.99999997 in float64 but rounds to 1 in float32 (a tie,
    # to even): the float32 subtraction puts the point in cell 1
    o = (2.0 ** -25, 0.0, 0.0)
    one = np.array([[1.0], [0.0], [0.0]], dtype=np.float32)
    assert L.finest_cells(one, o, delta0, K)[0].tolist() == [1]


def pin_morton_bits(L):
    cells = np.array([[1, 0, 0, 3, 2, (1 << 20)], [0, 1, 0, 0, 2, 0], [0, 0, 1, 0, 0, 1]])
    want = [1, 2, 4, 9, 24, (1 << 60) | 4]
    assert L.morton3(cells).tolist() == want


# ---------------------------------------------------------------- L_max(t)
def pin_ceiling_hand_values(L):
    # t0 = 2k, t1 = 32k, K = 5: levels unlock at 2k, 4k, 8k, 16k, 32k
    want = {0: 0, 1999: 0, 2000: 0, 3999: 0, 4000: 1, 7999: 1, 8000: 2, 15999: 2, 16000: 3, 31999: 3,
            32000: 4, 90000: 4}
    for t, lv in want.items():
        assert L.level_ceiling(t, 2000, 32000, 5) == lv, (t, L.level_ceiling(t, 2000, 32000, 5), lv)
    # geometric spacing: unlock times of K = 8 between 1k and 128k are powers of two
    prev = -1
    for t in range(0, 140_000, 250):
        lv = L.level_ceiling(t, 1000, 128_000, 8)
        assert lv >= prev
        prev = lv
        assert lv == (0 if t < 2000 else min(7, int(np.floor(np.log2(t / 1000) + 1e-12))))
    assert L.level_ceiling(10, 5, 50, 1) == 0


# ---------------------------------------------------------------- spawn gate
def pin_veto_count(L):
    for n in range(0, 400):
        assert L.veto_count(n, 0.6) == (3 * n + 4) // 5, n      # ceil(3n/5) exactly
        assert L.veto_count(n, 0.0) == 0
        assert L.veto_count(n, 1.0) == n


def pin_rank_veto_brute_force(L):
    """The vetoed set is the subset of size ceil(rho |C|) with the smallest
    summed survival (Appendix E veto equation), found by enumeration."""
    rng = np.random.default_rng(5)
    for n in range(0, 11):
        p = rng.random(n).astype(np.float32)
        keep = L.rank_veto(p, 0.6)
        v = L.veto_count(n, 0.6)
        best = min(itertools.combinations(range(n), v), key=lambda s: sum(float(p[j]) for j in s)) if n else ()
        assert sorted(np.nonzero(~keep)[0].tolist()) == sorted(best), (n, p)
    # ties: equal scores vetoed lowest index first
    keep = L.rank_veto(np.array([0.5, 0.2, 0.5, 0.5, 0.9], dtype=np.float32), 0.6)
    assert keep.tolist() == [False, False, False, True, True]


def pin_child_levels(L):
    lod = np.array([0, 3, 7, 2], dtype=np.uint8)
    parent, level, split = L.spawn_gate(lod, clone_parent=[0, 1, 2, 3, 1], split_parent=[2, 1, 0, 3],
                                        p_clone=[0.9, 0.1, 0.8, 0.7, 0.2], p_split=[0.3, 0.9, 0.4, 0.1],
                                        rho=0.6, n_levels=8)
    # clones: veto ceil(3) lowest -> candidates 1 (0.1), 4 (0.2), 3 (0.7) -> keep 0, 2
    # splits: veto ceil(2.4) = 3 lowest -> candidates 3, 0, 2 -> keep 1
    assert parent.tolist() == [0, 2, 1]
    assert level.tolist() == [0, 7, 4]        # clone keeps, split +1 (7 clamps at K-1 = 7)
    assert split.tolist() == [0, 0, 1]
    assert L.child_level(np.array([7, 6]), True, 8).tolist() == [7, 7]
    assert L.child_level(np.array([7, 6]), False, 8).tolist() == [7, 6]


def pin_stub_survival(L):
    p = L.stub_survival(np.array([0.0, 2.0, -1.0], dtype=np.float32), [2, 0, 1, 1])
    want = [1 / (1 + np.e), 0.5, 1 / (1 + np.exp(-2.0)), 1 / (1 + np.exp(-2.0))]
    assert np.allclose(p, want, rtol=1e-6)


def pin_reference_distance(L):
    mean = np.array([[-1.0, 1.0], [0.0, 0.0], [0.0, 0.0]])
    cams = np.array([[3.0, 0, 0], [0, 4.0, 0], [0, 0, 10.0]])
    assert L.reference_distance(cams, mean) == 4.0


PINS = [pin_hand_example, pin_one_per_occupied_cube, pin_brute_force_pairwise, pin_cell_decision_in_float32,
        pin_morton_bits, pin_ceiling_hand_values, pin_veto_count, pin_rank_veto_brute_force, pin_child_levels,
        pin_stub_survival, pin_reference_distance]


def test_hand_example():
    pin_hand_example(LV)


def test_one_per_occupied_cube():
    pin_one_per_occupied_cube(LV)


def test_brute_force_pairwise():
    pin_brute_force_pairwise(LV)


def test_cell_decision_in_float32():
    pin_cell_decision_in_float32(LV)


def test_morton_bits():
    pin_morton_bits(LV)


def test_ceiling_hand_values():
    pin_ceiling_hand_values(LV)


def test_veto_count():
    pin_veto_count(LV)


def test_rank_veto_brute_force():
    pin_rank_veto_brute_force(LV)


def test_child_levels():
    pin_child_levels(LV)


def test_stub_survival():
    pin_stub_survival(LV)


def test_reference_distance():
    pin_reference_distance(LV)
