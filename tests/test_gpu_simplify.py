"""GPU parity of the simplification passes (cumulative-mass cut, weighted
sampling without replacement, compaction) against the float64 reference."""
from __future__ import annotations

import numpy as np
import pytest
import torch

from tests.gpuhelp import device, gsmi, to_np, u32

pytestmark = pytest.mark.gpu


def _scores(n, seed):
    rng = np.random.default_rng(seed)
    s = rng.lognormal(0.0, 1.5, n).astype(np.float32)
    s[rng.random(n) < 0.2] = 0.0
    s[rng.random(n) < 0.02] = np.float32(1.0)   # ties
    return s


@pytest.mark.parametrize("n", [1000, 4096 + 7, 1 << 20])
def test_mass_keep_matches_reference(oracle, n):
    dev = device()
    G = gsmi()
    s = _scores(n, n)
    ref = oracle.mass_keep(s.astype(np.float64), 0.99)
    st = torch.from_numpy(s).to(dev)
    keep = torch.zeros((n + 31) // 32, dtype=torch.int32, device=dev)
    cnt = torch.zeros(1, dtype=torch.int64, device=dev)
    ws = torch.empty(G.gs_workspace_size(G.GS_OP_SIMPLIFY, n), dtype=torch.uint8, device=dev)
    G.gs_mass_keep_bits(st, n, 0.99, keep, cnt, ws)
    torch.cuda.synchronize()
    got = oracle.unpack_bits(u32(keep), n)
    assert int(cnt.item()) == int(got.sum())
    # decisions may differ only where the cumulative mass sits at the cut
    idx = np.nonzero(s > 0)[0]
    order = idx[np.lexsort((idx, -s[idx].astype(np.float64)))]
    cs = np.cumsum(s[order].astype(np.float64))
    before = cs - s[order]
    band = np.zeros(n, dtype=bool)
    band[order[np.abs(before - 0.99 * cs[-1]) <= 1e-9 * cs[-1]]] = True
    assert not ((got != ref) & ~band).any()


@pytest.mark.parametrize("n", [1000, 1 << 20])
def test_sample_keep_matches_reference(oracle, n):
    dev = device()
    G = gsmi()
    s = _scores(n, n + 1)
    rng = np.random.default_rng(5)
    u = (1.0 - rng.random(n)).astype(np.float32)
    n_keep = int(0.68 * n)
    ref = oracle.sample_keep(s.astype(np.float64), u.astype(np.float64), n_keep)
    keep = torch.zeros((n + 31) // 32, dtype=torch.int32, device=dev)
    ws = torch.empty(G.gs_workspace_size(G.GS_OP_SIMPLIFY, n), dtype=torch.uint8, device=dev)
    G.gs_sample_keep_bits(torch.from_numpy(s).to(dev), torch.from_numpy(u).to(dev), n, n_keep, keep, ws)
    torch.cuda.synchronize()
    got = oracle.unpack_bits(u32(keep), n)
    assert got.sum() == n_keep
    e = oracle.race_times(s, u)
    tau = np.sort(e, kind="stable")[n_keep - 1]
    band = np.abs(e - tau) <= 1e-5 * abs(tau) if np.isfinite(tau) else (e == tau)
    assert not ((got != ref) & ~band).any()


def test_compact_matches_reference(oracle):
    dev = device()
    G = gsmi()
    n = 100_003
    rng = np.random.default_rng(2)
    # the SH layout [16][3][n]: its leading dimensions together are the rows
    arrays = [rng.standard_normal((3, n)).astype(np.float32), rng.standard_normal((16, 3, n)).astype(np.float32),
              rng.standard_normal(n).astype(np.float32), rng.integers(0, 8, n).astype(np.uint8)]
    keep = rng.random(n) < 0.61
    n_keep = int(keep.sum())
    ref = oracle.compact(arrays, keep)
    src = [torch.from_numpy(a).to(dev) for a in arrays]
    dst = [torch.empty(*(a.shape[:-1] + (n_keep,)), dtype=t.dtype, device=dev) for a, t in zip(arrays, src)]
    kb = torch.from_numpy(oracle.pack_bits(keep).view(np.int32)).to(dev)
    ws = torch.empty(G.gs_workspace_size(G.GS_OP_SIMPLIFY, n), dtype=torch.uint8, device=dev)
    G.gs_compact(src, dst, n, n_keep, kb, ws)
    torch.cuda.synchronize()
    for r, d in zip(ref, dst):
        np.testing.assert_array_equal(to_np(d), r)


def test_compact_empty():
    """n = 0 (an empty keep array, whose pointer is null) launches nothing."""
    dev = device()
    G = gsmi()
    src = [torch.empty(3, 0, device=dev), torch.empty(16, 3, 0, device=dev), torch.empty(0, dtype=torch.uint8, device=dev)]
    dst = [torch.empty_like(t) for t in src]
    ws = torch.empty(max(G.gs_workspace_size(G.GS_OP_SIMPLIFY, 0), 256), dtype=torch.uint8, device=dev)
    G.gs_compact(src, dst, 0, 0, torch.empty(0, dtype=torch.int32, device=dev), ws)
    torch.cuda.synchronize()


@pytest.mark.parametrize("n", [1, 31, 1023, 1024, 1025, 4097])
def test_compact_edge_sizes(oracle, n):
    """Sizes around the 1,024 columns of a compaction workgroup and its
    32-column keep words, with every column kept, none kept and a random half
    (a float array of 9 rows, one of a single row and a byte array)."""
    dev = device()
    G = gsmi()
    rng = np.random.default_rng(n)
    arrays = [rng.standard_normal((9, n)).astype(np.float32), rng.standard_normal(n).astype(np.float32),
              rng.integers(0, 255, (2, n)).astype(np.uint8)]
    src = [torch.from_numpy(a).to(dev) for a in arrays]
    ws = torch.empty(G.gs_workspace_size(G.GS_OP_SIMPLIFY, n), dtype=torch.uint8, device=dev)
    for keep in (np.ones(n, dtype=bool), np.zeros(n, dtype=bool), rng.random(n) < 0.5):
        n_keep = int(keep.sum())
        ref = oracle.compact(arrays, keep)
        dst = [torch.full((*a.shape[:-1], max(n_keep, 1)), 7, dtype=t.dtype, device=dev) for a, t in zip(arrays, src)]
        kb = torch.from_numpy(oracle.pack_bits(keep).view(np.int32)).to(dev)
        G.gs_compact(src, dst, n, n_keep, kb, ws)
        torch.cuda.synchronize()
        for r, d in zip(ref, dst):
            if n_keep == 0:
                assert (to_np(d) == 7).all()  # nothing written
            else:
                np.testing.assert_array_equal(to_np(d), r)


def test_compact_large_offsets(oracle):
    """48 rows of 2^25 + 3 columns (6.4 GB): row offsets past 4 GB.  Values are
    integer bit patterns (row * 2654435761 + column, 32 bits); three windows
    of columns, the last one ragged, are compared with the reference's
    compaction of the same window in rows 0, 1, 23 and 47."""
    dev = device()
    G = gsmi()
    n, rows = (1 << 25) + 3, 48
    src = torch.empty(rows, n, dtype=torch.int32, device=dev)
    col = torch.arange(n, dtype=torch.int64, device=dev)
    for r in range(rows):
        v = (col + r * 2654435761) & 0xFFFFFFFF
        src[r] = torch.where(v >= 1 << 31, v - (1 << 32), v).to(torch.int32)
    del col, v
    rng = np.random.default_rng(5)
    words = rng.integers(0, 1 << 32, (n + 31) // 32, dtype=np.uint64).astype(np.uint32)
    keep = oracle.unpack_bits(words, n)
    n_keep = int(keep.sum())
    dst = torch.empty(rows, n_keep, dtype=torch.int32, device=dev)
    ws = torch.empty(G.gs_workspace_size(G.GS_OP_SIMPLIFY, n), dtype=torch.uint8, device=dev)
    kb = torch.from_numpy(words.view(np.int32)).to(dev)
    G.gs_compact([src.view(torch.float32)], [dst.view(torch.float32)], n, n_keep, kb, ws)
    torch.cuda.synchronize()
    before = np.concatenate([[0], np.cumsum(keep)])
    for c0, c1 in [(0, 100_000), (n // 2 - 50_000, n // 2 + 50_000), (n - 100_003, n)]:
        k0, k1 = int(before[c0]), int(before[c1])
        for r in (0, 1, 23, 47):
            window = to_np(src[r, c0:c1])
            (ref,) = oracle.compact([window], keep[c0:c1])
            np.testing.assert_array_equal(to_np(dst[r, k0:k1]), ref)

