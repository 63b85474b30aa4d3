"""GPU parity on the branches that ordinary inputs never reach.

Every case here is legal under the C ABI (k_max <= 100, r_c <= L, any
positions), and each asserts, through the plan's debug counters, that the
branch it is meant for really ran:

* k_max = 64, 84, 100: the vector-ALU structure factor (k_max > 47), fewer
  rows per phase-table block (tables longer than 64 entries), and in FP64
  the vector-ALU force gather (k_max > 83);
* r_c = L: the largest cutoff the ABI takes (many images per pair);
* a dense cluster in a dilute box: one cell with more than 2048 particles
  (the cell sort's global-memory path) and particles with more neighbours
  than the neighbour-list capacity (the direct loop).

Where no list overflows, the number of ordered pairs inside r_c that the
neighbour lists hold is an integer and is compared exactly with a
brute-force count over every image.

Bars are those of the other parity tests: relative norms and per-element
maxima against the FP64 oracle.
"""
import numpy as np
import pytest

import oracle
from paper_1708_01135_amd import workloads as wl

from gpu_helpers import compare

pytestmark = pytest.mark.gpu

PRECISIONS = ["fp64", "mixed"]


def brute_force_pairs(pos, L, rc):
    """Ordered pairs (i, j, image s) with |r_i - r_j - s| < r_c, i != j or s != 0,
    for positions in [0, L)^3 and r_c <= L (so |s_a| <= L per axis).  The
    displacement is formed as the kernel forms it, x_i - (x_j + s).  For
    r_c <= L/2 only the nearest image per axis can be inside r_c."""
    x = np.asarray(pos, dtype=np.float64)
    rc2 = rc * rc
    n = len(x)
    total = 0
    for i0 in range(0, n, 256):
        xi = x[i0:i0 + 256, None, :]
        idx = np.arange(i0, min(i0 + 256, n))
        if rc <= 0.5 * L:
            raw = xi - x[None, :, :]
            shifts = [np.where(raw > 0.5 * L, L, np.where(raw < -0.5 * L, -L, 0.0))]
        else:
            shifts = [np.broadcast_to(np.array([sx, sy, sz]), (len(idx), n, 3))
                      for sx in (-L, 0.0, L) for sy in (-L, 0.0, L) for sz in (-L, 0.0, L)]
        for sh in shifts:
            d = xi - (x[None, :, :] + sh)
            r2 = (d[..., 0] * d[..., 0] + d[..., 1] * d[..., 1]) + d[..., 2] * d[..., 2]
            hit = r2 < rc2
            zero = np.all(sh[np.arange(len(idx)), idx] == 0.0, axis=-1)
            hit[np.arange(len(idx))[zero], idx[zero]] = False
            total += int(hit.sum())
    return total


def run_with_stats(pos, q, L, a, rc, K, precision):
    import torch
    from paper_1708_01135_amd import ewald as ew
    dev = torch.device("cuda:0")
    tp = torch.tensor(pos, dtype=torch.float64, device=dev)
    tq = torch.tensor(q, dtype=torch.float64, device=dev)
    with ew.Plan(len(q), L, a, rc, K, precision) as p:
        e, f, g = p.energy_forces(tp, tq, True, True)
        torch.cuda.synchronize()
        st = p.status()
        stats = p.debug_stats(len(q))
        out = (e.cpu().numpy(), f.cpu().numpy(), g.cpu().numpy(), st)
    print(f"stats {precision} K={K}: {stats}", flush=True)
    return out, stats


@pytest.mark.parametrize("precision", PRECISIONS)
@pytest.mark.parametrize("K", [64, 84, 100])
def test_large_k_max(K, precision):
    n, L, a, rc = 150, 10.0, 1.0, 3.0
    pos, q = wl.random_neutral(n, L, seed=K)
    got, stats = run_with_stats(pos, q, L, a, rc, K, precision)
    compare(got, oracle.energy_forces(pos, q, L, a, rc, K, oracle.FAST), precision, f"k_max={K}")
    assert stats["sk_matrix_cores"] == 0            # k_max > 47: vector-ALU structure factor
    assert stats["phase_rows"] < 64                  # tables longer than 64 entries
    if precision == "fp64" and K > 83:
        assert stats["gather_matrix_cores"] == 0     # z powers above 64 KB of LDS
    elif precision == "mixed":
        assert stats["gather_matrix_cores"] == 1


@pytest.mark.parametrize("precision", PRECISIONS)
def test_cutoff_equal_to_box(precision):
    n, L, a, K = 240, 6.0, 1.2, 8
    pos, q = wl.random_neutral(n, L, seed=77)
    got, stats = run_with_stats(pos, q, L, a, L, K, precision)
    compare(got, oracle.energy_forces(pos, q, L, a, L, K, oracle.FAST), precision, "r_c=L")
    assert stats["cells_per_axis"] == 2
    assert stats["direct_particles"] == 0
    assert stats["listed_pairs"] == brute_force_pairs(pos, L, L)


@pytest.mark.parametrize("precision", PRECISIONS)
def test_dense_cluster_fallbacks(precision):
    # 3000 ions in a 1.6^3 cube inside one cell (h = 1.75), 3000 more spread
    # over the 14^3 box: the cluster's cell holds > 2048 particles and its ions
    # have about 50x the neighbours the plan's mean density predicts.
    L, a, rc, K = 14.0, 1.0, 3.5, 10
    pos, q = wl.clustered(3000, 3000, L, (0.05, 0.05, 0.05), 1.6, seed=11)
    got, stats = run_with_stats(pos, q, L, a, rc, K, precision)
    compare(got, oracle.energy_forces(pos, q, L, a, rc, K, oracle.FAST), precision, "cluster")
    assert stats["max_cell_count"] > 2048
    assert stats["direct_particles"] >= 3000


@pytest.mark.parametrize("precision", PRECISIONS)
def test_crowded_cell_sorted_in_lds(precision):
    # 1200 ions in a 1.2^3 cube inside one cell: between the directly ranked
    # cell sizes and the global-memory sort, the cell's indices are sorted in
    # LDS; the order (and so every sum) must not depend on the scatter's races
    L, a, rc, K = 14.0, 1.0, 3.5, 10
    pos, q = wl.clustered(1200, 2000, L, (0.3, 0.3, 0.3), 1.2, seed=12)
    got, stats = run_with_stats(pos, q, L, a, rc, K, precision)
    compare(got, oracle.energy_forces(pos, q, L, a, rc, K, oracle.FAST), precision, "crowded cell")
    assert 256 < stats["max_cell_count"] <= 2048
    again, _ = run_with_stats(pos, q, L, a, rc, K, precision)
    for x, y in zip(got, again):
        assert np.array_equal(np.asarray(x), np.asarray(y))


@pytest.mark.parametrize("precision", PRECISIONS)
@pytest.mark.parametrize("n, L", [(240, 9.0), (900, 12.0), (2000, 15.0), (3800, 18.0)])
def test_small_system_list_splits_find_every_pair(n, L, precision):
    # from a few hundred to a few thousand ions the list pass spreads each work
    # item's home particles over 8, 4 or 2 waves: the lists must still hold
    # every pair inside r_c exactly once, and the results match the oracle
    a, rc, K = 0.8, 4.0, 10
    pos, q = wl.random_neutral(n, L, seed=n)
    got, stats = run_with_stats(pos, q, L, a, rc, K, precision)
    compare(got, oracle.energy_forces(pos, q, L, a, rc, K, oracle.FAST), precision, f"n={n}")
    assert stats["direct_particles"] == 0
    assert stats["listed_pairs"] == brute_force_pairs(pos, L, rc)
