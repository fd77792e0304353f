"""The pair list and origins built on the GPU (Step II, Step III) against the
oracle's plain double loop, bit for bit, and the Alg. 1 owner assignment
against the oracle's, through the C ABI.

Cases: the small, 64-water and 512-water workloads; 16,384 random centres
(the regime where a host O(N^2) search stops being free); centres outside
the cell; a distance exactly at the cutoff and half-way midpoints; cells too
small for three cells per axis.
"""
import sys
import time

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from oracle import oracle as O  # noqa: E402
from paper_1911_10630_amd import exx as X  # noqa: E402
from paper_1911_10630_amd import synth as S  # noqa: E402


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _oracle_pairs(C, cell, r_pair, n_grid):
    pi, pj = O.pair_list(C, cell, r_pair)
    org = np.array([O.pair_origin(C[i], C[j], cell, n_grid) for i, j in zip(pi, pj)], np.int32).reshape(-1, 3)
    return pi, pj, org


def _check(ctx, C, cell, r_pair, n_grid, owners=True):
    t0 = time.perf_counter()
    n = ctx.pairs(C)
    t_gpu = time.perf_counter() - t0
    info = ctx.pair_info(results=False)
    t0 = time.perf_counter()
    pi, pj, org = _oracle_pairs(C, cell, r_pair, n_grid)
    t_ref = time.perf_counter() - t0
    assert n == len(pi)
    assert np.array_equal(info["i"], pi) and np.array_equal(info["j"], pj)
    assert np.array_equal(info["origin"], org)
    if owners:
        own, sweeps = ctx.pair_owners()
        ref_own, ref_sweeps = O.unique_pair_owners(C, cell, r_pair)
        assert sweeps == ref_sweeps
        assert np.array_equal(own, ref_own)
    return n, t_gpu, t_ref


def _tiny_ctx(cell, r_pair, n_grid=(48, 48, 48)):
    """A context whose subdomains are small: only the pair list matters."""
    h = max(c / n for c, n in zip(cell, n_grid))
    return X.Exx(n_grid, cell, r_pair, 3.0 * h, 6.2 * h, autotune=False)


@pytest.mark.parametrize("name", ["c1", "c2", "c5"])
def test_workload_pairs_and_owners(name):
    wl = S.WORKLOADS[name]()
    _say(f"[gpu] pair list of {wl.name}")
    ctx = X.Exx.from_workload(wl, autotune=False)
    n, t_gpu, t_ref = _check(ctx, wl.orbitals.centers, wl.cell, wl.r_pair, wl.n_grid)
    _say(f"[gpu] {n} pairs: exx_pairs {t_gpu * 1e3:.1f} ms")
    ctx.close()


def test_random_16k_centres():
    rng = np.random.default_rng(2024)
    cell = (120.0, 110.0, 130.0)
    C = rng.uniform(0.0, 1.0, size=(16384, 3)) * np.array(cell)
    ctx = _tiny_ctx(cell, 6.0, (64, 64, 64))
    n, t_gpu, t_ref = _check(ctx, C, cell, 6.0, (64, 64, 64), owners=False)
    _say(f"[gpu] 16,384 centres, {n} pairs: exx_pairs {t_gpu * 1e3:.1f} ms (with the per-pair set-up), "
         f"oracle double loop + origins {t_ref * 1e3:.0f} ms")
    assert n > 80000                                  # about 8.6 partners per centre
    ctx.close()


def test_centres_outside_the_cell():
    rng = np.random.default_rng(7)
    cell = (20.0, 20.0, 20.0)
    C = rng.uniform(-30.0, 50.0, size=(300, 3))
    ctx = _tiny_ctx(cell, 4.0)
    _check(ctx, C, cell, 4.0, (48, 48, 48))
    ctx.close()


def test_cutoff_is_strict_and_half_way_midpoints_round_away():
    cell = (24.0, 24.0, 24.0)                         # h = 0.5 on 48 points
    C = np.array([[0.0, 0.0, 0.0],
                  [3.0, 0.0, 0.0],                    # exactly R_pair from 0: not a pair
                  [0.25, 2.5, 0.0],                   # midpoint with 0 at x = 0.125, y = 1.25: half-way
                  [23.75, 0.0, 0.0],                  # across the boundary from 0: midpoint -0.125
                  [12.0, 12.0, 12.0],
                  [12.0, 12.0, 14.999999999999998]], float)
    ctx = _tiny_ctx(cell, 3.0)
    n, *_ = _check(ctx, C, cell, 3.0, (48, 48, 48))
    info = ctx.pair_info(results=False)
    got = set(zip(info["i"].tolist(), info["j"].tolist()))
    assert (0, 1) not in got and (4, 5) in got and (0, 3) in got
    ctx.close()


@pytest.mark.parametrize("ratio", [1.5, 2.5, 3.0])
def test_cells_too_small_for_three_bins(ratio):
    """L / R_pair of 1.5 and 2.5 give one and two cells per axis (every cell
    is a neighbour, scanned once); 3.0 sits on the edge of three."""
    rng = np.random.default_rng(int(ratio * 10))
    r_pair = 4.0
    cell = (ratio * r_pair,) * 3
    C = rng.uniform(0.0, cell[0], size=(120, 3))
    ctx = _tiny_ctx(cell, r_pair, (32, 32, 32))
    _check(ctx, C, cell, r_pair, (32, 32, 32))
    ctx.close()


def test_sparse_centres_in_a_large_cell():
    """Few centres in a cell of many R_pair: the cell list is coarsened to a
    few cells per centre, the pairs stay exact."""
    rng = np.random.default_rng(99)
    cell = (400.0, 380.0, 420.0)
    C = rng.uniform(0.0, 1.0, size=(40, 3)) * np.array(cell)
    C[1] = C[0] + np.array([1.5, -0.5, 0.25])                 # a few close pairs
    C[2] = C[0] + np.array([-2.0, 1.0, 0.0])
    ctx = _tiny_ctx(cell, 3.0, (64, 64, 64))
    n, *_ = _check(ctx, C, cell, 3.0, (64, 64, 64))
    assert n >= 40 + 2                                  # 0-1 and 0-2; 1-2 is 3.8 bohr apart
    ctx.close()
