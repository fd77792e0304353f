"""Orbitals and D on local boxes, and D summed wave by wave, through the C ABI.

The oracle sees the same orbitals placed into zero grids (the box values
are the orbital; it is zero outside its box), so E and D compare element by
element: E to 1e-8 relative, D on every box to gamma <= 1e-7, and the
oracle's D is exactly zero outside the boxes (every ME sphere lies inside
the boxes of its two orbitals, which exx_pairs checks).
"""
import sys

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


def gamma(D_ref, D):
    num = np.abs(D_ref - D).reshape(D.shape[0], -1).sum(axis=1)
    return num / np.abs(D_ref).reshape(D.shape[0], -1).sum(axis=1)


@pytest.fixture(scope="module")
def boxed():
    wl = S.c1_boxed()
    ctx = X.Exx.from_workload(wl)
    n = ctx.pairs(wl.orbitals.centers)
    org = ctx.box_origins()
    phi_box = S.orbitals_np(wl, origins=org)
    phi_full = S.embed_boxes(phi_box, org, wl.n_grid)
    E, D, out = O.exx(wl.n_grid, wl.cell, wl.r_pair, wl.r_pe, wl.r_me, wl.orbitals.centers, phi_full)
    return wl, ctx, n, org, phi_box, E, D, out


def test_box_origins_follow_the_centres(boxed):
    wl, ctx, n, org, *_ = boxed
    h = np.array(wl.h)
    C = np.mod(wl.orbitals.centers, np.array(wl.cell))
    near = np.floor(C / h + 0.5).astype(int)            # centres are never at a half-way point here
    want = np.mod(near - np.array(wl.box) // 2, np.array(wl.n_grid))
    assert np.array_equal(org, want)


def test_boxed_solve_matches_the_oracle(boxed):
    wl, ctx, n, org, phi_box, E, D, out = boxed
    _say(f"[gpu] boxed: {n} pairs, box {wl.box}")
    assert n == len(out["e"])
    Eg, Dg = ctx.step(torch.from_numpy(phi_box).cuda())
    assert Dg.shape == (16, 76, 76, 76)
    assert abs(Eg - E) <= 1e-8 * abs(E), (Eg, E)
    D_box = S.extract_boxes(D, org, wl.box)
    assert gamma(D_box, Dg.cpu().numpy()).max() <= 1e-7
    # nothing of the oracle's D lies outside the boxes
    outside = D.copy()
    for k in range(D.shape[0]):
        outside[k] -= S.embed_boxes(D_box[k:k + 1], org[k:k + 1], wl.n_grid)[0]
    assert np.abs(outside).max() == 0.0


def test_waves_sum_D_bitwise(boxed):
    """Pairs in waves of 5: D is summed wave by wave into FP64 partial sums
    and equals the one-wave result bit for bit; E too."""
    wl, ctx, n, org, phi_box, *_ = boxed
    phit = torch.from_numpy(phi_box).cuda()
    # the same kernel variant as the fixture's context (the variant fixes the
    # reduction order; the autotuner may choose differently per context)
    E1, D1 = ctx.step(phit)
    w = X.Exx.from_workload(wl, wave_pairs=5, block_threads=ctx.stats()["solve_block"],
                            cg_cols=ctx.stats()["cg_cols"])
    w.pairs(wl.orbitals.centers)
    E2, D2 = w.step(phit)
    assert w.stats()["n_waves"] == (n + 4) // 5
    assert E2 == E1 and torch.equal(D2, D1)
    # potentials of earlier waves are released
    st = w.stats()
    with pytest.raises(X.ExxError) as ei:
        w.debug_pair(0, st["n_pe"][0], st["n_me"][0] - st["n_pe"][0])
    assert ei.value.status == X.EXX_ESTATE


def test_box_too_small_is_rejected(boxed):
    wl, *_ = boxed
    ctx = X.Exx.from_workload(wl, box=(60, 60, 60))
    with pytest.raises(X.ExxError) as ei:
        ctx.pairs(wl.orbitals.centers)
    assert ei.value.status == X.EXX_EINVAL and "box_dims" in str(ei.value)


def test_history_guess_across_waves():
    """The previous-step guess saved and read wave by wave: a re-solve of the
    same step converges to the same energy in fewer iterations."""
    wl = S.c1_small()
    phit = torch.from_numpy(S.orbitals_np(wl)).cuda()
    ctx = X.Exx.from_workload(wl, guess="previous", wave_pairs=7)
    ctx.pairs(wl.orbitals.centers)
    E1, _ = ctx.step(phit)
    it1 = ctx.pair_info()["iters"].mean()
    E2, _ = ctx.step(phit)
    it2 = ctx.pair_info()["iters"].mean()
    assert ctx.stats()["n_waves"] == 9
    assert abs(E2 - E1) <= 1e-10 * abs(E1)
    assert it2 < 0.5 * it1, (it1, it2)
