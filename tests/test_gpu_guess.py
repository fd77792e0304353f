"""Initial guesses from earlier steps (polynomial extrapolation of the pair
potentials, Sec. III.C Step IV) on a short synthetic MD trajectory of the
small configuration.  Every step must match the FP64 oracle exactly as a
zero-guess solve does; the guess only changes the iteration count."""
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


def _gamma(D_ref, D):
    return (np.abs(D_ref - D).reshape(D.shape[0], -1).sum(1) / np.abs(D_ref).reshape(D.shape[0], -1).sum(1)).max()


def test_resolve_same_step_needs_no_iterations():
    wl = S.c1_small()
    phi = torch.from_numpy(S.orbitals_np(wl)).cuda()
    ctx = X.Exx.from_workload(wl, guess="previous")
    ctx.pairs(wl.orbitals.centers)
    E1, _ = ctx.step(phi)
    it1 = ctx.pair_info()["iters"]
    ctx.pairs(wl.orbitals.centers)
    E2, _ = ctx.step(phi)
    info = ctx.pair_info()
    assert np.all(it1 > 100)
    # the history is kept in FP32: the restarted residual is ~1e-5 relative,
    # so a few decades of CG remain (against ~160 iterations from zero)
    assert np.all(info["iters"] <= 0.25 * it1) and np.all(info["converged"] == 1)
    assert abs(E2 - E1) <= 1e-10 * abs(E1)


@pytest.mark.parametrize("precision", ["fp64", "fp32_refine"])
def test_md_trajectory_matches_oracle(precision):
    wl = S.c1_small()
    rng = np.random.default_rng(99)
    orbs = wl.orbitals
    ctx = X.Exx.from_workload(wl, guess="extrap", precision=precision)
    zero = X.Exx.from_workload(wl, precision=precision)
    its, its0 = [], []
    for step in range(4):
        _say(f"[gpu] md step {step} ({precision})")
        wl_s = S.Workload(wl.name, wl.n_grid, wl.cell, orbs, wl.r_pair, wl.r_pe, wl.r_me)
        phi_np = S.orbitals_np(wl_s)
        phi = torch.from_numpy(phi_np).cuda()
        n = ctx.pairs(orbs.centers)
        zero.pairs(orbs.centers)
        E, D = ctx.step(phi)
        E0, D0 = zero.step(phi)
        Er, Dr, out = O.exx(wl.n_grid, wl.cell, wl.r_pair, wl.r_pe, wl.r_me, orbs.centers, phi_np)
        info = ctx.pair_info()
        assert np.all(info["converged"] == 1) and info["relres"].max() <= 1e-9
        assert abs(E - Er) <= 1e-8 * abs(Er), (step, E, Er)
        assert _gamma(Dr, D.cpu().numpy()) <= 1e-7
        assert abs(E0 - Er) <= 1e-8 * abs(Er)
        its.append(info["iters"].mean())
        its0.append(zero.pair_info()["iters"].mean())
        orbs = S.md_displace(orbs, wl.cell[0], rng)
    _say(f"[gpu] mean iterations with guess {its}, zero guess {its0}")
    # from the second step on, the extrapolated guess saves iterations
    assert all(g < z for g, z in zip(its[1:], its0[1:]))
