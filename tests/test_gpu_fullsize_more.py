"""Full-size parity for the remaining workloads, in the launch configuration
the benchmark times, on sampled outputs the oracle computes one by one:

* water64 with FP32 CG and FP64 reliable updates (9,966 pairs);
* water128 (512 orbitals, 160^3, 17k pairs) over two MD steps with the
  previous-step guess: the second step starts every pair from the first
  step's potential and must still meet the oracle.

Each module-level fixture releases its context before the next one runs.
"""
import concurrent.futures as cf
import gc
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

# The CG stops when its recursive residual reaches 1e-10 ||b|| (as the
# oracle's CG does); the true residual recomputed after the last step can sit
# above that by the drift between the two (2.8e-7 relative seen on water64).
RELRES_BAR = 1e-10 * (1 + 1e-4)


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _check_pairs(wl, ctx, info, pick, phis, tol_x=1e-7):
    subs = [O.Subdomain(wl.n_grid, wl.cell, wl.r_pe[c], wl.r_me[c]) for c in (0, 1)]

    def ref(p):
        i, j = int(info["i"][p]), int(info["j"][p])
        return subs[0 if i == j else 1].solve_pair(phis[i], phis[j], info["origin"][p])

    _say(f"[gpu] oracle on sampled pairs {pick}")
    with cf.ThreadPoolExecutor(len(pick)) as ex:
        refs = list(ex.map(ref, pick))
    for p, r in zip(pick, refs):
        sub = subs[0 if info["i"][p] == info["j"][p] else 1]
        got = ctx.debug_pair(p, sub.n_pe, sub.n_shell)
        assert abs(info["e"][p] - r["e"]) <= 1e-8 * abs(r["e"]), (p, info["e"][p], r["e"])
        assert np.max(np.abs(got["x"] - r["x"])) <= tol_x * np.max(np.abs(r["x"])), p


def test_c3_mixed_precision_full_size():
    wl = S.c3_water64_mixed()
    _say("[gpu] 64-water workload, FP32 CG with FP64 reliable updates")
    phi = S.orbitals_torch(wl, device="cuda:0")
    ctx = X.Exx.from_workload(wl)
    n = ctx.pairs(wl.orbitals.centers)
    E, D = ctx.step(phi)
    info = ctx.pair_info()
    st = ctx.stats()
    assert n == 9966 and st["n_waves"] == 1
    assert np.all(info["converged"] == 1) and info["relres"].max() <= RELRES_BAR
    assert st["outer_total"] >= 3 * n
    w = np.where(info["i"] == info["j"], 1.0, 2.0)
    assert abs(E + np.sum(w * info["e"])) <= 1e-12 * abs(E)
    other = np.nonzero(info["i"] != info["j"])[0]
    pick = [int(np.nonzero(info["i"] == info["j"])[0][3]), int(other[100]),
            int(other[np.argmax(info["iters"][other])])]
    orbs = sorted({int(info["i"][p]) for p in pick} | {int(info["j"][p]) for p in pick})
    _check_pairs(wl, ctx, info, pick, dict(zip(orbs, S.orbitals_np(wl, orbs))))
    ctx.close()
    del phi, D
    gc.collect()


def test_c4_md_previous_guess_full_size():
    wl = S.c4_water128()
    _say("[gpu] 128-water workload, two MD steps with the previous-step guess")
    rng = np.random.default_rng(7)
    ctx = X.Exx.from_workload(wl, guess="previous")
    phi = torch.empty((wl.orbitals.n,) + tuple(reversed(wl.n_grid)), dtype=torch.float64, device="cuda:0")
    dxx = torch.empty_like(phi)
    orbs = wl.orbitals
    iters = []
    for step in range(2):
        wl_s = S.Workload(wl.name, wl.n_grid, wl.cell, orbs, wl.r_pair, wl.r_pe, wl.r_me)
        n = ctx.pairs(orbs.centers)
        S.orbitals_torch(wl_s, device="cuda:0", out=phi)
        E, _ = ctx.step(phi, dxx)
        info = ctx.pair_info()
        iters.append(info["iters"].mean())
        _say(f"[gpu] step {step}: {n} pairs, mean iterations {iters[-1]:.1f}, E {E}")
        assert np.all(info["converged"] == 1) and info["relres"].max() <= 1e-9
        w = np.where(info["i"] == info["j"], 1.0, 2.0)
        assert abs(E + np.sum(w * info["e"])) <= 1e-12 * abs(E)
        if step == 1:
            assert ctx.stats()["guess_pairs"] > 0.99 * n
            other = np.nonzero(info["i"] != info["j"])[0]
            pick = [int(np.nonzero(info["i"] == info["j"])[0][7]), int(other[5000])]
            used = sorted({int(info["i"][p]) for p in pick} | {int(info["j"][p]) for p in pick})
            _check_pairs(wl_s, ctx, info, pick, dict(zip(used, S.orbitals_np(wl_s, used))))
        orbs = S.md_displace(orbs, wl.cell[0], rng)
    assert iters[1] < iters[0]
    ctx.close()
