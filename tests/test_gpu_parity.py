"""GPU path (through the C ABI) against the FP64 CPU oracle, element by element.

Tolerances (FP64 path): E_xx to 1e-8 relative; per-pair energies to 1e-8;
D_xx per orbital to gamma^i <= 1e-7 (relative L1 norm, Eq. gammaxx_i).
Both sides stop CG at ||r|| <= 1e-10 ||b||, so their potentials differ by
at most the solver tolerance amplified by the conditioning; the energy is
stationary in v and agrees more tightly.
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

# The CG stops when its recursive residual reaches 1e-10 ||b|| (as the
# oracle's CG does); the true residual recomputed after the last step can sit
# above that by the drift between the two (2.8e-7 relative seen on water64).
RELRES_BAR = 1e-10 * (1 + 1e-4)


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def gamma(D_ref, D):
    """Eq. gammaxx_i per orbital."""
    num = np.abs(D_ref - D).reshape(D.shape[0], -1).sum(axis=1)
    den = np.abs(D_ref).reshape(D.shape[0], -1).sum(axis=1)
    return num / den


@pytest.fixture(scope="module")
def c1():
    wl = S.c1_small()
    phi = S.orbitals_np(wl)
    E, D, out = O.exx(wl.n_grid, wl.cell, wl.r_pair, wl.r_pe, wl.r_me, wl.orbitals.centers, phi)
    return wl, phi, E, D, out


@pytest.fixture(scope="module")
def c1_gpu(c1):
    wl, phi, *_ = c1
    _say("[gpu] small config, keep_intermediates")
    ctx = X.Exx.from_workload(wl, keep_intermediates=True)
    n = ctx.pairs(wl.orbitals.centers)
    phit = torch.from_numpy(phi).cuda()
    E, D = ctx.step(phit)
    torch.cuda.synchronize()
    return ctx, n, E, D.cpu().numpy(), ctx.pair_info(), phit


def test_c1_pair_list_and_origins(c1, c1_gpu):
    wl, phi, E, D, out = c1
    ctx, n, *_ , info, _ = c1_gpu
    assert n == len(out["e"]) == 60
    assert np.array_equal(info["i"], out["i"]) and np.array_equal(info["j"], out["j"])
    C = wl.orbitals.centers
    for p in range(n):
        gc = O.pair_origin(C[info["i"][p]], C[info["j"][p]], wl.cell, wl.n_grid)
        assert np.array_equal(gc, info["origin"][p])


def test_c1_energy(c1, c1_gpu):
    wl, phi, E, D, out = c1
    ctx, n, Eg, Dg, info, _ = c1_gpu
    assert np.all(info["converged"] == 1)
    assert np.all(info["relres"] <= 1e-9)
    assert abs(Eg - E) <= 1e-8 * abs(E), (Eg, E)
    rel = np.abs(info["e"] - out["e"]) / np.abs(out["e"])
    assert rel.max() <= 1e-8, rel.max()


def test_c1_potentials(c1, c1_gpu):
    wl, phi, E, D, out = c1
    ctx, n, Eg, Dg, info, _ = c1_gpu
    g = gamma(D, Dg)
    assert g.max() <= 1e-7, g.max()
    assert np.max(np.abs(Dg - D)) <= 1e-7 * np.max(np.abs(D))


@pytest.mark.parametrize("p", [0, 1, 7, 30, 59])
def test_c1_pair_intermediates(c1, c1_gpu, p):
    """Each step of one pair: density, moments, shell potential, rhs, solution."""
    wl, phi, E, D, out = c1
    ctx, n, Eg, Dg, info, _ = c1_gpu
    i, j = int(info["i"][p]), int(info["j"][p])
    cls = 0 if i == j else 1
    sub = O.Subdomain(wl.n_grid, wl.cell, wl.r_pe[cls], wl.r_me[cls])
    ref = sub.solve_pair(phi[i], phi[j], info["origin"][p])
    got = ctx.debug_pair(p, sub.n_pe, sub.n_shell, intermediates=True)
    assert np.array_equal(got["rho"], ref["rho"])                       # same product, same order
    # moments: real and complex harmonics span the same space per l
    for l in range(7):
        sl = slice(l * l, (l + 1) * (l + 1))
        pr, pg = np.sum(np.abs(ref["Q"][sl]) ** 2), np.sum(got["Q"][sl] ** 2)
        assert abs(pr - pg) <= 1e-12 * max(pr, 1e-30) + 1e-28, (l, pr, pg)
    assert np.max(np.abs(got["vsh"] - ref["vsh"])) <= 1e-12 * np.max(np.abs(ref["vsh"]))
    assert np.max(np.abs(got["b"] - ref["b"])) <= 1e-12 * np.max(np.abs(ref["b"]))
    assert np.max(np.abs(got["x"] - ref["x"])) <= 1e-7 * np.max(np.abs(ref["x"]))


def test_c1_bitwise_reproducible(c1, c1_gpu):
    wl, phi, *_ = c1
    ctx, n, Eg, Dg, info, phit = c1_gpu
    E2, D2 = ctx.step(phit)
    assert E2 == Eg
    assert np.array_equal(D2.cpu().numpy(), Dg)


def test_c1_nonconvergence_flag(c1):
    wl, phi, *_ = c1
    ctx = X.Exx.from_workload(wl, cg_max_iter=3)
    ctx.pairs(wl.orbitals.centers)
    phit = torch.from_numpy(phi).cuda()
    ctx.solve(phit)
    with pytest.raises(X.ExxError) as ei:
        ctx.energy_potential(torch.empty_like(phit))
    assert ei.value.status == X.EXX_ENOCONV
    info = ctx.pair_info()
    assert np.all(info["iters"] == 3) and np.all(info["converged"] == 0)


def test_call_order(c1):
    wl, phi, *_ = c1
    ctx = X.Exx.from_workload(wl)
    phit = torch.from_numpy(phi).cuda()
    with pytest.raises(X.ExxError) as ei:
        ctx._check(X.load().exx_solve(ctx._h, X._ptr(phit), None))
    assert ei.value.status == X.EXX_ESTATE
    ctx.pairs(wl.orbitals.centers)
    e = __import__("ctypes").c_double()
    st = X.load().exx_energy_potential(ctx._h, __import__("ctypes").byref(e), X._ptr(phit), None)
    assert st == X.EXX_ESTATE


def test_c1_waves_match_single_launch(c1, c1_gpu):
    """Pairs split into several launch waves give bitwise the same results."""
    wl, phi, *_ = c1
    ctx0, n, Eg, Dg, info, phit = c1_gpu
    ctx = X.Exx.from_workload(wl, wave_pairs=7)
    ctx.pairs(wl.orbitals.centers)
    E2, D2 = ctx.step(phit)
    assert ctx.stats()["n_waves"] == 9
    assert E2 == Eg and np.array_equal(D2.cpu().numpy(), Dg)


@pytest.mark.parametrize("block,cols", [(256, -1), (256, 4), (512, 4), (512, 6)])
def test_c1_cg_kernel_variants(c1, block, cols):
    """Every CG kernel variant (flat, and z-march tilings with 1-2 bands)."""
    wl, phi, E, D, out = c1
    _say(f"[gpu] variant block={block} cols={cols}")
    ctx = X.Exx.from_workload(wl, block_threads=block, cg_cols=cols)
    ctx.pairs(wl.orbitals.centers)
    Eg, Dg = ctx.step(torch.from_numpy(phi).cuda())
    st = ctx.stats()
    assert st["cg_cols"] == max(cols, 0)
    info = ctx.pair_info()
    assert np.all(info["converged"] == 1) and np.all(info["relres"] <= 1e-9)
    assert abs(Eg - E) <= 1e-8 * abs(E), (Eg, E)
    assert gamma(D, Dg.cpu().numpy()).max() <= 1e-7
    assert np.all(np.abs(info["iters"] - out["iters"]) <= 2)


def test_c1_fp32_refinement(c1):
    """FP32 inner CG with FP64 refinement reaches the FP64 residual target."""
    wl, phi, E, D, out = c1
    _say("[gpu] fp32 refinement")
    ctx = X.Exx.from_workload(wl, precision="fp32_refine", inner_rtol=1e-4)
    ctx.pairs(wl.orbitals.centers)
    Eg, Dg = ctx.step(torch.from_numpy(phi).cuda())
    info = ctx.pair_info()
    st = ctx.stats()
    assert np.all(info["converged"] == 1)
    assert info["relres"].max() <= RELRES_BAR
    assert st["outer_total"] >= 3 * len(info["e"])          # at least three FP64 residual passes per pair
    assert abs(Eg - E) <= 1e-8 * abs(E), (Eg, E)
    assert gamma(D, Dg.cpu().numpy()).max() <= 1e-7


def test_c1_fp32_orbitals(c1):
    """Orbitals and D stored in FP32; arithmetic FP64.  The oracle sees the same
    FP32-rounded orbitals; D differs by its final rounding to FP32."""
    wl, phi, *_ = c1
    phi32 = phi.astype(np.float32)
    E, D, _ = O.exx(wl.n_grid, wl.cell, wl.r_pair, wl.r_pe, wl.r_me, wl.orbitals.centers, phi32.astype(np.float64))
    ctx = X.Exx.from_workload(wl, orbital_dtype="f32")
    ctx.pairs(wl.orbitals.centers)
    Eg, Dg = ctx.step(torch.from_numpy(phi32).cuda())
    assert Dg.dtype == torch.float32
    assert abs(Eg - E) <= 1e-8 * abs(E)
    assert gamma(D, Dg.cpu().numpy().astype(np.float64)).max() <= 1e-6


def test_uneven_subdomain_classes_in_one_launch():
    """Self and non-self pairs with different (R_PE, R_ME) (the paper's two
    proto-subdomain classes) solved in one persistent launch."""
    wl = S.c1_small()
    wl.r_pe = (4.0 * S.ANG, 3.3 * S.ANG)
    wl.r_me = (5.0 * S.ANG, 4.3 * S.ANG)
    phi = S.orbitals_np(wl)
    E, D, out = O.exx(wl.n_grid, wl.cell, wl.r_pair, wl.r_pe, wl.r_me, wl.orbitals.centers, phi)
    for prec in ("fp64", "fp32_refine"):
        _say(f"[gpu] uneven classes {prec}")
        ctx = X.Exx.from_workload(wl, precision=prec)
        ctx.pairs(wl.orbitals.centers)
        Eg, Dg = ctx.step(torch.from_numpy(phi).cuda())
        st = ctx.stats()
        assert st["n_pe"][0] != st["n_pe"][1] and st["n_waves"] == 1
        info = ctx.pair_info()
        assert np.all(info["converged"] == 1)
        assert abs(Eg - E) <= 1e-8 * abs(E), (prec, Eg, E)
        assert np.max(np.abs(info["e"] - out["e"]) / np.abs(out["e"])) <= 1e-8
        assert gamma(D, Dg.cpu().numpy()).max() <= 1e-7


def test_autotuner_times_every_fitting_variant(c1):
    """exx_setup times each z-march variant that fits (all three on the small
    spheres) and keeps one of them; the solve still matches the oracle.  With
    autotune off the occupancy rule decides and no variant is timed."""
    wl, phi, E, D, out = c1
    _say("[gpu] autotune")
    ctx = X.Exx.from_workload(wl, autotune=True)
    ctx.pairs(wl.orbitals.centers)
    Eg, Dg = ctx.step(torch.from_numpy(phi).cuda())
    st = ctx.stats()
    assert st["tuned"] == 3 and st["tune_ms"] > 0.0
    assert (st["solve_block"], st["cg_cols"]) in [(256, 4), (512, 4), (512, 6)]
    assert abs(Eg - E) <= 1e-8 * abs(E)
    assert gamma(D, Dg.cpu().numpy()).max() <= 1e-7
    off = X.Exx.from_workload(wl, autotune=False)
    off.pairs(wl.orbitals.centers)
    off.step(torch.from_numpy(phi).cuda())
    assert off.stats()["tuned"] == 0


def test_graph_mode_replays_bitwise(c1, c1_gpu):
    """Graph mode: the first solve captures, later solves replay; each replay
    (with eager device work and synchronizations between) gives bitwise the
    eager result.  New pairs re-capture."""
    wl, phi, E, D, out = c1
    ctx0, n, Eg, Dg, info, phit = c1_gpu
    _say("[gpu] graph mode")
    ctx = X.Exx.from_workload(wl, graph=True)
    ctx.pairs(wl.orbitals.centers)
    for k in range(3):
        E2, D2 = ctx.step(phit)
        junk = torch.randn(1 << 20, device="cuda").sum().item()   # eager work between replays
        assert np.isfinite(junk)
        assert E2 == Eg and np.array_equal(D2.cpu().numpy(), Dg), k
    st = ctx.stats()
    assert st["graph_builds"] == 1 and st["graph_launches"] == 3
    assert st["prep_ms"] == -1.0 and st["solve_ms"] > 0.0
    ctx.pairs(wl.orbitals.centers)
    E3, _ = ctx.step(phit)
    assert E3 == Eg and ctx.stats()["graph_builds"] == 2
