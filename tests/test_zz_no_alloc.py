"""exx_solve_static, the allocation-free solve for callers that cannot
allocate (graph capture, serving loops): through the C ABI, against exx_solve
on the same context, two calls in a row, the second on a smaller pair list.

Both paths run the same kernels on the same pairs; only the CG work vectors
(the library's fixed device array instead of the context's buffers) and the
number of CG work-groups differ, and each pair's CG does not depend on which
work-group or slot runs it.  So E_xx and D must agree bit for bit.
"""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_1911_10630_amd import exx as X  # noqa: E402
from paper_1911_10630_amd import synth as S  # noqa: E402


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


MODES = [dict(), dict(precond="mg"), dict(precision="fp32_refine"), dict(precond="mg", precision="fp32_refine")]
IDS = ["plain", "mg", "fp32", "mg-fp32"]


@pytest.mark.parametrize("kw", MODES, ids=IDS)
def test_static_solve_matches_exx_solve_twice(kw):
    wl = S.c1_small()
    phi = S.orbitals_np(wl)
    ctx = X.Exx.from_workload(wl, **kw)
    C = wl.orbitals.centers
    for keep in (np.arange(16), np.array([0, 2, 3, 5, 9, 11])):        # second call: a smaller input
        _say(f"[gpu] static solve {kw}, {len(keep)} orbitals")
        ctx.pairs(C[keep])
        phit = torch.from_numpy(np.ascontiguousarray(phi[keep])).cuda()
        E_ref, D_ref = ctx.step(phit)
        info_ref = ctx.pair_info()
        D = torch.empty_like(phit)
        ctx.solve_static(phit)
        E = ctx.energy_potential(D)
        info = ctx.pair_info()
        assert E == E_ref, (E, E_ref)
        assert torch.equal(D, D_ref)
        assert np.array_equal(info["e"], info_ref["e"]) and np.array_equal(info["iters"], info_ref["iters"])
        assert np.all(info["converged"] == 1)
    ctx.close()


def test_static_solve_in_waves_and_repeated():
    """Waves (D summed wave by wave) and a repeat on the same array: still the
    same bits as exx_solve."""
    wl = S.c1_small()
    phit = torch.from_numpy(S.orbitals_np(wl)).cuda()
    ctx = X.Exx.from_workload(wl, wave_pairs=13)
    ctx.pairs(wl.orbitals.centers)
    E_ref, D_ref = ctx.step(phit)
    assert ctx.stats()["n_waves"] > 1
    for _ in range(2):
        D = torch.empty_like(phit)
        ctx.solve_static(phit)
        assert ctx.energy_potential(D) == E_ref
        assert torch.equal(D, D_ref)
    ctx.close()


def test_static_solve_refuses_the_allocating_guesses():
    wl = S.c1_small()
    phit = torch.from_numpy(S.orbitals_np(wl)).cuda()
    ctx = X.Exx.from_workload(wl, guess="previous")
    ctx.pairs(wl.orbitals.centers)
    with pytest.raises(X.ExxError) as ei:
        ctx.solve_static(phit)
    assert ei.value.status == X.EXX_EINVAL and "zero initial guess" in str(ei.value)
    ctx.close()
