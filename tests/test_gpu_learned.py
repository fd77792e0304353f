"""Learned initial guess on the GPU, through the C ABI.

* The model's MFMA convolution kernels (forward, input-gradient and
  weight-gradient) against torch's CPU conv3d in float64 on the same
  bf16-rounded operands.  Bound: a sum of K products in FP32, in any order,
  is within (K + 1) 2^-24 sum|terms| of the exact sum, and the products of
  two bf16 values are exact in FP32.
* CG from the learned guess converges to the same tolerance as from zero:
  E_xx against the FP64 oracle to 1e-8 relative, D to gamma <= 1e-7.  The
  guess itself has no oracle (parity unpinned); it is judged by the CG.
* A corrupt model (non-finite weights) yields a zero guess, never NaNs.
"""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import torch.nn.functional as F  # noqa: E402

from oracle import oracle as O  # noqa: E402
from paper_1911_10630_amd import exx as X  # noqa: E402
from paper_1911_10630_amd import synth as S  # noqa: E402

# The CG stops when its recursive residual reaches 1e-10 ||b|| (as the
# oracle's CG does); the true residual recomputed after the last step can sit
# above that by the drift between the two (2.8e-7 relative seen on water64).
RELRES_BAR = 1e-10 * (1 + 1e-4)

LAYERS = [(16, 16), (16, 16), (16, 32), (32, 32), (32, 64), (64, 64), (64, 64), (64, 64), (128, 64), (96, 32),
          (48, 16), (16, 16)]


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def bf16_round(a):
    """Round float32 to the nearest bf16 (ties to even), returned as float32 and raw uint16."""
    u = np.ascontiguousarray(a, dtype=np.float32).view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16).astype(np.uint16)
    return (r.astype(np.uint32) << 16).view(np.float32), r


def layer_weights(blob, layer):
    """FP32 weights [27][Cout][Cin] of one layer from a model blob."""
    off = 16
    for l, (ci, co) in enumerate(LAYERS):
        n = 27 * ci * co
        if l == layer:
            return np.frombuffer(blob, dtype=np.float32, count=n, offset=off).reshape(27, co, ci)
        off += 4 * n
    raise IndexError(layer)


def torch_weight(W):
    """[27][Cout][Cin] (tap = 9 kz + 3 ky + kx) -> torch [Cout][Cin][kz][ky][kx]."""
    co, ci = W.shape[1], W.shape[2]
    return torch.from_numpy(W.reshape(3, 3, 3, co, ci).transpose(3, 4, 0, 1, 2).copy()).double()


def to_ncdhw(a, n, d, c):
    return torch.from_numpy(a.reshape(n, d, d, d, c).transpose(0, 4, 1, 2, 3).copy()).double()


@pytest.fixture(scope="module")
def ctx():
    wl = S.c1_small()
    c = X.Exx.from_workload(wl)
    c.model_init(2, seed=7)
    return c


@pytest.mark.parametrize("layer,n,d", [(0, 3, 6), (2, 2, 5), (5, 1, 7), (8, 2, 4), (9, 1, 6), (11, 2, 8)])
@pytest.mark.parametrize("transposed", [False, True])
def test_conv_matches_torch(ctx, layer, n, d, transposed):
    _say(f"[gpu] conv layer={layer} n={n} d={d} transposed={transposed}")
    blob = ctx.model_save()
    W = layer_weights(blob, layer)
    Wb, _ = bf16_round(W)
    ci, co = LAYERS[layer]
    cin, cout = (co, ci) if transposed else (ci, co)
    rng = np.random.default_rng(layer * 10 + transposed)
    xf, xr = bf16_round(rng.standard_normal((n * d ** 3, cin)).astype(np.float32))
    xg = torch.from_numpy(xr.view(np.int16)).cuda()
    yg = torch.empty(n * d ** 3 * cout, dtype=torch.float32, device="cuda")
    ctx.model_conv(layer, xg, yg, n, d, transposed=transposed)
    torch.cuda.synchronize()
    y = yg.cpu().numpy().reshape(n, d, d, d, cout)
    xt, wt = to_ncdhw(xf, n, d, cin), torch_weight(Wb)
    if transposed:
        ref = F.conv_transpose3d(xt, wt, padding=1)
        mag = F.conv_transpose3d(xt.abs(), wt.abs(), padding=1)
    else:
        ref = F.conv3d(xt, wt, padding=1)
        mag = F.conv3d(xt.abs(), wt.abs(), padding=1)
    ref = ref.numpy().transpose(0, 2, 3, 4, 1)
    mag = mag.numpy().transpose(0, 2, 3, 4, 1)
    K = 27 * cin
    err = np.abs(y - ref)
    assert np.all(err <= (K + 1) * 2.0 ** -24 * mag + 1e-30), err.max()


@pytest.mark.parametrize("layer,n,d", [(0, 3, 6), (3, 2, 5), (8, 2, 4), (10, 1, 8)])
def test_wgrad_matches_torch(ctx, layer, n, d):
    _say(f"[gpu] wgrad layer={layer} n={n} d={d}")
    ci, co = LAYERS[layer]
    rng = np.random.default_rng(100 + layer)
    xf, xr = bf16_round(rng.standard_normal((n * d ** 3, ci)).astype(np.float32))
    gf, gr = bf16_round(rng.standard_normal((n * d ** 3, co)).astype(np.float32))
    xg = torch.from_numpy(xr.view(np.int16)).cuda()
    gg = torch.from_numpy(gr.view(np.int16)).cuda()
    dw = torch.empty(27 * co * ci, dtype=torch.float32, device="cuda")
    ctx.model_wgrad(layer, xg, gg, dw, n, d)
    torch.cuda.synchronize()
    got = dw.cpu().numpy().reshape(3, 3, 3, co, ci).transpose(3, 4, 0, 1, 2)
    xt, gt = to_ncdhw(xf, n, d, ci), to_ncdhw(gf, n, d, co)
    ref = torch.nn.grad.conv3d_weight(xt, (co, ci, 3, 3, 3), gt, padding=1).numpy()
    mag = torch.nn.grad.conv3d_weight(xt.abs(), (co, ci, 3, 3, 3), gt.abs(), padding=1).numpy()
    K = n * d ** 3
    err = np.abs(got - ref)
    assert np.all(err <= (K + 8) * 2.0 ** -24 * mag + 1e-30), err.max()


def test_model_blob_round_trip(ctx):
    blob = ctx.model_save()
    wl = S.c1_small()
    other = X.Exx.from_workload(wl)
    other.load_model(blob)
    assert other.model_save() == blob
    assert other.model_edge() == ctx.model_edge() == 24
    with pytest.raises(X.ExxError) as ei:
        other.load_model(blob[:-4])
    assert ei.value.status == X.EXX_EINVAL


@pytest.fixture(scope="module")
def c1_ref():
    wl = S.c1_small()
    phi = S.orbitals_np(wl)
    E, D, out = O.exx(wl.n_grid, wl.cell, wl.r_pair, wl.r_pe, wl.r_me, wl.orbitals.centers, phi)
    return wl, phi, E, D, out


def _gamma(D_ref, D):
    num = np.abs(D_ref - D).reshape(D.shape[0], -1).sum(axis=1)
    return num / np.abs(D_ref).reshape(D.shape[0], -1).sum(axis=1)


@pytest.fixture(scope="module")
def trained(c1_ref):
    """A model trained on the small configuration with other orbital seeds."""
    wl, *_ = c1_ref
    losses = []
    ctx = X.Exx.from_workload(wl)
    ctx.model_init(2, seed=3)
    for seed in (11, 12, 13):
        w = S.c1_small(seed=seed)
        phi = torch.from_numpy(S.orbitals_np(w)).cuda()
        ctx.pairs(w.orbitals.centers)
        ctx.step(phi)
        for _ in range(4):
            losses.append(ctx.model_train(epochs=5, batch=4, lr=2e-3, seed=seed))
        _say(f"[gpu] trained on seed {seed}: loss {losses[-1]:.4g}")
    return ctx.model_save(), losses


def test_training_lowers_the_loss(trained):
    _, losses = trained
    assert all(np.isfinite(losses))
    assert losses[-1] < 0.5 * losses[0], losses


def _solve(wl, phi, guess, blob=None, precision="fp64"):
    ctx = X.Exx.from_workload(wl, guess=guess, precision=precision)
    if blob is not None:
        ctx.load_model(blob)
    ctx.pairs(wl.orbitals.centers)
    E, D = ctx.step(torch.from_numpy(phi).cuda())
    return ctx, E, D.cpu().numpy()


def test_model_generalizes_to_a_held_out_configuration(c1_ref, trained):
    """On the evaluation configuration (never trained on), the trained model's
    coarse potential error is well below that of a zero output."""
    wl, phi, *_ = c1_ref
    blob, _ = trained
    ctx = X.Exx.from_workload(wl)
    ctx.pairs(wl.orbitals.centers)
    ctx.step(torch.from_numpy(phi).cuda())
    ctx.load_model(blob)
    err = ctx.model_loss()
    zero = bytearray(blob)
    np.frombuffer(zero, dtype=np.float32, offset=16)[:] = 0.0
    ctx.load_model(bytes(zero))
    power = ctx.model_loss()
    _say(f"  held-out loss {err:.4g}, zero-output loss {power:.4g}")
    assert power > 0 and err < 0.1 * power, (err, power)


@pytest.mark.parametrize("precision", ["fp64", "fp32_refine"])
def test_learned_guess_same_result(c1_ref, trained, precision):
    """CG from the learned guess reaches the oracle's E and D.  Iteration
    counts are reported, not asserted: on this small grid the coarse guess
    is too coarse to shorten the solve (the gain is measured on the water
    workloads by bench.py)."""
    wl, phi, E, D, out = c1_ref
    blob, _ = trained
    _say(f"[gpu] learned guess {precision}")
    c0, E0, D0 = _solve(wl, phi, "zero", precision=precision)
    cl, El, Dl = _solve(wl, phi, "learned", blob, precision=precision)
    i0, il = c0.pair_info(), cl.pair_info()
    st = cl.stats()
    assert st["guess_pairs"] == len(il["e"]) and st["guess_ms"] >= 0.0
    assert np.all(il["converged"] == 1) and il["relres"].max() <= RELRES_BAR
    assert abs(El - E) <= 1e-8 * abs(E), (El, E)
    assert _gamma(D, Dl).max() <= 1e-7
    _say(f"  iterations zero {i0['iters'].mean():.1f} learned {il['iters'].mean():.1f}")


def test_learned_guess_is_deterministic(c1_ref, trained):
    wl, phi, *_ = c1_ref
    blob, _ = trained
    ctx = X.Exx.from_workload(wl, guess="learned")
    ctx.load_model(blob)
    ctx.pairs(wl.orbitals.centers)
    phit = torch.from_numpy(phi).cuda()
    E1, D1 = ctx.step(phit)
    it1 = ctx.pair_info()["iters"]
    E2, D2 = ctx.step(phit)
    assert E1 == E2 and torch.equal(D1, D2)
    assert np.array_equal(it1, ctx.pair_info()["iters"])


@pytest.mark.parametrize("coarsen", [4, 8])
def test_untrained_and_corrupt_models_still_converge(c1_ref, coarsen):
    """A random model gives a poor but finite guess; non-finite weights give
    non-finite net outputs, which become a zero guess.  Both reach the same
    result (at 8 grid points per coarse cell the small workload's cube is 8
    cells wide and the net's coarsest level a single cell)."""
    wl, phi, E, D, out = c1_ref
    ctx = X.Exx.from_workload(wl)
    ctx.model_init(coarsen, seed=1)
    good = ctx.model_save()
    bad = bytearray(good)
    w = np.frombuffer(bad, dtype=np.float32, offset=16)
    w[:] = np.float32(np.inf)
    for name, blob in (("random", good), ("corrupt", bytes(bad))):
        _say(f"[gpu] {name} model")
        cl, El, Dl = _solve(wl, phi, "learned", blob)
        info = cl.pair_info()
        assert np.all(info["converged"] == 1), name
        assert abs(El - E) <= 1e-8 * abs(E), (name, El, E)
        assert _gamma(D, Dl).max() <= 1e-7, name


def test_learned_guess_needs_a_model(c1_ref):
    wl, phi, *_ = c1_ref
    ctx = X.Exx.from_workload(wl, guess="learned")
    ctx.pairs(wl.orbitals.centers)
    with pytest.raises(X.ExxError) as ei:
        ctx.solve(torch.from_numpy(phi).cuda())
    assert ei.value.status == X.EXX_ESTATE


def test_training_in_waves_uses_the_last_wave(c1_ref):
    """After a solve in waves only the last wave's right-hand sides are
    resident: training runs on those (60 pairs in waves of 7 leave 4), a
    batch larger than that is refused, and the loss it reports equals the
    evaluation over the same pairs."""
    wl, phi, *_ = c1_ref
    ctx = X.Exx.from_workload(wl, wave_pairs=7)
    ctx.model_init(2, seed=3)
    ctx.pairs(wl.orbitals.centers)
    ctx.step(torch.from_numpy(phi).cuda())
    assert ctx.stats()["n_waves"] == 9
    with pytest.raises(X.ExxError) as ei:
        ctx.model_train(epochs=1, batch=5)
    assert ei.value.status == X.EXX_EINVAL
    before = ctx.model_loss(batch=4)
    for ep in range(20):
        loss = ctx.model_train(epochs=1, batch=4, lr=1e-3, seed=ep)
    assert np.isfinite(before) and np.isfinite(loss)
    assert ctx.model_loss(batch=4) < before


def test_learned_guess_in_graph_mode(c1_ref, trained):
    """The learned guess (net inference kernels) captured in the solve graph
    replays to the eager result bitwise."""
    wl, phi, *_ = c1_ref
    blob, _ = trained
    eager = X.Exx.from_workload(wl, guess="learned")
    eager.load_model(blob)
    eager.pairs(wl.orbitals.centers)
    phit = torch.from_numpy(phi).cuda()
    E0, D0 = eager.step(phit)
    g = X.Exx.from_workload(wl, guess="learned", graph=True)
    g.load_model(blob)
    g.pairs(wl.orbitals.centers)
    for k in range(3):
        E1, D1 = g.step(phit)
        assert E1 == E0 and torch.equal(D1, D0), k
    assert g.stats()["graph_launches"] == 3 and g.stats()["graph_builds"] == 1
