"""The multigrid preconditioner's algebra, on the CPU (no GPU): a dense model
of M = (2S - S A S) + (I - S A) P C R (I - A S) built exactly as the CG kernel
applies it (the fine operator A of a tiny PE sphere from the oracle; level-1
cells are 2x2x2 blocks of the PE bounding box, coarser levels halve down to
<= 6 cells per edge; R averages a cell's children in the domain and P injects,
R = P^T / 8; C is the V-cycle of 7-point Laplacians at spacing 2^l h with
Dirichlet zero outside the mask, one damped Jacobi step down and up, one on
the coarsest level, the correction handed to the fine level scaled by gamma).

PCG needs M symmetric positive definite.  The kernel's parameters (omega 0.8,
omega_c 1.0, gamma 0.5) give that; a coarse damping beyond 2 / lambda_max of
the coarse operator makes the coarse V-cycle indefinite, which the check
catches.  The preconditioner has no oracle of its own (the oracle runs the
paper's plain CG): on the GPU it is judged by the PCG that applies it."""
import numpy as np
import pytest

from oracle import oracle as O

H = 0.5


def _sphere():
    s = O.Subdomain((32, 32, 32), (32 * H,) * 3, 6 * H, 9 * H)
    n = s.n_pe
    A = np.zeros((n, n))
    for k in range(n):
        e = np.zeros(n)
        e[k] = 1.0
        A[:, k] = s.apply_A(e)
    return s, A, s.offsets()[:n]


def _levels(off):
    """Masks and parent maps of the coarse levels, as the host builds them."""
    lo = off.min(axis=0)
    dims = (off.max(axis=0) - lo) // 2 + 1
    cells = (off - lo) // 2                       # level-1 cell of each fine point
    levels = []
    idx = np.ravel_multi_index(cells.T, dims)
    mask = np.zeros(int(np.prod(dims)), bool)
    mask[idx] = True
    levels.append(dict(dims=dims, mask=mask, child_of_fine=idx))
    while max(dims) > 6 and len(levels) < 6:
        cd = (dims + 1) // 2
        grid = np.stack(np.unravel_index(np.arange(int(np.prod(dims))), dims), axis=1)
        parent = np.ravel_multi_index((grid // 2).T, cd)
        m2 = np.zeros(int(np.prod(cd)), bool)
        m2[parent[levels[-1]["mask"]]] = True
        levels[-1]["parent"] = parent
        levels.append(dict(dims=cd, mask=m2))
        dims = cd
    return levels


def _laplacian(lv, l):
    """7-point Laplacian of level l (spacing 2^(l+1) h) on the masked cells."""
    dims, mask = lv["dims"], lv["mask"]
    s = 1.0 / ((2 ** (l + 1)) * H) ** 2
    cells = np.nonzero(mask)[0]
    pos = {c: i for i, c in enumerate(cells)}
    L = np.zeros((len(cells), len(cells)))
    for i, c in enumerate(cells):
        x = np.array(np.unravel_index(c, dims))
        L[i, i] = 6.0 * s
        for a in range(3):
            for d in (-1, 1):
                y = x.copy()
                y[a] += d
                if 0 <= y[a] < dims[a]:
                    j = pos.get(int(np.ravel_multi_index(y, dims)))
                    if j is not None:
                        L[i, j] = -s
    return L, cells, 6.0 * s


def _model(A, off, omega=0.8, omega_c=1.0, gamma=0.5):
    lv = _levels(off)
    ops = [_laplacian(v, l) for l, v in enumerate(lv)]
    # restriction fine -> level 1 (masked cells) and between masked levels
    cells1 = ops[0][1]
    pos1 = {c: i for i, c in enumerate(cells1)}
    R0 = np.zeros((len(cells1), A.shape[0]))
    for q, c in enumerate(lv[0]["child_of_fine"]):
        R0[pos1[int(c)], q] = 0.125
    Rs = []
    for l in range(len(lv) - 1):
        ca, cb = ops[l][1], ops[l + 1][1]
        pb = {c: i for i, c in enumerate(cb)}
        R = np.zeros((len(cb), len(ca)))
        for i, c in enumerate(ca):
            R[pb[int(lv[l]["parent"][c])], i] = 0.125
        Rs.append(R)
    # V-cycle from the coarsest level up: C = S there, then
    # C_l = (2S - S L S) + (I - S L) P C_{l+1} R (I - L S)
    L, _, D = ops[-1]
    C = (omega_c / D) * np.eye(L.shape[0])
    for l in range(len(lv) - 2, -1, -1):
        L, _, D = ops[l]
        S = (omega_c / D) * np.eye(L.shape[0])
        I = np.eye(L.shape[0])
        R = Rs[l]
        C = 2 * S - S @ L @ S + (I - S @ L) @ (8.0 * R.T) @ C @ R @ (I - L @ S)
    C = gamma * C
    S = (omega / A[0, 0]) * np.eye(A.shape[0])
    I = np.eye(A.shape[0])
    M = 2 * S - S @ A @ S + (I - S @ A) @ (8.0 * R0.T) @ C @ R0 @ (I - A @ S)
    return M, C, len(lv)


@pytest.fixture(scope="module")
def sphere():
    return _sphere()


def test_kernel_parameters_give_an_spd_preconditioner(sphere):
    s, A, off = sphere
    assert np.allclose(np.diag(A), A[0, 0])            # the reduced operator's diagonal is constant
    M, C, nl = _model(A, off)
    assert nl >= 2
    assert np.max(np.abs(M - M.T)) <= 1e-12 * np.max(np.abs(M))
    assert np.linalg.eigvalsh(0.5 * (M + M.T)).min() > 0.0
    assert np.linalg.eigvalsh(0.5 * (C + C.T)).min() > 0.0


def test_pcg_with_the_model_needs_fewer_iterations(sphere):
    """Preconditioned CG with the model M, stopped like the kernel's (on the
    unpreconditioned recursive residual), against plain CG on the same
    system."""
    s, A, off = sphere
    M, _, _ = _model(A, off)
    b = np.random.default_rng(3).normal(size=A.shape[0])

    def pcg(Mop):
        x = np.zeros_like(b)
        r = b.copy()
        z = Mop(r)
        p = z.copy()
        rz = r @ z
        for it in range(1, 10000):
            Ap = A @ p
            a = rz / (p @ Ap)
            x += a * p
            r -= a * Ap
            if np.linalg.norm(r) <= 1e-10 * np.linalg.norm(b):
                return it, x
            z = Mop(r)
            rz_new = r @ z
            p = z + (rz_new / rz) * p
            rz = rz_new
        raise AssertionError("no convergence")

    it_plain, x0 = pcg(lambda r: r)
    it_mg, x1 = pcg(lambda r: M @ r)
    assert it_mg < 0.5 * it_plain, (it_mg, it_plain)
    assert np.max(np.abs(x1 - x0)) <= 1e-8 * np.max(np.abs(x0))


def test_too_much_coarse_damping_is_caught(sphere):
    """omega_c beyond 2 / lambda_max(D^-1 L) makes 2S - S L S indefinite:
    the coarse V-cycle loses definiteness (the check above can fail)."""
    s, A, off = sphere
    _, C, _ = _model(A, off, omega_c=2.2)
    assert np.linalg.eigvalsh(0.5 * (C + C.T)).min() < 0.0
